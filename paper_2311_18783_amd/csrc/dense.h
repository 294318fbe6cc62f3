// Batched dense factorisation / solve plans (see dense.hip).
#pragma once

#include "internal.h"

namespace geneo {

struct MatDesc {
  int64_t off;       // element offset of the matrix (column-major, ld)
  int64_t inv_off;   // element offset of its diagonal-block inverses: nblk blocks of inv(L_II), then nblk of inv(U_II)
  int64_t diag_off;  // offset into the original-diagonal array, or -1
  int64_t voff;      // offset of its segment in a batch vector
  int32_t ld;        // = n_pad, multiple of NB
  int32_t nblk;      // n_pad / NB
  int32_t flag_off;  // first block-done flag of this matrix
  int32_t n;         // true size
};

struct SyrkLaunch {
  int64_t pre_off, tiles;   // prefix array offset (nmat+1 entries), total tiles
  int kcol0, kb, b0, ncols; // panel group columns, first trailing block, column limit (0 = all)
};

// Schedule of a batched factorisation: tile mode of the trailing updates
// (0: 64x64 per wave, operands from L2, 4 waves; 1: the same with 8 waves;
// 2: operands staged through LDS), panels per trailing-update group, and the
// diagonal-block kernel (1: recursive, in FP64 in LDS for both precisions;
// 0: register kernel in the factor's precision).
struct FactorConfig {
  int mode = 0;
  int group = 8;
  int rec_potrf = 1;
};
// The schedule for a batch: the autotuner's entry for (precision, largest
// block count, batch-size class floor(log2 nmat)) if it has one, else the
// nearest tuned block count of that precision and class, else the defaults.
FactorConfig tuned_factor_config(int precision, int max_blk, int nmat);
void set_tuned_factor_config(int precision, int max_blk, int nmat, const FactorConfig& c, double ms);
std::string tune_db_text();
void tune_db_parse(const std::string& text);

struct FactorPlan {
  int nmat = 0, max_blk = 0;
  std::vector<MatDesc> h_desc;
  std::vector<int> cnt;              // matrices active at each panel step
  std::vector<int64_t> trsm_tiles, syrk_tiles, pre_off;
  int64_t n_items = 0;               // triangular-solve work items (blocks)
  int64_t mirror_tiles = 0;          // strictly-lower 128x128 blocks
  int group = 8;                     // panels per trailing update
  FactorConfig cfg;                  // schedule (the autotuner's table, or the defaults)
  // solve form (off-diagonal blocks premultiplied by their row's diagonal
  // inverse, shorter dependency chain; the coarse factor) or plain form
  // (x_I = inv(D_II) (b_I - sum L(I,J) x_J); the batched local factors,
  // whose solves are bandwidth bound)
  bool solve_form = true;
  std::vector<SyrkLaunch> syrk;      // trailing-update launches in execution order
  DevBuf<int64_t> d_syrk_prefix;
  DevBuf<int64_t> d_mirror_prefix;
  DevBuf<MatDesc> d_desc;
  DevBuf<int32_t> d_order;
  DevBuf<int64_t> d_prefix;
  DevBuf<int32_t> d_items_fwd, d_items_bwd;
  DevBuf<double> d_y;                // single-right-hand-side solves: intermediate vector
  mutable DevBuf<double> d_ym;       // many-right-hand-side solves: intermediate block (on first use)
  // precision: the factor's type (GENEO_FP64 or GENEO_FP32_REFINE1), selects the schedule
  void build(const std::vector<MatDesc>& descs, hipStream_t st, int precision = GENEO_FP64);
  // The same plan with only what factor(..., for_solves = false) reads on the
  // device (descriptors, order, per-step and trailing-update prefixes), placed
  // in caller-owned device memory [mem, mem + bytes) instead of allocated;
  // throws GENEO_EINVAL if it does not fit.  Returns the bytes used (multiple
  // of 256).  Host copies stay in the plan until it is destroyed.
  size_t build_in(const std::vector<MatDesc>& descs, void* mem, size_t bytes, hipStream_t st,
                  int precision = GENEO_FP64);
  // host side of build(): ordering, prefixes, launches, solve items (with
  // the schedule `force` instead of the table's, if given)
  void plan_host(const std::vector<MatDesc>& descs, int precision = GENEO_FP64,
                 const FactorConfig* force = nullptr);
  std::vector<int32_t> h_order, h_items_fwd, h_items_bwd;
  std::vector<int64_t> h_prefix, h_syrk_prefix, h_mirror_prefix;

  // Block-sparse single matrix: only the tiles of the factor's fill pattern
  // are touched (explicit tile lists), the solves follow per-row dependency
  // lists.  fill[I * nblk + J] (I >= J) must contain the pattern of L,
  // i.e. be closed under the symbolic elimination.
  bool sparse = false;
  std::vector<int64_t> trsm_off;         // [max_blk + 1] into d_trsm_rows
  DevBuf<int32_t> d_trsm_rows;           // row blocks of each panel step
  std::vector<int64_t> syrk_off;         // per entry of `syrk`: offset (in pairs) into d_syrk_pairs
  DevBuf<int32_t> d_syrk_pairs;          // (ti, tj) of every trailing-update tile
  int64_t n_lower = 0;                   // strictly lower tiles in the pattern
  DevBuf<int32_t> d_lower_pairs;
  DevBuf<int32_t> d_dep_fwd_ptr, d_dep_fwd, d_dep_bwd_ptr, d_dep_bwd;
  // Split rows of the single-RHS solves (per direction, 0 forward, 1
  // backward): a row with many dependencies hands the leading chunks of its
  // list to helper work items that post partial sums Q(I, J) x_J, and keeps
  // the last ones itself.  Work items (m, I) in ticket order, a helper h
  // encoded as (-1 - h, I) right before its row.
  int64_t n_sitems[2] = {0, 0};
  int32_t n_help[2] = {0, 0};
  DevBuf<int32_t> d_sitems[2];
  DevBuf<int32_t> d_help_rng[2];     // helper h: dependency index range [lo, hi) of its row
  DevBuf<int32_t> d_row_lo[2];       // row I: first dependency index it handles itself
  DevBuf<int32_t> d_row_help[2];     // row I: its helpers [beg, end) (pairs)
  DevBuf<double> d_part;             // partial sums, 128 per helper
  int64_t fill_tiles = 0;                // lower tiles (with diagonal) in the pattern
  double sparse_flops = 0;               // factorisation flops on the pattern
  // Level schedule of a block-sparse factorisation: block column J's parent
  // in the elimination tree is the first I > J with L(I, J) != 0; columns of
  // equal height in that tree are independent (a column is updated only by
  // its descendants), so each level is one launch of diagonal blocks (lv_cols)
  // and one of column tiles (rows lv_trsm_rows of steps lv_trsm_steps); the
  // tile updates run as launches over listed tiles (lv_pairs), each tile with
  // the columns that update it in that launch (lv_k[lv_kptr[p] ..
  // lv_kptr[p+1])); update launch u runs after level lv_launch_after[u].
  bool levels = false;
  int32_t n_levels = 0;                  // tree height + 1 (computed for every block-sparse plan)
  std::vector<int64_t> lv_col_off, lv_trsm_off, lv_pair_off;
  std::vector<int32_t> lv_launch_after;
  DevBuf<int32_t> d_lv_cols, d_lv_trsm_rows, d_lv_trsm_steps, d_lv_pairs, d_lv_kptr, d_lv_k;
  // schedule: 1 = panel steps, 0 or 2 = levels
  void build_sparse(const MatDesc& d, const std::vector<uint8_t>& fill, hipStream_t st, int schedule = 0);
  void build_levels(const std::vector<int32_t>& height, const std::vector<int32_t>& tr, hipStream_t st);
};

// Symbolic block elimination: closes the lower tile pattern pat[I * nb + J]
// (I >= J) under fill-in.
void symbolic_fill(int nb, std::vector<uint8_t>& pat);

// failed: if given, a non-positive pivot of matrix m sets failed[m] = 1 and
// the column is treated as dropped, instead of raising GENEO_ENOTSPD.
// for_solves = false leaves L in the lower triangle (upper untouched);
// otherwise the factor is put in solve form: the strictly upper blocks
// receive U = L^T, then every off-diagonal block is premultiplied by the
// inverse of its row's diagonal block (lower: inv(L_II) L(I,J); upper:
// inv(U_II) U(I,J)); only solve() / solve_multi() read that form.
void factor(const FactorPlan& P, double* A, double* Ainv, const double* odiag, double drop_tol, double* pivrel,
            DevErr* err, hipStream_t st, int32_t* failed = nullptr, bool for_solves = true);
void factor(const FactorPlan& P, float* A, float* Ainv, const double* odiag, double drop_tol, double* pivrel,
            DevErr* err, hipStream_t st, int32_t* failed = nullptr, bool for_solves = true);
// x <- (L L^T)^-1 x on every matrix segment of the batch vector x (other
// segments are left as they are; the plan's d_y holds the intermediate).
void solve(const FactorPlan& P, const double* A, const double* Ainv, double* x, unsigned* sync, DevErr* err,
           hipStream_t st);
void solve(const FactorPlan& P, const float* A, const float* Ainv, double* x, unsigned* sync, DevErr* err,
           hipStream_t st);
// X <- (L L^T)^-1 X for k <= 32 columns: the block of matrix m starts at
// X + voff_m * ldk, column q at + q * ld_m.
void solve_multi(const FactorPlan& P, const double* A, const double* Ainv, double* X, int ldk, int k,
                 unsigned* sync, unsigned* flags, DevErr* err, hipStream_t st);
void solve_multi(const FactorPlan& P, const float* A, const float* Ainv, double* X, int ldk, int k,
                 unsigned* sync, unsigned* flags, DevErr* err, hipStream_t st);

}  // namespace geneo
