// The two-level preconditioner handle and the kernels shared by setup,
// apply, the eigensolver and PCG.
#pragma once

#include "dense.h"

struct geneo_precond {
  const geneo_system* sys = nullptr;
  const geneo_decomp* dec = nullptr;
  geneo_setup_opts opts{};
  geneo_precond_info info{};
  int32_t N = 0;
  int precision = GENEO_FP64;

  // local dense factors (one of the two precisions), batch layout
  geneo::FactorPlan local;
  geneo::DevBuf<double> dL, dLinv;
  geneo::DevBuf<float> fL, fLinv;
  geneo::DevBuf<unsigned> d_flags_local;
  // FP32_REFINE1: subdomains that kept their FP32 factor and those refactored
  // in FP64 after the probe (empty when none fell back: `local` serves all)
  geneo::FactorPlan local32, local64;
  int32_t n_fallback = 0;
  geneo::DevBuf<int8_t> d_refine;            // batch row -> 1 if its subdomain is refined (FP32)
  // batch-row CSR of the local matrices A_i (columns = batch positions,
  // values = slots of the global CSR), for the FP64 residual of the refinement
  geneo::DevBuf<int64_t> d_brp;
  geneo::DevBuf<int32_t> d_bcol;                // FP32 path: batch columns of the local triplets
  int64_t batch_len = 0;                     // sum of n_pad
  std::vector<int64_t> voff;                 // batch offset of each subdomain
  geneo::DevBuf<int32_t> d_bmap;             // batch index -> free edge (-1 in pads)
  geneo::DevBuf<double> d_bpou;              // batch index -> D_i value (0 in pads)
  geneo::DevBuf<int32_t> d_inv_ptr, d_inv_idx;  // free edge -> batch indices
  // local sparse matrices (CSR, local column ids) for refinement / eigensolver
  std::vector<int64_t> lnnz_off;             // [N+1]
  geneo::DevBuf<int32_t> d_lrowptr;          // [sum(n_i)+N], per subdomain rowptr segment
  geneo::DevBuf<int64_t> d_lrow_off;         // [N+1] start of each rowptr segment
  geneo::DevBuf<int32_t> d_lcol, d_lslot, d_lrow;
  geneo::HostVec<int32_t> h_lrow, h_lcol;     // host copies of the local rows / columns (eigensolver plans)
  geneo::DevBuf<int64_t> d_lnnz_off;

  // coarse space: SNK columns (sparse) + GenEO columns (dense local blocks)
  int32_t n0 = 0, n_snk = 0, n_gen = 0;   // columns of the assembled coarse matrix (after the local test)
  int32_t n_snk_all = 0;                    // SNK columns before it (the paper's SNK size)
  geneo::FactorPlan coarse;
  geneo::DevBuf<double> dE, dEinv, d_odiag, d_pivrel;
  geneo::DevBuf<int32_t> d_zc_ptr, d_zc_row;   // SNK columns: free edges
  geneo::DevBuf<double> d_zc_val;
  geneo::DevBuf<int32_t> d_zr_ptr, d_zr_col;   // SNK rows: coarse columns
  geneo::DevBuf<double> d_zr_val;
  std::vector<int32_t> gen_cnt;              // GenEO columns per subdomain
  std::vector<int64_t> gen_off;              // first GenEO coarse column of each subdomain (relative)
  std::vector<int64_t> w_off;                // element offset of W_j in d_W (column-major n_pad x m_j)
  geneo::DevBuf<double> d_W;                 // D_j (I - xi_j) V_j, batch-row layout
  geneo::DevBuf<int64_t> d_w_off, d_gen_off;
  geneo::DevBuf<int32_t> d_gen_cnt;
  geneo::DevBuf<int64_t> d_voff;
  geneo::DevBuf<int32_t> d_n;

  // final Ritz block of the eigensolver (kept on request, for training the warm start)
  geneo::DevBuf<double> d_ritz;
  int32_t ritz_k = 0;

  // eigen results (host)
  std::vector<std::vector<double>> eigs;
  std::vector<int32_t> eig_sel;

  // work vectors
  geneo::DevBuf<double> w_b1, w_b2, w_b3;    // batch vectors
  geneo::DevBuf<double> w_n1, w_n2, w_n3, w_n4;  // length n
  geneo::DevBuf<double> w_c1, w_c2, w_c3;    // length n0_pad
  // coarse columns in the factor's order: natural column c sits at position
  // d_cperm[c] (empty: natural order); every group of the order starts at a
  // multiple of 128, the positions in between are unit pad columns
  geneo::DevBuf<int32_t> d_cperm;
};

namespace geneo {

void launch_spmv(const geneo_system* s, const double* x, double* y, hipStream_t st);
// y = |b| + |A| |x| (componentwise)
void launch_spmv_abs(const geneo_system* s, const double* x, const double* b, double* y, hipStream_t st);
void setup_precond(geneo_ctx* ctx, geneo_precond* pc);
void apply_precond(geneo_ctx* ctx, const geneo_precond* pc, const double* r, double* z);
void pcg(geneo_ctx* ctx, const geneo_system* sys, const geneo_precond* pc, const double* b, double* x,
         const geneo_solve_opts* o, geneo_solve_info* info);
// right-preconditioned GMRES (restart opts->restart, 0 = none)
void gmres(geneo_ctx* ctx, const geneo_system* sys, const geneo_precond* pc, const double* b, double* x,
           const geneo_solve_opts* o, geneo_solve_info* info);
void check_device_error(geneo_ctx* ctx);
// nested-dissection order of the subdomains on their coupling graph: groups
// (leaves and separators) in elimination order; *levels = dissection depth
std::vector<std::vector<int32_t>> subdomain_elimination_order(const geneo_system* s, const geneo_decomp* dec,
                                                              int* levels,
                                                              std::vector<std::vector<int32_t>>* adj_out = nullptr);
// longest dependency chain of E's block triangular solves for the column
// order pos_sub (subdomain of each factor position, -1 = pad), predicted from
// the subdomain adjacency
int predicted_solve_depth(const std::vector<int32_t>& pos_sub, const std::vector<std::vector<int32_t>>& adj);
// eigensolver (geneo_eig.hip)
void solve_local_gevps(geneo_ctx* ctx, geneo_precond* pc);

// deterministic dot product: out[0] = x . y  (device scalar)
void dot(const double* x, const double* y, int64_t n, double* partial, double* out, hipStream_t st);

}  // namespace geneo
