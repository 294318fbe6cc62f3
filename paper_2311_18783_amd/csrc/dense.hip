// Batched dense Cholesky factorisation and triangular solves for matrices of
// uneven size (the overlapping local matrices A_i and the coarse matrix E).
//
// Layout: matrix m is column-major, ld = n_pad (a multiple of NB = 128),
// starting at element offset off; pad rows/columns hold the identity, so
// every panel and tile is a full 128 x 128 block.  Blocked right-looking
// Cholesky, one launch per phase per panel step covers every matrix still
// active at that step:
//   potrf : the 128 x 128 diagonal block, factored and inverted in LDS;
//   trsm  : L21 = A21 inv(L11)^T as MFMA GEMM tiles (128 rows per workgroup);
//   syrk  : A22 -= L21 L21^T on the lower 128 x 128 tiles (MFMA).
// The inverses of the diagonal blocks are kept and used by the triangular
// solves.  Each MFMA workgroup is 4 waves, one 64 x 64 sub-tile each, with
// operands read straight from L2/HBM: at the FP64 MFMA rate of gfx950 the
// operand stream per CU is a small fraction of what the caches deliver.
//
// Pivot rule: a non-positive pivot is an error (matrix, column) unless a
// drop tolerance is given; then a column whose Schur pivot is <= drop_tol
// times its original diagonal is dependent on the earlier columns: it gets a
// unit diagonal, a zero column, and zero row and column in the block
// inverse, so every solve returns 0 in that position.
#include <algorithm>
#include <cstdlib>
#include <string>
#include <type_traits>

#include "dense.h"

namespace geneo {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T> struct AccT;
template <> struct AccT<double> { using type = d4_t; };
template <> struct AccT<float> { using type = f4_t; };

__device__ inline d4_t mfma16(double a, double b, d4_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline f4_t mfma16(float a, float b, f4_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

__device__ inline void set_err(DevErr* e, int code, int mat, int idx) {
  if (atomicCAS(&e->code, 0, code) == 0) {
    e->mat = mat;
    e->idx = idx;
  }
}

// ---------------------------------------------------------------- potrf
constexpr int LDA = NB + 1;

// The diagonal block is factored and inverted with its elements held in
// registers: each thread owns one row i and the 16 columns c = h + 8q of one
// column phase h (q = 0..15).  Column j of the Schur complement travels
// through a double-buffered LDS vector, so every column step costs one
// barrier; chunks of columns and waves of rows that have left the active
// trailing triangle skip their work.  This step is sequential (the rest of
// the panel step waits on it), so its latency, not its flop rate, matters.
constexpr int kPotrfThreads = 1024;
constexpr int kPotrfCols = NB * NB / kPotrfThreads;   // 16 register columns per thread

template <typename T>
__global__ __launch_bounds__(kPotrfThreads) void k_potrf(const MatDesc* __restrict__ desc,
                                                         const int32_t* __restrict__ order, int step_arg,
                                                         T* __restrict__ A, T* __restrict__ Ainv,
                                                         const double* __restrict__ odiag, double drop_tol,
                                                         double* __restrict__ pivrel, DevErr* err,
                                                         int32_t* __restrict__ failed,
                                                         const int32_t* __restrict__ steps) {
  extern __shared__ unsigned char smem_raw[];
  T* Ls = reinterpret_cast<T*>(smem_raw);   // [NB * LDA] column-major: L, later X = inv(L)
  __shared__ double colbuf[2][NB];          // current Schur column (unscaled)
  __shared__ double xrow[2][NB];            // finished row of X
  __shared__ double invd[NB];               // 1 / L[j][j], 0 for a dropped or failed pivot
  __shared__ double od[NB];                 // original diagonal (drop rule)
  constexpr int H = kPotrfThreads / NB;     // column phases (8)
  // steps != nullptr: one matrix, workgroup b factors the diagonal block of step steps[b]
  const int m = steps ? order[0] : order[blockIdx.x];
  const int step = steps ? steps[blockIdx.x] : step_arg;
  if (failed && failed[m]) return;          // abandoned at an earlier step
  const MatDesc d = desc[m];
  const int t = threadIdx.x;
  // wave w holds rows 64 rh .. 64 rh + 63 for column phase h; rh alternates
  // with w / 4 so that the waves of each SIMD (w mod 4) cover both row halves
  const int w = t >> 6;
  const int rh = (w >> 2) & 1;
  const int h = (w & 3) + 4 * (w >> 3);
  const int i = 64 * rh + (t & 63);
  const int wave_row_max = (i | 63);
  const int64_t k0 = (int64_t)step * NB;
  T* blk = A + d.off + k0 * d.ld + k0;
  const bool use_drop = drop_tol > 0.0;
  const bool have_od = odiag && d.diag_off >= 0;
  T a[kPotrfCols];
#pragma unroll
  for (int q = 0; q < kPotrfCols; ++q) {
    const int c = h + H * q;
    a[q] = (i >= c) ? blk[(int64_t)c * d.ld + i] : T(0);
  }
  if (h == 0) {
    colbuf[0][i] = (double)a[0];
    od[i] = have_od ? odiag[d.diag_off + k0 + i] : 0.0;
  }
  __syncthreads();
  // ---- factorisation, column by column
  for (int j = 0; j < NB; ++j) {
    const double* buf = colbuf[j & 1];
    const double p = buf[j];
    const double o = od[j];
    bool fail = false, drop = false;
    if (use_drop) drop = !(p > drop_tol * o) || !(o > 0.0);
    if (!drop && !(p > 0.0)) fail = true;
    const double sq = (drop || fail) ? 1.0 : sqrt(p);
    const double s = (drop || fail) ? 0.0 : 1.0 / sq;
    if (t == 0) {
      if (use_drop && pivrel && d.diag_off >= 0) pivrel[d.diag_off + k0 + j] = o > 0.0 ? p / o : 0.0;
      if (fail) {
        if (failed)
          failed[m] = 1;   // caller handles it (the column is treated as dropped)
        else
          set_err(err, GENEO_ENOTSPD, m, (int)(k0 + j));
      }
      invd[j] = s;
    }
    if (wave_row_max >= j) {
      const T li = (i > j) ? (T)(buf[i] * s) : T(0);
      T nxt = T(0);
#pragma unroll
      for (int g = 0; g < kPotrfCols / 4; ++g) {
        if (32 * g + 31 >= j) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int q = 4 * g + e;
            const int c = h + H * q;
            T v = a[q];
            if (c == j) {
              v = (i == j) ? (T)sq : li;
            } else if (c > j && i >= c) {
              v -= li * (T)(buf[c] * s);
            }
            a[q] = v;
            if (c == j + 1) nxt = v;
          }
        }
      }
      if (j + 1 < NB && h == ((j + 1) & (H - 1)) && i >= j + 1) colbuf[(j + 1) & 1][i] = (double)nxt;
    }
    __syncthreads();
  }
  // L back to the matrix (lower part of the block) and into LDS
#pragma unroll
  for (int q = 0; q < kPotrfCols; ++q) {
    const int c = h + H * q;
    if (i >= c) blk[(int64_t)c * d.ld + i] = a[q];
    Ls[c * LDA + i] = a[q];
    a[q] = T(0);
  }
  __syncthreads();
  // ---- X = inv(L) by forward substitution L X = I, one row of X per step:
  // row k is final once the updates of steps < k are in; it is scaled by
  // 1 / L[k][k] and broadcast, then rows i > k take X[i][c] -= L[i][k] X[k][c].
  for (int k = 0; k < NB; ++k) {
    double* xr = xrow[k & 1];
    if (i == k) {
      const double dk = invd[k];
#pragma unroll
      for (int q = 0; q < kPotrfCols; ++q) {
        const int c = h + H * q;
        if (c <= k) {
          const T x = (c == k) ? (T)dk : (T)((double)a[q] * dk);
          a[q] = x;
          xr[c] = (double)x;
        }
      }
    }
    __syncthreads();
    if (wave_row_max > k) {
      const T lik = (i > k) ? Ls[k * LDA + i] : T(0);
#pragma unroll
      for (int g = 0; g < kPotrfCols / 4; ++g) {
        if (32 * g <= k) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int q = 4 * g + e;
            const int c = h + H * q;
            if (c <= k && i > k) a[q] -= lik * (T)xr[c];
          }
        }
      }
    }
  }
  T* inv = Ainv + d.inv_off + (int64_t)step * NB * NB;
  T* uinv = Ainv + d.inv_off + ((int64_t)d.nblk + step) * NB * NB;   // inv(U_II) = inv(L_II)^T
#pragma unroll
  for (int q = 0; q < kPotrfCols; ++q) {
    const int c = h + H * q;
    inv[(int64_t)c * NB + i] = (i >= c) ? a[q] : T(0);
  }
  __syncthreads();   // every read of L in LDS is done
#pragma unroll
  for (int q = 0; q < kPotrfCols; ++q) {
    const int c = h + H * q;
    Ls[c * LDA + i] = (i >= c) ? a[q] : T(0);
  }
  __syncthreads();
  // uinv[c][r] (column-major) = X[c][r]: lanes over r for coalesced stores
#pragma unroll
  for (int q = 0; q < kPotrfCols; ++q) {
    const int c = h + H * q;
    uinv[(int64_t)c * NB + i] = Ls[i * LDA + c];
  }
}

// ------------------------------------------------------------ MFMA tiles
// A workgroup owns a 128 x 128 output tile C and accumulates
//   C (+)= sum_k Arow[r][k] * Brow[c][k]
// with Arow/Brow column-major (leading dimensions lda/ldb).  Lane l of a
// 16x16x4 MFMA supplies A[l%16][l/16] and B[l/16][l%16]; it receives
// D[4*(l/16)+v][l%16] (FP32) or D[(l/16)+4*v][l%16] (FP64), v = 0..3.
//
// Tile modes: 0 = 4 waves of 64 x 64, operands straight from L2/HBM;
// 1 = 8 waves of 64 x 32 (half the accumulators per wave, two workgroups
// per CU to hide load latency); 2 = 4 waves, operands staged through LDS.
template <int MODE> struct TileGeo {
  static constexpr int WAVES = MODE == 1 ? 8 : 4;
  static constexpr int BJ = MODE == 1 ? 2 : 4;    // 16-column blocks per wave
  static constexpr int WCOL = 16 * BJ;            // columns per wave
  __device__ static int wr() { return (threadIdx.x >> 6) & 1; }
  __device__ static int wc() { return (threadIdx.x >> 6) >> 1; }
};

template <typename T, int MODE>
__device__ inline void tile_mma_direct(const T* __restrict__ Ar, int64_t lda, const T* __restrict__ Br, int64_t ldb,
                                       typename AccT<T>::type acc[4][TileGeo<MODE>::BJ], bool negate, int K) {
  constexpr int BJ = TileGeo<MODE>::BJ;
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
  Ar += 64 * TileGeo<MODE>::wr();
  Br += TileGeo<MODE>::WCOL * TileGeo<MODE>::wc();
  for (int kk = 0; kk < K; kk += 4) {
    T af[4], bf[BJ];
#pragma unroll
    for (int b = 0; b < 4; ++b) af[b] = Ar[(int64_t)(kk + lk) * lda + 16 * b + lr];
#pragma unroll
    for (int b = 0; b < BJ; ++b) bf[b] = Br[(int64_t)(kk + lk) * ldb + 16 * b + lr];
    if (negate) {
#pragma unroll
      for (int b = 0; b < 4; ++b) af[b] = -af[b];
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj) acc[bi][bj] = mfma16(af[bi], bf[bj], acc[bi][bj]);
  }
}

constexpr int KCH = 32;   // K-chunk staged through LDS (mode 2)

// Mode 2: the workgroup's 128 A rows and 128 B rows are copied chunk by chunk
// (32 columns, 16-byte loads) into a double-buffered LDS stage while the
// MFMAs consume the previous chunk.
template <typename T>
__device__ inline void tile_mma_lds(const T* __restrict__ Ar, int64_t lda, const T* __restrict__ Br, int64_t ldb,
                                    typename AccT<T>::type acc[4][4], bool negate, T* smem, int NCH) {
  constexpr int E = 16 / sizeof(T);                 // elements per 16-byte unit
  constexpr int UNITS = KCH * NB / E;               // units per matrix per chunk
  constexpr int PER = UNITS / 256;                  // units per thread
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = w & 1, wc = w >> 1;
  const int lr = lane & 15, lk = lane >> 4;
  float4 ra[PER], rb[PER];
  int koff[PER], roff[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int u = tid + 256 * i;
    koff[i] = u / (NB / E);
    roff[i] = (u % (NB / E)) * E;
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    ra[i] = *reinterpret_cast<const float4*>(Ar + (int64_t)koff[i] * lda + roff[i]);
    rb[i] = *reinterpret_cast<const float4*>(Br + (int64_t)koff[i] * ldb + roff[i]);
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    *reinterpret_cast<float4*>(smem + koff[i] * NB + roff[i]) = ra[i];
    *reinterpret_cast<float4*>(smem + KCH * NB + koff[i] * NB + roff[i]) = rb[i];
  }
  __syncthreads();
  for (int c = 0; c < NCH; ++c) {
    if (c + 1 < NCH) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        ra[i] = *reinterpret_cast<const float4*>(Ar + (int64_t)((c + 1) * KCH + koff[i]) * lda + roff[i]);
        rb[i] = *reinterpret_cast<const float4*>(Br + (int64_t)((c + 1) * KCH + koff[i]) * ldb + roff[i]);
      }
    }
    const T* As = smem + (c & 1) * 2 * KCH * NB + 64 * wr;
    const T* Bs = smem + (c & 1) * 2 * KCH * NB + KCH * NB + 64 * wc;
#pragma unroll
    for (int kk = 0; kk < KCH; kk += 4) {
      T af[4], bf[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        af[b] = As[(kk + lk) * NB + 16 * b + lr];
        bf[b] = Bs[(kk + lk) * NB + 16 * b + lr];
      }
      if (negate) {
#pragma unroll
        for (int b = 0; b < 4; ++b) af[b] = -af[b];
      }
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mfma16(af[bi], bf[bj], acc[bi][bj]);
    }
    if (c + 1 < NCH) {
      T* As1 = smem + ((c + 1) & 1) * 2 * KCH * NB;
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        *reinterpret_cast<float4*>(As1 + koff[i] * NB + roff[i]) = ra[i];
        *reinterpret_cast<float4*>(As1 + KCH * NB + koff[i] * NB + roff[i]) = rb[i];
      }
    }
    __syncthreads();
  }
}

// row of accumulator element v held by `lane` in a 16x16 output block
template <typename T> __device__ inline int acc_row(int lane, int v);
template <> __device__ inline int acc_row<float>(int lane, int v) { return 4 * (lane >> 4) + v; }
template <> __device__ inline int acc_row<double>(int lane, int v) { return (lane >> 4) + 4 * v; }

// C points at the wave's 64 x (16 BJ) sub-tile
template <typename T, int BJ>
__device__ inline void tile_load(const T* C, int64_t ldc, typename AccT<T>::type acc[4][BJ]) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15;
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[bi][bj][v] = C[(int64_t)(16 * bj + col) * ldc + 16 * bi + acc_row<T>(lane, v)];
}

template <typename T, int BJ>
__device__ inline void tile_store(T* C, int64_t ldc, typename AccT<T>::type acc[4][BJ]) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15;
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) C[(int64_t)(16 * bj + col) * ldc + 16 * bi + acc_row<T>(lane, v)] = acc[bi][bj][v];
}

template <typename T, int MODE>
__device__ inline void tile_mma(const T* Ar, int64_t lda, const T* Br, int64_t ldb,
                                typename AccT<T>::type acc[4][TileGeo<MODE>::BJ], bool negate, int K, T* smem) {
  if constexpr (MODE == 2)
    tile_mma_lds<T>(Ar, lda, Br, ldb, acc, negate, smem, K / KCH);
  else
    tile_mma_direct<T, MODE>(Ar, lda, Br, ldb, acc, negate, K);
}

__device__ inline int find_mat(const int64_t* __restrict__ prefix, int cnt, int64_t w) {
  int lo = 0, hi = cnt - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= w) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// L21 = A21 * inv(L11)^T, one 128-row tile per workgroup.  With `steps` (a
// block-sparse matrix): workgroup b takes row block rows[b] of step steps[b].
template <typename T, int MODE>
__global__ __launch_bounds__(64 * TileGeo<MODE>::WAVES) __attribute__((amdgpu_waves_per_eu(1, MODE == 2 ? 1 : 4))) void k_trsm(
    const MatDesc* __restrict__ desc, const int32_t* __restrict__ order, const int64_t* __restrict__ prefix, int cnt,
    int step_arg, T* __restrict__ A, const T* __restrict__ Ainv, const int32_t* __restrict__ rows,
    const int32_t* __restrict__ skip, const int32_t* __restrict__ steps) {
  using G = TileGeo<MODE>;
  const int step = steps ? steps[blockIdx.x] : step_arg;
  extern __shared__ unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int j = rows ? 0 : find_mat(prefix, cnt, blockIdx.x);
  if (skip && skip[order[j]]) return;   // factor already abandoned (non-positive pivot)
  const MatDesc d = desc[order[j]];
  const int64_t k0 = (int64_t)step * NB;
  // first row of the tile: dense = every block below the panel, sparse = the listed ones
  const int64_t rt = rows ? (int64_t)rows[blockIdx.x] * NB : k0 + NB + (blockIdx.x - prefix[j]) * NB;
  using Acc = typename AccT<T>::type;
  Acc acc[4][G::BJ];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < G::BJ; ++bj) acc[bi][bj] = Acc{0, 0, 0, 0};
  const T* inv = Ainv + d.inv_off + (int64_t)step * NB * NB;   // B rows: inv[c][k] at k*NB + c
  tile_mma<T, MODE>(A + d.off + k0 * d.ld + rt, d.ld, inv, NB, acc, false, NB, smem);
  __syncthreads();   // every wave has read the A21 tile: safe to overwrite
  tile_store<T, G::BJ>(A + d.off + (k0 + G::WCOL * G::wc()) * d.ld + rt + 64 * G::wr(), d.ld, acc);
}

// Trailing update with a group of kb panels:
//   C[ti][tj] -= sum over panel columns [kcol0*NB, (kcol0+kb)*NB) of L[ti] L[tj]^T
// for block tiles ti >= tj >= b0; ncols == 0: every trailing column block,
// else only the ncols block columns from b0 (enumerated column by column).
template <typename T, int MODE>
__global__ __launch_bounds__(64 * TileGeo<MODE>::WAVES) __attribute__((amdgpu_waves_per_eu(1, MODE == 2 ? 1 : 4))) void k_syrk(
    const MatDesc* __restrict__ desc, const int32_t* __restrict__ order, const int64_t* __restrict__ prefix, int cnt,
    int kcol0, int kb, int b0, int ncols, T* __restrict__ A, const int32_t* __restrict__ pairs,
    const int32_t* __restrict__ skip) {
  using G = TileGeo<MODE>;
  const int j = pairs ? 0 : find_mat(prefix, cnt, blockIdx.x);
  if (skip && skip[order[j]]) return;   // factor already abandoned (non-positive pivot)
  const MatDesc d = desc[order[j]];
  int64_t u = pairs ? 0 : blockIdx.x - prefix[j];
  int64_t ti, tj;
  if (pairs) {
    ti = pairs[2 * (int64_t)blockIdx.x];
    tj = pairs[2 * (int64_t)blockIdx.x + 1];
  } else if (ncols == 0) {
    ti = (int64_t)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > u) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= u) ++ti;
    tj = u - ti * (ti + 1) / 2;
    ti += b0;
    tj += b0;
  } else {
    tj = b0;
    while (u >= d.nblk - tj) {
      u -= d.nblk - tj;
      ++tj;
    }
    ti = tj + u;
  }
  const int64_t k0 = (int64_t)kcol0 * NB;
  extern __shared__ unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  using Acc = typename AccT<T>::type;
  Acc acc[4][G::BJ];
  T* C = A + d.off + (tj * NB + G::WCOL * G::wc()) * d.ld + ti * NB + 64 * G::wr();
  tile_load<T, G::BJ>(C, d.ld, acc);
  tile_mma<T, MODE>(A + d.off + k0 * d.ld + ti * NB, d.ld, A + d.off + k0 * d.ld + tj * NB, d.ld, acc, true,
                    kb * NB, smem);
  tile_store<T, G::BJ>(C, d.ld, acc);
}

// Update of a block-sparse matrix by one elimination-tree level: tile b is
// (pairs[2b], pairs[2b+1]) and receives
//   C -= sum over q in [kptr[b], kptr[b+1]) of L[ti][klist[q]] L[tj][klist[q]]^T
// (in that order).  A kernel of its own: the list loop in k_syrk doubles
// that kernel's registers.
template <typename T, int MODE>
__global__ __launch_bounds__(64 * TileGeo<MODE>::WAVES) __attribute__((amdgpu_waves_per_eu(1, MODE == 2 ? 1 : 4))) void k_syrk_lv(
    const MatDesc* __restrict__ desc, const int32_t* __restrict__ order, T* __restrict__ A,
    const int32_t* __restrict__ pairs, const int32_t* __restrict__ kptr, const int32_t* __restrict__ klist,
    const int32_t* __restrict__ skip) {
  using G = TileGeo<MODE>;
  if (skip && skip[order[0]]) return;
  const MatDesc d = desc[order[0]];
  const int64_t ti = pairs[2 * (int64_t)blockIdx.x], tj = pairs[2 * (int64_t)blockIdx.x + 1];
  extern __shared__ unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  using Acc = typename AccT<T>::type;
  Acc acc[4][G::BJ];
  T* C = A + d.off + (tj * NB + G::WCOL * G::wc()) * d.ld + ti * NB + 64 * G::wr();
  tile_load<T, G::BJ>(C, d.ld, acc);
  const int q1 = kptr[blockIdx.x + 1];
  for (int q = kptr[blockIdx.x]; q < q1; ++q) {
    const int64_t kc = (int64_t)klist[q] * NB;
    tile_mma<T, MODE>(A + d.off + kc * d.ld + ti * NB, d.ld, A + d.off + kc * d.ld + tj * NB, d.ld, acc, true, NB,
                      smem);
  }
  tile_store<T, G::BJ>(C, d.ld, acc);
}

// ------------------------------------------- recursive diagonal block (FP64)
constexpr int kRecThreads = 256;

__device__ inline double rl(double v, int lane) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Storage of the block while it is worked on (LDS, column-major, leading
// dimension LDA): the strictly lower triangle holds L, the diagonal and the
// strict upper triangle hold X = inv(L) transposed (X[r][c], r >= c, at
// Ls[r * LDA + c]); the diagonal of L sits in ldg.

// One wavefront factors and inverts the 16 x 16 block at (r0, r0): lane i
// (mod 16) holds row i, lanes 16..63 duplicate lanes 0..15 and store
// nothing.  Entries above the diagonal are carried along unmasked (finite,
// never read back), which keeps per-lane predicates out of the column loop.
// Lane j keeps the pivot data of column j; pivot ratios and failures are
// written lane-parallel at the end.  Forced inline: as a called function it
// saves and restores the caller's registers through scratch memory on every
// one of the eight calls per diagonal block.
__device__ __attribute__((always_inline)) inline void leaf16(double* Ls, double* ldg, const double* od, int r0, double drop_tol,
                              double* pivrel_row, int m, int64_t gcol0, DevErr* err, int32_t* failed) {
  const int lane = threadIdx.x & 63;
  int i = lane & 15;
  // opaque per call: keeps the lane predicates below from being hoisted out
  // of the caller's loop and held across all leaves
  asm volatile("" : "+v"(i));
  const bool use_drop = drop_tol > 0.0;
  double v[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) v[c] = Ls[(r0 + c) * LDA + r0 + i];
  const double my_o = od[r0 + i];
  double my_dinv = 0.0, my_p = 0.0, my_sq = 1.0;
  bool my_fail = false;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const double p = rl(v[j], j);
    bool drop = false;
    if (use_drop) {
      const double o = rl(my_o, j);
      drop = !(p > drop_tol * o) || !(o > 0.0);
    }
    const bool fail = !drop && !(p > 0.0);
    // 1 / sqrt(p): hardware estimate and two Newton steps (relative error
    // squares each step), then sqrt(p) = p / sqrt(p); short dependent chain
    double y = __builtin_amdgcn_rsq(p);
    y = y * (1.5 - 0.5 * p * y * y);
    y = y * (1.5 - 0.5 * p * y * y);
    const double sq = (drop || fail) ? 1.0 : p * y;
    const double sc = (drop || fail) ? 0.0 : y;
    const bool below = i > j, diag = i == j;
    if (diag) {
      my_dinv = sc;
      my_p = p;
      my_sq = sq;
      my_fail = fail;
    }
    const double l = below ? v[j] * sc : 0.0;
    v[j] = l;
#pragma unroll
    for (int c = j + 1; c < 16; ++c) v[c] -= l * rl(l, c);
  }
  const uint64_t fails = __ballot(my_fail && lane < 16);
  if (lane < 16) {
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (c < i) Ls[(r0 + c) * LDA + r0 + i] = v[c];
    Ls[(r0 + i) * LDA + r0 + i] = my_dinv;
    ldg[r0 + i] = my_sq;
    if (use_drop && pivrel_row) pivrel_row[r0 + i] = my_o > 0.0 ? my_p / my_o : 0.0;
    if (fails && lane == __builtin_ctzll(fails)) {   // first failing column of the leaf
      if (failed)
        failed[m] = 1;   // caller handles it (the column is treated as dropped)
      else
        set_err(err, GENEO_ENOTSPD, m, (int)(gcol0 + r0 + i));
    }
  }
  // X = inv(L) column by column: lane i solves L x = e_i top to bottom (the
  // entries above i come out as exact zeros).  L[r][t] and 1 / L[r][r] are
  // read back from LDS at the same address in every lane (a broadcast); LDS
  // accesses of one wavefront complete in order, so the stores above are
  // visible.  Two partial sums halve the dependent FMA chain.
  double x[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    double acc0 = r == i ? 1.0 : 0.0, acc1 = 0.0;
#pragma unroll
    for (int t = 0; t + 1 < r; t += 2) {
      acc0 -= Ls[(r0 + t) * LDA + r0 + r] * x[t];
      acc1 -= Ls[(r0 + t + 1) * LDA + r0 + r] * x[t + 1];
    }
    if (r & 1) acc0 -= Ls[(r0 + r - 1) * LDA + r0 + r] * x[r - 1];
    x[r] = (acc0 + acc1) * Ls[(r0 + r) * LDA + r0 + r];
  }
  if (lane < 16) {
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (c > i) Ls[(r0 + c) * LDA + r0 + i] = x[c];   // X[c][i]
  }
}

// Products of the recursion for a block [L11 0; L21 L22] whose halves start
// at rows a0 and b0 = a0 + H (H = 16 NT).  Output tiles are 16 x 16 on
// v_mfma_f64_16x16x4; a triangular operand contributes only its nonzero
// k-tiles, its diagonal k-tile is masked.
//   0: L21 = A21 X11^T (in place)       1: A22 -= L21 L21^T (lower tiles)
//   2: T = L21 X11 (upper right block)  3: X21 = -X22 T (over T)
// For H = 64 wave w owns tile row w (kinds 0-2, operand A shared across the
// row) or tile column w (kind 3); for H = 32 one tile each; H = 16 wave 0.
template <int KIND>
struct RecOp {
  double* Ls;
  int a0, b0;
  __device__ double X(int base, int r, int c) const {   // inv(L) block at (base, base), masked
    const double v = Ls[(base + r) * LDA + base + c];
    return r >= c ? v : 0.0;
  }
  __device__ double L21(int m, int k) const { return Ls[(a0 + k) * LDA + b0 + m]; }
  __device__ double A(int m, int k) const {
    if constexpr (KIND == 3) return X(b0, m, k);
    else return L21(m, k);
  }
  __device__ double B(int k, int n) const {
    if constexpr (KIND == 0) return X(a0, n, k);
    else if constexpr (KIND == 1) return L21(n, k);
    else if constexpr (KIND == 2) return X(a0, k, n);
    else return Ls[(b0 + n) * LDA + a0 + k];   // T[k][n]
  }
  // nonzero k-tile range of output tile (ti, tj)
  __device__ static int kt_lo(int ti, int tj) { return KIND == 2 ? tj : 0; }
  __device__ static int kt_hi(int ti, int tj, int nt) { return KIND == 0 ? tj : (KIND == 3 ? ti : nt - 1); }
  __device__ void put(int m, int n, double v) const {
    if constexpr (KIND == 0) Ls[(a0 + n) * LDA + b0 + m] = v;
    else if constexpr (KIND == 1) Ls[(b0 + n) * LDA + b0 + m] -= v;
    else if constexpr (KIND == 2) Ls[(b0 + n) * LDA + a0 + m] = v;
    else Ls[(b0 + m) * LDA + a0 + n] = -v;
  }
};

template <int KIND>
__device__ inline d4_t rec_tile(const RecOp<KIND>& op, int ti, int tj, int kt0, int kt1, d4_t acc) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  for (int kt = kt0; kt <= kt1; ++kt) {
    double a[4], b[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      a[s] = op.A(16 * ti + lr, 16 * kt + 4 * s + lk);
      b[s] = op.B(16 * kt + 4 * s + lk, 16 * tj + lr);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) acc = mfma16(a[s], b[s], acc);
  }
  return acc;
}

template <int KIND>
__device__ inline void rec_put(const RecOp<KIND>& op, int ti, int tj, const d4_t& acc) {
  const int lane = threadIdx.x & 63;
  if (KIND == 1 && tj > ti) return;   // upper tiles of A22 are not needed
#pragma unroll
  for (int v = 0; v < 4; ++v) op.put(16 * ti + acc_row<double>(lane, v), 16 * tj + (lane & 15), acc[v]);
}

template <int H, int KIND>
__device__ inline void rec_prod(double* Ls, int a0, int b0) {
  constexpr int NT = H / 16;
  constexpr bool STAGED = KIND == 0 || KIND == 3;
  const RecOp<KIND> op{Ls, a0, b0};
  const int w = threadIdx.x >> 6;
  if constexpr (NT == 4) {
    d4_t acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ti = KIND == 3 ? q : w, tj = KIND == 3 ? w : q;
      acc[q] = rec_tile(op, ti, tj, op.kt_lo(ti, tj), op.kt_hi(ti, tj, NT), d4_t{0, 0, 0, 0});
    }
    if constexpr (STAGED) __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) rec_put(op, KIND == 3 ? q : w, KIND == 3 ? w : q, acc[q]);
  } else {
    const int ti = NT == 2 ? (w >> 1) : 0, tj = NT == 2 ? (w & 1) : 0;
    const bool active = NT == 2 || w == 0;
    d4_t acc = d4_t{0, 0, 0, 0};
    if (active) acc = rec_tile(op, ti, tj, op.kt_lo(ti, tj), op.kt_hi(ti, tj, NT), acc);
    if constexpr (STAGED) __syncthreads();
    if (active) rec_put(op, ti, tj, acc);
  }
  __syncthreads();
}

// Diagonal block factorisation and inversion, recursive in halves
// (128 -> 64 -> 32 -> 16): with [L11 0; L21 L22] and X = inv(L),
//   L11, X11 from the upper half;  L21 = A21 X11^T;  A22 -= L21 L21^T;
//   L22, X22 from the lower half;  X21 = -X22 L21 X11.
// The products run as FP64 MFMA tiles on all four waves; the 16 x 16 leaves
// are factored and inverted by one wavefront in registers with cross-lane
// broadcasts and no barriers, so the sequential part drops from 2 x 128
// barrier-separated column steps (k_potrf) to 8 short leaves.  The
// recursion runs as a loop over the leaves in its post-order: after leaf
// lf, each level whose subtree ends at lf finishes its block (kinds 2 and 3
// for a right half, which may close the parent too; kinds 0 and 1 for a left
// half, which hands over to the right sibling).  Same pivot rule and outputs
// as k_potrf.
// two consecutive entries of a T array as doubles, and back
template <typename T> __device__ inline double2 ld2(const T* p);
template <> __device__ inline double2 ld2<double>(const double* p) { return *reinterpret_cast<const double2*>(p); }
template <> __device__ inline double2 ld2<float>(const float* p) {
  const float2 v = *reinterpret_cast<const float2*>(p);
  return double2{(double)v.x, (double)v.y};
}
template <typename T> __device__ inline void st2(T* p, double2 v);
template <> __device__ inline void st2<double>(double* p, double2 v) { *reinterpret_cast<double2*>(p) = v; }
template <> __device__ inline void st2<float>(float* p, double2 v) {
  *reinterpret_cast<float2*>(p) = float2{(float)v.x, (float)v.y};
}

// The diagonal block is worked on in FP64 in LDS for both storage types T:
// an FP32 factor stores the FP64 result rounded to FP32.
template <typename T>
__global__ __launch_bounds__(kRecThreads) void k_potrf_rec(const MatDesc* __restrict__ desc,
                                                           const int32_t* __restrict__ order, int step_arg,
                                                           T* __restrict__ A, T* __restrict__ Ainv,
                                                           const double* __restrict__ odiag, double drop_tol,
                                                           double* __restrict__ pivrel, DevErr* err,
                                                           int32_t* __restrict__ failed,
                                                           const int32_t* __restrict__ steps) {
  extern __shared__ unsigned char smem_raw[];
  double* Ls = reinterpret_cast<double*>(smem_raw);   // [NB * LDA], column-major
  __shared__ double ldg[NB], od[NB];
  // steps != nullptr: one matrix, workgroup b factors the diagonal block of step steps[b]
  const int m = steps ? order[0] : order[blockIdx.x];
  const int step = steps ? steps[blockIdx.x] : step_arg;
  if (failed && failed[m]) return;   // abandoned at an earlier step
  const MatDesc d = desc[m];
  const int tid = threadIdx.x;
  const int64_t k0 = (int64_t)step * NB;
  T* blk = A + d.off + k0 * d.ld + k0;
  const bool have_od = odiag && d.diag_off >= 0;
  // load the lower triangle (two entries per thread and column, 64 threads
  // per column, 4 columns per pass; entries above the diagonal are replaced by zeros)
  const int rr = 2 * (tid & 63), cq = tid >> 6;
  for (int c0 = 0; c0 < NB; c0 += 32) {
    double2 buf[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) buf[u] = ld2<T>(blk + (int64_t)(c0 + 4 * u + cq) * d.ld + rr);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = c0 + 4 * u + cq;
      Ls[c * LDA + rr] = rr >= c ? buf[u].x : 0.0;
      Ls[c * LDA + rr + 1] = rr + 1 >= c ? buf[u].y : 0.0;
    }
  }
  if (tid < NB) od[tid] = have_od ? odiag[d.diag_off + k0 + tid] : 0.0;
  __syncthreads();
  double* pivrel_row = (pivrel && d.diag_off >= 0) ? pivrel + d.diag_off + k0 : nullptr;
  for (int lf = 0; lf < NB / 16; ++lf) {
    if (tid < 64) leaf16(Ls, ldg, od, 16 * lf, drop_tol, pivrel_row, m, k0, err, failed);
    __syncthreads();
    for (int s = 0; s < 3; ++s) {
      if (((lf + 1) & ((1 << s) - 1)) != 0) break;   // lf does not end a level-s subtree
      const int idx = lf >> s, H = 16 << s;
      if ((idx & 1) == 0) {
        const int a0 = idx * H;
        if (s == 0) {
          rec_prod<16, 0>(Ls, a0, a0 + 16);
          rec_prod<16, 1>(Ls, a0, a0 + 16);
        } else if (s == 1) {
          rec_prod<32, 0>(Ls, a0, a0 + 32);
          rec_prod<32, 1>(Ls, a0, a0 + 32);
        } else {
          rec_prod<64, 0>(Ls, a0, a0 + 64);
          rec_prod<64, 1>(Ls, a0, a0 + 64);
        }
        break;
      }
      const int a0 = (idx - 1) * H;
      if (s == 0) {
        rec_prod<16, 2>(Ls, a0, a0 + 16);
        rec_prod<16, 3>(Ls, a0, a0 + 16);
      } else if (s == 1) {
        rec_prod<32, 2>(Ls, a0, a0 + 32);
        rec_prod<32, 3>(Ls, a0, a0 + 32);
      } else {
        rec_prod<64, 2>(Ls, a0, a0 + 64);
        rec_prod<64, 3>(Ls, a0, a0 + 64);
      }
    }
  }
  T* inv = Ainv + d.inv_off + (int64_t)step * NB * NB;
  T* uinv = Ainv + d.inv_off + ((int64_t)d.nblk + step) * NB * NB;   // inv(U_II) = inv(L_II)^T
  for (int c0 = 0; c0 < NB; c0 += 4) {
    const int c = c0 + cq;
    double2 l, x, u;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int r = rr + e;
      const double lo = Ls[c * LDA + r];   // L[r][c] for r > c, X[c][r] for r <= c
      const double up = Ls[r * LDA + c];   // X[r][c] for r >= c
      const double lv = r == c ? ldg[r] : lo;
      const double xv = r >= c ? up : 0.0;
      const double uv = r <= c ? lo : 0.0;
      if (e == 0) { l.x = lv; x.x = xv; u.x = uv; } else { l.y = lv; x.y = xv; u.y = uv; }
    }
    if (rr >= c) {
      st2<T>(blk + (int64_t)c * d.ld + rr, l);
    } else if (rr + 1 == c) {
      blk[(int64_t)c * d.ld + rr + 1] = (T)l.y;
    }
    st2<T>(inv + (int64_t)c * NB + rr, x);
    st2<T>(uinv + (int64_t)c * NB + rr, u);
  }
}

// --------------------------------------------------------------- plan

void FactorPlan::plan_host(const std::vector<MatDesc>& descs, int precision, const FactorConfig* force) {
  h_desc = descs;
  nmat = (int)descs.size();
  std::vector<int32_t>& ord = h_order;
  ord.resize(nmat);
  for (int i = 0; i < nmat; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return descs[a].nblk > descs[b].nblk; });
  max_blk = nmat ? descs[ord[0]].nblk : 0;
  cnt.assign(max_blk, 0);
  trsm_tiles.assign(max_blk, 0);
  syrk_tiles.assign(max_blk, 0);
  pre_off.assign(max_blk, 0);
  std::vector<int64_t>& pre = h_prefix;
  pre.clear();
  for (int s = 0; s < max_blk; ++s) {
    int c = 0;
    while (c < nmat && descs[ord[c]].nblk > s) ++c;
    cnt[s] = c;
    pre_off[s] = (int64_t)pre.size();
    int64_t acc_t = 0, acc_s = 0;
    std::vector<int64_t> pt(c + 1), ps(c + 1);
    for (int k = 0; k < c; ++k) {
      pt[k] = acc_t;
      ps[k] = acc_s;
      int64_t T = descs[ord[k]].nblk - s - 1;
      acc_t += T;
      acc_s += T * (T + 1) / 2;
    }
    pt[c] = acc_t;
    ps[c] = acc_s;
    trsm_tiles[s] = acc_t;
    syrk_tiles[s] = acc_s;
    pre.insert(pre.end(), pt.begin(), pt.end());
    pre.insert(pre.end(), ps.begin(), ps.end());
  }
  // trailing updates for panel groups of G panels: inside a group, block
  // column s0 + g receives the updates of the group's earlier panels in one
  // launch right before its diagonal block (left-looking: K = g * NB, each
  // of its tiles read and written once); after the group, one update with
  // all G panels (K = G * NB) covers the later columns
  cfg = force ? *force : tuned_factor_config(precision, max_blk, nmat);
  group = std::max(1, cfg.group);
  syrk.clear();
  std::vector<int64_t>& spre = h_syrk_prefix;
  spre.clear();
  auto add_launch = [&](int kcol0, int kb, int b0, int ncols) {
    SyrkLaunch L{(int64_t)spre.size(), 0, kcol0, kb, b0, ncols};
    int64_t acc = 0;
    for (int k = 0; k < nmat; ++k) {
      spre.push_back(acc);
      const int64_t N = descs[ord[k]].nblk;
      if (kb > 0 && b0 < N && kcol0 + kb <= N) {
        const int64_t cend = ncols ? std::min<int64_t>(N, b0 + ncols) : N;
        for (int64_t c = b0; c < cend; ++c) acc += N - c;
      }
    }
    spre.push_back(acc);
    L.tiles = acc;
    syrk.push_back(L);
  };
  for (int s0 = 0; s0 < max_blk; s0 += group) {
    for (int g = 0; g < group && s0 + g < max_blk; ++g) {
      const int sg = s0 + g;
      if (g > 0) add_launch(s0, g, sg, 1);   // column sg from panels s0 .. sg - 1
      else add_launch(-1, 0, 0, 0);          // placeholder: none
    }
    add_launch(s0, group, s0 + group, 0);                            // trailing, K = group * NB
  }
  std::vector<int64_t>& mp = h_mirror_prefix;
  mp.assign(nmat + 1, 0);
  for (int k = 0; k < nmat; ++k) {
    int64_t T = descs[ord[k]].nblk;
    mp[k + 1] = mp[k] + T * (T - 1) / 2;
  }
  mirror_tiles = mp[nmat];
  // triangular-solve work items: forward in increasing block order across
  // matrices, backward in decreasing order
  h_items_fwd.clear();
  h_items_bwd.clear();
  for (int s = 0; s < max_blk; ++s)
    for (int k = 0; k < cnt[s]; ++k) {
      int m = ord[k];
      h_items_fwd.push_back(m);
      h_items_fwd.push_back(s);
      h_items_bwd.push_back(m);
      h_items_bwd.push_back(descs[m].nblk - 1 - s);
    }
  n_items = (int64_t)h_items_fwd.size() / 2;
}

void FactorPlan::build(const std::vector<MatDesc>& descs, hipStream_t st, int precision) {
  plan_host(descs, precision);
  d_desc.upload(descs, st);
  d_order.upload(h_order, st);
  d_prefix.upload(h_prefix, st);
  int64_t vec_len = 0;
  for (const auto& dd : descs) vec_len = std::max<int64_t>(vec_len, dd.voff + dd.ld);
  d_y.alloc(std::max<int64_t>(vec_len, 1));
  d_syrk_prefix.upload(h_syrk_prefix, st);
  d_mirror_prefix.upload(h_mirror_prefix, st);
  d_items_fwd.upload(h_items_fwd, st);
  d_items_bwd.upload(h_items_bwd, st);
}

size_t FactorPlan::build_in(const std::vector<MatDesc>& descs, void* mem, size_t bytes, hipStream_t st,
                            int precision) {
  plan_host(descs, precision);
  char* base = static_cast<char*>(mem);
  size_t used = 0;
  auto place = [&](auto& buf, const auto& host) {
    using E = typename std::remove_reference<decltype(host)>::type::value_type;
    const size_t nb = round_up((int64_t)(host.size() * sizeof(E)), 256);
    if (used + nb > bytes) throw Error(GENEO_EINVAL, "plan does not fit the scratch area");
    buf.view(reinterpret_cast<E*>(base + used), host.size());
    if (!host.empty())
      HIP_CHECK(hipMemcpyAsync(buf.p, host.data(), host.size() * sizeof(E), hipMemcpyHostToDevice, st));
    used += nb;
  };
  place(d_desc, h_desc);
  place(d_order, h_order);
  place(d_prefix, h_prefix);
  place(d_syrk_prefix, h_syrk_prefix);
  return used;
}

void symbolic_fill(int nb, std::vector<uint8_t>& pat) {
  std::vector<int> rows;
  for (int k = 0; k < nb; ++k) {
    pat[(size_t)k * nb + k] = 1;
    rows.clear();
    for (int i = k + 1; i < nb; ++i)
      if (pat[(size_t)i * nb + k]) rows.push_back(i);
    for (size_t a = 0; a < rows.size(); ++a)
      for (size_t b = 0; b <= a; ++b) pat[(size_t)rows[a] * nb + rows[b]] = 1;
  }
}

void FactorPlan::build_sparse(const MatDesc& dsc, const std::vector<uint8_t>& F, hipStream_t st, int schedule) {
  build(std::vector<MatDesc>(1, dsc), st);   // dense plan of the single matrix: panel steps, items, groups
  sparse = true;
  const int nb = dsc.nblk;
  auto f = [&](int i, int j) { return F[(size_t)i * nb + j] != 0; };
  // trsm rows per step
  std::vector<int32_t> tr;
  trsm_off.assign(nb + 1, 0);
  for (int s = 0; s < nb; ++s) {
    trsm_off[s] = (int64_t)tr.size();
    for (int i = s + 1; i < nb; ++i)
      if (f(i, s)) tr.push_back(i);
    trsm_tiles[s] = (int64_t)tr.size() - trsm_off[s];
  }
  trsm_off[nb] = (int64_t)tr.size();
  d_trsm_rows.upload(tr.empty() ? std::vector<int32_t>(1, 0) : tr, st);
  // factorisation flops on the pattern (either schedule): per block column k
  // with r_k tiles below the diagonal, its diagonal block, r_k triangular
  // solves and r_k (r_k + 1) / 2 tile products of the update
  sparse_flops = 0;
  for (int k = 0; k < nb; ++k) {
    const double r = (double)trsm_tiles[k];
    sparse_flops += (double)NB * NB * NB * (1.0 / 3.0 + r + r * (r + 1.0));
  }
  // elimination tree: parent = first row block below the diagonal; height
  std::vector<int32_t> height(nb, 0);
  for (int j = 0; j < nb; ++j)
    if (trsm_tiles[j] > 0) {
      const int par = tr[trsm_off[j]];
      height[par] = std::max(height[par], height[j] + 1);
    }
  n_levels = 0;
  for (int j = 0; j < nb; ++j) n_levels = std::max(n_levels, height[j] + 1);
  levels = schedule != 1;
  syrk_off.assign(syrk.size(), 0);
  if (!levels) {
    // trailing-update tiles of each launch of the (dense) launch sequence:
    // (ti, tj) with tj in the launch's column range and L(ti, sp), L(tj, sp)
    // both in the pattern for a panel column sp of the launch, ordered by tj
    // then ti (enumerated from the panels' row lists)
    std::vector<int32_t> pairs;
    std::vector<uint8_t> mark((size_t)nb * nb, 0);
    std::vector<int64_t> keys;
    for (size_t li = 0; li < syrk.size(); ++li) {
      SyrkLaunch& L = syrk[li];
      syrk_off[li] = (int64_t)pairs.size() / 2;
      keys.clear();
      if (L.kb > 0) {
        const int cend = L.ncols ? std::min(nb, L.b0 + L.ncols) : nb;
        for (int sp = L.kcol0; sp < L.kcol0 + L.kb && sp < nb; ++sp) {
          const int32_t* rb = tr.data() + trsm_off[sp];
          const int64_t nr = trsm_off[sp + 1] - trsm_off[sp];
          for (int64_t bq = 0; bq < nr; ++bq) {
            const int tj = rb[bq];
            if (tj < L.b0 || tj >= cend) continue;
            for (int64_t aq = bq; aq < nr; ++aq) {
              const int64_t key = (int64_t)tj * nb + rb[aq];
              if (!mark[(size_t)key]) {
                mark[(size_t)key] = 1;
                keys.push_back(key);
              }
            }
          }
        }
      }
      std::sort(keys.begin(), keys.end());
      for (int64_t key : keys) {
        mark[(size_t)key] = 0;
        pairs.push_back((int32_t)(key % nb));
        pairs.push_back((int32_t)(key / nb));
      }
      L.tiles = (int64_t)keys.size();
    }
    d_syrk_pairs.upload(pairs.empty() ? std::vector<int32_t>(2, 0) : pairs, st);
  } else {
    for (auto& L : syrk) L.tiles = 0;
    build_levels(height, tr, st);
  }
  // strictly lower tiles; solve dependencies
  std::vector<int32_t> lo, fp(nb + 1, 0), fd, bp(nb + 1, 0), bd;
  fill_tiles = 0;
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j <= i; ++j)
      if (f(i, j)) {
        ++fill_tiles;
        if (i > j) {
          lo.push_back(i);
          lo.push_back(j);
        }
      }
  n_lower = (int64_t)lo.size() / 2;
  mirror_tiles = n_lower;
  d_lower_pairs.upload(lo.empty() ? std::vector<int32_t>(2, 0) : lo, st);
  for (int i = 0; i < nb; ++i) {           // forward: J < I with L(I,J) != 0, increasing
    for (int j = 0; j < i; ++j)
      if (f(i, j)) fd.push_back(j);
    fp[i + 1] = (int32_t)fd.size();
  }
  for (int i = 0; i < nb; ++i) {           // backward: J > I with U(I,J) = L(J,I)^T != 0, decreasing
    for (int j = nb - 1; j > i; --j)
      if (f(j, i)) bd.push_back(j);
    bp[i + 1] = (int32_t)bd.size();
  }
  d_dep_fwd_ptr.upload(fp, st);
  d_dep_fwd.upload(fd.empty() ? std::vector<int32_t>(1, 0) : fd, st);
  d_dep_bwd_ptr.upload(bp, st);
  d_dep_bwd.upload(bd.empty() ? std::vector<int32_t>(1, 0) : bd, st);
  // split rows: more than kSplitMin dependencies -> helpers of kSplitChunk
  // dependencies each over all but the row's last kSplitKeep
  constexpr int kSplitMin = 48, kSplitChunk = 32, kSplitKeep = 16;
  int32_t max_help = 0;
  for (int d = 0; d < 2; ++d) {
    const std::vector<int32_t>& ptr = d == 0 ? fp : bp;
    std::vector<int32_t> items, rng, rlo(nb, 0), rhelp(2 * (size_t)nb, 0);
    int32_t nh = 0;
    for (int k = 0; k < nb; ++k) {
      const int I = d == 0 ? k : nb - 1 - k;
      const int nd = ptr[I + 1] - ptr[I];
      rhelp[2 * I] = nh;
      if (nd > kSplitMin) {
        for (int c = 0; c < nd - kSplitKeep; c += kSplitChunk) {
          items.push_back(-1 - nh);
          items.push_back(I);
          rng.push_back(c);
          rng.push_back(std::min(c + kSplitChunk, nd - kSplitKeep));
          ++nh;
        }
        rlo[I] = nd - kSplitKeep;
      }
      rhelp[2 * I + 1] = nh;
      items.push_back(0);
      items.push_back(I);
    }
    n_sitems[d] = (int64_t)items.size() / 2;
    n_help[d] = nh;
    max_help = std::max(max_help, nh);
    d_sitems[d].upload(items, st);
    d_help_rng[d].upload(rng.empty() ? std::vector<int32_t>(2, 0) : rng, st);
    d_row_lo[d].upload(rlo, st);
    d_row_help[d].upload(rhelp, st);
  }
  d_part.alloc(std::max<int64_t>((int64_t)max_help * NB, 1));
}

// Level schedule (see FactorPlan): levels are taken in groups of
// kLevelGroup consecutive ones.  Inside a group, after the diagonal blocks
// and column tiles of a level, a "thin" update applies the level's columns
// to the tiles of the group's later columns; after the group, one update
// applies all the group's columns to every other tile they reach, so such a
// tile is read and written once per group.  Each (tile, column) product
// falls in exactly one of the two.
void FactorPlan::build_levels(const std::vector<int32_t>& height, const std::vector<int32_t>& tr, hipStream_t st) {
  constexpr int kLevelGroup = 8;
  const int nb = (int)height.size();
  std::vector<std::vector<int32_t>> by_level(n_levels);
  for (int j = 0; j < nb; ++j) by_level[height[j]].push_back(j);
  std::vector<int32_t> cols, trows, tsteps, lpairs, kptr(1, 0), klist;
  lv_col_off.assign(1, 0);
  lv_trsm_off.assign(1, 0);
  lv_pair_off.assign(1, 0);   // [thin of level 0, ..., thin of the group's last level, trailing of the group, ...]
  lv_launch_after.clear();
  std::vector<int32_t> slot((size_t)nb * nb, -1);
  std::vector<int32_t> cnt, tiles;   // per pair of the launch being built
  auto rows_of = [&](int k) { return std::make_pair(tr.data() + trsm_off[k], trsm_off[k + 1] - trsm_off[k]); };
  // one update launch from the (k, ti, tj) triples that `emit` enumerates
  auto add_launch = [&](auto&& emit, int after_level) {
    tiles.clear();
    cnt.clear();
    emit([&](int k, int a, int b) {
      int32_t& sl = slot[(size_t)a * nb + b];
      if (sl < 0) {
        sl = (int32_t)tiles.size();
        tiles.push_back(a * nb + b);
        cnt.push_back(0);
      }
      (void)k;
      ++cnt[sl];
    });
    std::vector<int32_t> pos(tiles.size());
    int32_t base = (int32_t)klist.size(), acc = base;
    for (size_t p = 0; p < tiles.size(); ++p) {
      pos[p] = acc;
      acc += cnt[p];
      kptr.push_back(acc);
      lpairs.push_back(tiles[p] / nb);
      lpairs.push_back(tiles[p] % nb);
    }
    klist.resize(acc);
    emit([&](int k, int a, int b) { klist[pos[slot[(size_t)a * nb + b]]++] = k; });
    for (int32_t t : tiles) slot[(size_t)t] = -1;
    lv_pair_off.push_back((int64_t)lpairs.size() / 2);
    lv_launch_after.push_back(after_level);
  };
  for (int h0 = 0; h0 < n_levels; h0 += kLevelGroup) {
    const int h1 = std::min(n_levels, h0 + kLevelGroup);
    for (int h = h0; h < h1; ++h) {
      for (int k : by_level[h]) {
        cols.push_back(k);
        auto [rb, nr] = rows_of(k);
        for (int64_t a = 0; a < nr; ++a) {
          trows.push_back(rb[a]);
          tsteps.push_back(k);
        }
      }
      lv_col_off.push_back((int64_t)cols.size());
      lv_trsm_off.push_back((int64_t)trows.size());
      if (h + 1 < h1)   // thin: targets in columns of the group's later levels
        add_launch([&](auto&& visit) {
          for (int k : by_level[h]) {
            auto [rb, nr] = rows_of(k);
            for (int64_t a = 0; a < nr; ++a)
              for (int64_t b = 0; b <= a; ++b)
                if (height[rb[b]] < h1) visit(k, rb[a], rb[b]);
          }
        }, h);
    }
    // trailing: targets in columns beyond the group
    add_launch([&](auto&& visit) {
      for (int h = h0; h < h1; ++h)
        for (int k : by_level[h]) {
          auto [rb, nr] = rows_of(k);
          for (int64_t a = 0; a < nr; ++a)
            for (int64_t b = 0; b <= a; ++b)
              if (height[rb[b]] >= h1) visit(k, rb[a], rb[b]);
        }
    }, h1 - 1);
  }
  d_lv_cols.upload(cols, st);
  d_lv_trsm_rows.upload(trows.empty() ? std::vector<int32_t>(1, 0) : trows, st);
  d_lv_trsm_steps.upload(tsteps.empty() ? std::vector<int32_t>(1, 0) : tsteps, st);
  d_lv_pairs.upload(lpairs.empty() ? std::vector<int32_t>(2, 0) : lpairs, st);
  d_lv_kptr.upload(kptr, st);
  d_lv_k.upload(klist.empty() ? std::vector<int32_t>(1, 0) : klist, st);
}

template <typename T, int MODE>
static void factor_run(const FactorPlan& P, T* A, T* Ainv, const double* odiag, double drop_tol, double* pivrel,
                       DevErr* err, hipStream_t st, int32_t* failed) {
  const size_t lds = sizeof(T) * NB * LDA;
  const size_t mma_lds = MODE == 2 ? sizeof(T) * 4 * KCH * NB : 0;   // two stages of A and B chunks
  const unsigned threads = 64 * TileGeo<MODE>::WAVES;
  static bool attr_set = false;
  // diagonal blocks: recursive FP64 kernel in LDS or the register one (schedule)
  const bool rec_potrf = P.cfg.rec_potrf != 0;
  if (!attr_set) {
    HIP_CHECK(hipFuncSetAttribute((const void*)k_potrf<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    HIP_CHECK(hipFuncSetAttribute((const void*)k_potrf_rec<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(sizeof(double) * NB * LDA)));
    if (MODE == 2) {
      HIP_CHECK(hipFuncSetAttribute((const void*)k_trsm<T, MODE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)mma_lds));
      HIP_CHECK(hipFuncSetAttribute((const void*)k_syrk<T, MODE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)mma_lds));
      HIP_CHECK(hipFuncSetAttribute((const void*)k_syrk_lv<T, MODE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)mma_lds));
    }
    attr_set = true;
  }
  const int G = P.group;
  size_t li = 0;
  auto li_of = [&](const SyrkLaunch& L) { return (size_t)(&L - P.syrk.data()); };
  auto run_syrk = [&](const SyrkLaunch& L) {
    if (L.tiles > 0 && L.kb > 0)
      k_syrk<T, MODE><<<dim3((unsigned)L.tiles), dim3(threads), mma_lds, st>>>(
          P.d_desc.p, P.d_order.p, P.d_syrk_prefix.p + L.pre_off, P.nmat, L.kcol0, L.kb, L.b0, L.ncols, A,
          P.sparse ? P.d_syrk_pairs.p + 2 * P.syrk_off[li_of(L)] : nullptr, failed);
  };
  if (P.levels) {
    // elimination-tree levels: the block columns of a level are independent
    // (none updates another); per level one launch each for their diagonal
    // blocks and their column tiles, then the update launches due after it
    size_t u = 0;   // next update launch
    for (size_t h = 0; h + 1 < P.lv_col_off.size(); ++h) {
      const int64_t c0 = P.lv_col_off[h], nc = P.lv_col_off[h + 1] - c0;
      if (rec_potrf)
        k_potrf_rec<T><<<dim3((unsigned)nc), dim3(kRecThreads), sizeof(double) * NB * LDA, st>>>(
            P.d_desc.p, P.d_order.p, 0, A, Ainv, odiag, drop_tol, pivrel, err, failed, P.d_lv_cols.p + c0);
      else
        k_potrf<T><<<dim3((unsigned)nc), dim3(kPotrfThreads), lds, st>>>(P.d_desc.p, P.d_order.p, 0, A, Ainv, odiag,
                                                                        drop_tol, pivrel, err, failed,
                                                                        P.d_lv_cols.p + c0);
      const int64_t t0 = P.lv_trsm_off[h], nt = P.lv_trsm_off[h + 1] - t0;
      if (nt > 0)
        k_trsm<T, MODE><<<dim3((unsigned)nt), dim3(threads), mma_lds, st>>>(
            P.d_desc.p, P.d_order.p, P.d_prefix.p, 1, 0, A, Ainv, P.d_lv_trsm_rows.p + t0, failed,
            P.d_lv_trsm_steps.p + t0);
      for (; u < P.lv_launch_after.size() && P.lv_launch_after[u] == (int32_t)h; ++u) {
        const int64_t p0 = P.lv_pair_off[u], np = P.lv_pair_off[u + 1] - p0;
        if (np > 0)
          k_syrk_lv<T, MODE><<<dim3((unsigned)np), dim3(threads), mma_lds, st>>>(
              P.d_desc.p, P.d_order.p, A, P.d_lv_pairs.p + 2 * p0, P.d_lv_kptr.p + p0, P.d_lv_k.p, failed);
      }
    }
    HIP_CHECK(hipGetLastError());
    return;
  }
  for (int s0 = 0; s0 < P.max_blk; s0 += G) {
    for (int g = 0; g < G && s0 + g < P.max_blk; ++g) {
      const int s = s0 + g;
      run_syrk(P.syrk[li++]);   // column s from the group's earlier panels
      const int64_t* pt = P.d_prefix.p + P.pre_off[s];
      if (rec_potrf)
        k_potrf_rec<T><<<dim3(P.cnt[s]), dim3(kRecThreads), sizeof(double) * NB * LDA, st>>>(
            P.d_desc.p, P.d_order.p, s, A, Ainv, odiag, drop_tol, pivrel, err, failed, nullptr);
      else
        k_potrf<T><<<dim3(P.cnt[s]), dim3(kPotrfThreads), lds, st>>>(P.d_desc.p, P.d_order.p, s, A, Ainv, odiag,
                                                                       drop_tol, pivrel, err, failed, nullptr);
      if (P.trsm_tiles[s] > 0)
        k_trsm<T, MODE><<<dim3((unsigned)P.trsm_tiles[s]), dim3(threads), mma_lds, st>>>(
            P.d_desc.p, P.d_order.p, pt, P.cnt[s], s, A, Ainv, P.sparse ? P.d_trsm_rows.p + P.trsm_off[s] : nullptr,
            failed, nullptr);
    }
    run_syrk(P.syrk[li++]);
  }
  HIP_CHECK(hipGetLastError());
}

template <typename T>
static void factor_impl(const FactorPlan& P, T* A, T* Ainv, const double* odiag, double drop_tol, double* pivrel,
                        DevErr* err, hipStream_t st, int32_t* failed) {
  // tile mode of the schedule (the autotuner's choice, default measured on MI355X)
  const int mode = P.cfg.mode;
  if (mode == 0)
    factor_run<T, 0>(P, A, Ainv, odiag, drop_tol, pivrel, err, st, failed);
  else if (mode == 1)
    factor_run<T, 1>(P, A, Ainv, odiag, drop_tol, pivrel, err, st, failed);
  else
    factor_run<T, 2>(P, A, Ainv, odiag, drop_tol, pivrel, err, st, failed);
}

template <typename T>
static void mirror_impl(const FactorPlan& P, T* A, hipStream_t st);

template <typename T>
static void qblocks_impl(const FactorPlan& P, T* A, const T* Ainv, hipStream_t st);

void factor(const FactorPlan& P, double* A, double* Ainv, const double* odiag, double drop_tol, double* pivrel,
            DevErr* err, hipStream_t st, int32_t* failed, bool for_solves) {
  factor_impl<double>(P, A, Ainv, odiag, drop_tol, pivrel, err, st, failed);
  if (!for_solves) return;
  mirror_impl<double>(P, A, st);
  if (P.solve_form) qblocks_impl<double>(P, A, Ainv, st);
}
void factor(const FactorPlan& P, float* A, float* Ainv, const double* odiag, double drop_tol, double* pivrel,
            DevErr* err, hipStream_t st, int32_t* failed, bool for_solves) {
  factor_impl<float>(P, A, Ainv, odiag, drop_tol, pivrel, err, st, failed);
  if (!for_solves) return;
  mirror_impl<float>(P, A, st);
  if (P.solve_form) qblocks_impl<float>(P, A, Ainv, st);
}

// ------------------------------------------------------- triangular solves
// After factorisation the strictly lower blocks of L are mirrored into the
// (otherwise unused) strictly upper blocks, so U = L^T is stored
// column-major as well, and the diagonal-block inverses are kept both as
// inv(L_II) and inv(U_II) = inv(L_II)^T (second half of the inverse
// buffer).  A backward solve with U then reads memory exactly like a
// forward solve with L: block (I, J) at column J*NB+c, row I*NB+r.
//
// Sync-free blocked solves over the whole batch.  Work item = (matrix, block
// row); a workgroup takes the next item from a ticket counter, so every item
// it waits on was taken earlier by a running workgroup and no wait can
// deadlock.  Block-done flags carry an epoch number that is bumped before
// each solve, so flags never need clearing.  Every wait is bounded; on
// expiry the workgroup records GENEO_ESYNC and goes on, so the kernel always
// drains.
constexpr unsigned kSpinLimit = 1u << 24;

// U block (J, I) = L block (I, J)^T for every I > J, through LDS 64x64 tiles.
// strictly lower tile (ti > tj) of launch index u: the full triangle, or the
// listed pairs of a block-sparse matrix
__device__ inline void lower_tile(const int32_t* pairs, int64_t u, int64_t& ti, int64_t& tj) {
  if (pairs) {
    ti = pairs[2 * u];
    tj = pairs[2 * u + 1];
    return;
  }
  ti = (int64_t)((sqrt(8.0 * (double)u + 1.0) + 1.0) * 0.5);
  while (ti * (ti - 1) / 2 > u) --ti;
  while ((ti + 1) * ti / 2 <= u) ++ti;
  tj = u - ti * (ti - 1) / 2;
}

template <typename T>
__global__ __launch_bounds__(256) void k_mirror(const MatDesc* __restrict__ desc, const int32_t* __restrict__ order,
                                                const int64_t* __restrict__ prefix, int cnt, T* __restrict__ A,
                                                const int32_t* __restrict__ pairs) {
  __shared__ T tile[64][65];
  const int j = pairs ? 0 : find_mat(prefix, cnt, blockIdx.x);
  const MatDesc d = desc[order[j]];
  int64_t ti, tj;   // ti > tj
  lower_tile(pairs, pairs ? (int64_t)blockIdx.x : (int64_t)blockIdx.x - prefix[j], ti, tj);
  const int tid = threadIdx.x;
  for (int sub = 0; sub < 4; ++sub) {
    const int64_t r0 = ti * NB + 64 * (sub & 1), c0 = tj * NB + 64 * (sub >> 1);
    for (int idx = tid; idx < 64 * 64; idx += 256) {
      int r = idx & 63, c = idx >> 6;
      tile[c][r] = A[d.off + (c0 + c) * d.ld + r0 + r];
    }
    __syncthreads();
    // destination: row c0 + c, column r0 + r  (U = L^T)
    for (int idx = tid; idx < 64 * 64; idx += 256) {
      int c = idx & 63, r = idx >> 6;
      A[d.off + (r0 + r) * d.ld + c0 + c] = tile[c][r];
    }
    __syncthreads();
  }
}

// C[m][n] = sum_k Ar[k lda + m] Bt[n ldb + k] over K = NB (B read transposed),
// four waves of 64 x 64 as in mode 0
template <typename T>
__device__ inline void tile_mma_bt(const T* __restrict__ Ar, int64_t lda, const T* __restrict__ Bt, int64_t ldb,
                                   typename AccT<T>::type acc[4][4]) {
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
  Ar += 64 * TileGeo<0>::wr();
  Bt += 64 * TileGeo<0>::wc() * ldb;
  for (int kk = 0; kk < NB; kk += 4) {
    T af[4], bf[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      af[b] = Ar[(int64_t)(kk + lk) * lda + 16 * b + lr];
      bf[b] = Bt[(int64_t)(16 * b + lr) * ldb + kk + lk];
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mfma16(af[bi], bf[bj], acc[bi][bj]);
  }
}

// Solve form of the factor: every strictly lower block L(I,J) becomes
// inv(L_II) L(I,J) and every strictly upper block U(J,I) (the mirror)
// becomes inv(U_JJ) U(J,I), in place.  A block solve then reads
//   x_I = inv(L_II) b_I - sum_J [inv(L_II) L(I,J)] x_J,
// so once the last dependency arrives only one block product remains on the
// critical path.  One workgroup per pair of mirrored blocks.
template <typename T>
__global__ __launch_bounds__(256) void k_qblocks(const MatDesc* __restrict__ desc, const int32_t* __restrict__ order,
                                                 const int64_t* __restrict__ prefix, int cnt, T* __restrict__ A,
                                                 const T* __restrict__ Ainv, const int32_t* __restrict__ pairs) {
  const int j = pairs ? 0 : find_mat(prefix, cnt, blockIdx.x);
  const MatDesc d = desc[order[j]];
  int64_t ti, tj;   // ti > tj
  lower_tile(pairs, pairs ? (int64_t)blockIdx.x : (int64_t)blockIdx.x - prefix[j], ti, tj);
  using Acc = typename AccT<T>::type;
  Acc lo[4][4], up[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      lo[bi][bj] = Acc{0, 0, 0, 0};
      up[bi][bj] = Acc{0, 0, 0, 0};
    }
  // lower block (ti, tj): column-major at column tj*NB, row ti*NB
  T* L = A + d.off + tj * NB * d.ld + ti * NB;
  // upper block (tj, ti): column-major at column ti*NB, row tj*NB
  T* U = A + d.off + ti * NB * d.ld + tj * NB;
  const T* invL = Ainv + d.inv_off + ti * NB * NB;
  const T* invU = Ainv + d.inv_off + ((int64_t)d.nblk + tj) * NB * NB;
  // B(k, n) = block[k][n] = block[n * ld + k]
  tile_mma_bt<T>(invL, NB, L, d.ld, lo);
  tile_mma_bt<T>(invU, NB, U, d.ld, up);
  __syncthreads();   // both blocks fully read
  const int64_t off = (int64_t)(TileGeo<0>::WCOL * TileGeo<0>::wc()) * d.ld + 64 * TileGeo<0>::wr();
  tile_store<T, 4>(L + off, d.ld, lo);
  tile_store<T, 4>(U + off, d.ld, up);
}

__global__ void k_solve_begin(unsigned* sync) {
  sync[0] = 0;
  sync[1] = sync[1] + 1;
}

// Blocks of one matrix complete in order (block I publishes only after it
// has consumed every block it depends on), so once flag J is seen the
// frontier can be advanced over every later flag already set.  Polls are
// relaxed loads; a single agent-scope acquire fence follows each catch-up.
// Returns the first block (in the solve's direction) not yet known done.
__device__ inline int wait_frontier(const unsigned* flags, int J, int Jend, int step, unsigned epoch, DevErr* err) {
  unsigned spins = 0;
  while (__hip_atomic_load(flags + J, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
    if (++spins > kSpinLimit) {
      set_err(err, GENEO_ESYNC, -1, -1);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  int k = J + step;
  while (k != Jend && __hip_atomic_load(flags + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) k += step;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return k;
}

__device__ inline void publish(unsigned* flag, unsigned epoch) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __hip_atomic_store(flag, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline double load_coherent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_coherent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kTrsvThreads = 512;   // 4 column groups of 32: more loads in flight per block row

// Values of a single-right-hand-side solve travel without flags: the output
// vector is preset to a signalling-NaN pattern (arithmetic never produces
// it), each finished block stores its 128 values with agent-scope atomic
// stores, and a consumer polls the values themselves with agent-scope
// atomic loads until none is pending.  No fences are needed: each value is
// its own atomic object and nothing else written by the producer is read.
constexpr uint64_t kPending = 0x7FF4DEADBEEF0001ull;

__device__ inline double poll_value(const double* p, DevErr* err) {
  unsigned spins = 0;
  for (;;) {
    const double v = load_coherent(p);
    if (__builtin_bit_cast(uint64_t, v) != kPending) return v;
    if (++spins > kSpinLimit) {
      set_err(err, GENEO_ESYNC, -1, -1);
      return 0.0;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// marks the segments of the solve's blocks pending (one block per item)
__global__ void k_pending(const MatDesc* __restrict__ desc, const int32_t* __restrict__ items, double* x) {
  const int m = items[2 * blockIdx.x], I = items[2 * blockIdx.x + 1];
  x[desc[m].voff + (int64_t)I * NB + threadIdx.x] = __builtin_bit_cast(double, kPending);
}

// One triangular solve, single right-hand side: xout <- L^-1 xin
// (UPPER = false) or U^-1 xin (UPPER = true) on every matrix segment of the
// batch vector, with the factor in solve form (k_qblocks):
// x_I = c_I - sum_J Q(I,J) x_J, c_I = inv(D_II) b_I.  The workgroup computes
// c_I first; the blocks Q(I,J) are streamed one dependency ahead through
// two register buffers, so the block of a dependency is already in
// registers when its values land.
// Split rows (block-sparse plans, help_rng != nullptr): a helper item
// accumulates its dependency range and stores the partial sum to part; the
// row itself starts at row_lo[I] and adds its helpers' partials at the end.
template <typename T, bool UPPER>
__global__ __launch_bounds__(kTrsvThreads) void k_trsv(const MatDesc* __restrict__ desc,
                                                       const int32_t* __restrict__ items, const T* __restrict__ A,
                                                       const T* __restrict__ Ainv, const double* __restrict__ xin,
                                                       double* xout, unsigned* sync, DevErr* err,
                                                       const int32_t* __restrict__ dep_ptr,
                                                       const int32_t* __restrict__ dep,
                                                       const int32_t* __restrict__ help_rng,
                                                       const int32_t* __restrict__ row_lo,
                                                       const int32_t* __restrict__ row_help, double* part,
                                                       int qform) {
  constexpr int H = kTrsvThreads / NB;   // column groups
  constexpr int CW = NB / H;             // columns per group
  __shared__ double xs[NB];
  __shared__ double red[kTrsvThreads];
  __shared__ int s_t;
  const int tid = threadIdx.x;
  if (tid == 0) s_t = (int)atomicAdd(&sync[0], 1u);
  __syncthreads();
  const int mi = items[2 * s_t], I = items[2 * s_t + 1];
  const bool helper = mi < 0;
  const int hid = -1 - mi;
  const MatDesc d = desc[helper ? 0 : mi];
  const double* xi = xin + d.voff;
  double* xo = xout + d.voff;
  const int r = tid & (NB - 1), h = tid >> 7;
  // dependencies: forward J = 0..I-1 (increasing), backward J = nblk-1..I+1
  // (decreasing), or for a block-sparse factor the listed ones in that order
  const int J0 = UPPER ? d.nblk - 1 : 0, dir = UPPER ? -1 : 1;
  const int nd = dep ? dep_ptr[I + 1] - dep_ptr[I] : (UPPER ? d.nblk - 1 - I : I);
  const int32_t* dl = dep ? dep + dep_ptr[I] : nullptr;
  auto dep_at = [&](int e) { return dl ? dl[e] : J0 + dir * e; };
  auto load_block = [&](T* q, int J) {   // q[c] = Q(I,J)[r][CW h + c]
    const T* col = A + d.off + ((int64_t)J * NB + CW * h) * d.ld + (int64_t)I * NB + r;
#pragma unroll
    for (int c = 0; c < CW; ++c) q[c] = col[(int64_t)c * d.ld];
  };
  int e0 = 0, e1 = nd;
  if (help_rng) {
    if (helper) {
      e0 = help_rng[2 * hid];
      e1 = help_rng[2 * hid + 1];
    } else {
      e0 = row_lo[I];
    }
  }
  T qa[CW], qb[CW];
  if (e1 > e0) load_block(qa, dep_at(e0));
  double acc = 0.0;
  const T* inv = Ainv + d.inv_off + ((UPPER ? d.nblk : 0) + (int64_t)I) * NB * NB;
  if (!helper && qform) {
    // c_I = inv(D_II) b_I
    if (tid < NB) xs[tid] = xi[(int64_t)I * NB + tid];
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < CW; ++c) acc -= (double)inv[(int64_t)(CW * h + c) * NB + r] * xs[CW * h + c];
  }
  auto consume = [&](const T* q, int J) {
    __syncthreads();   // the previous values in xs are consumed
    if (tid < NB) xs[tid] = poll_value(xo + (int64_t)J * NB + tid, err);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CW; ++c) acc += (double)q[c] * xs[CW * h + c];
  };
  for (int e = e0; e < e1; e += 2) {
    if (e + 1 < e1) load_block(qb, dep_at(e + 1));
    consume(qa, dep_at(e));
    if (e + 1 < e1) {
      if (e + 2 < e1) load_block(qa, dep_at(e + 2));
      consume(qb, dep_at(e + 1));
    }
  }
  red[tid] = acc;
  __syncthreads();
  double v = 0.0;
  if (tid < NB) {
#pragma unroll
    for (int g = 0; g < H; ++g) v += red[g * NB + tid];
    if (helper) {
      store_coherent(part + (int64_t)hid * NB + tid, v);
    } else if (help_rng) {
      for (int hh = row_help[2 * I]; hh < row_help[2 * I + 1]; ++hh)
        v += poll_value(part + (int64_t)hh * NB + tid, err);
    }
  }
  if (helper) return;
  if (qform) {
    if (tid < NB) store_coherent(xo + (int64_t)I * NB + tid, -v);
    return;
  }
  // plain form: x_I = inv(D_II) (b_I - sum_J L(I,J) x_J)
  if (tid < NB) xs[tid] = xi[(int64_t)I * NB + tid] - v;
  __syncthreads();
  double a2 = 0.0;
#pragma unroll 8
  for (int c = 0; c < CW; ++c) a2 += (double)inv[(int64_t)(CW * h + c) * NB + r] * xs[CW * h + c];
  red[tid] = a2;
  __syncthreads();
  if (tid < NB) {
    double x = 0.0;
#pragma unroll
    for (int g = 0; g < H; ++g) x += red[g * NB + tid];
    store_coherent(xo + (int64_t)I * NB + tid, x);
  }
}

// marks n slots of 128 values pending
__global__ void k_pending_slots(double* p) {
  p[(int64_t)blockIdx.x * NB + threadIdx.x] = __builtin_bit_cast(double, kPending);
}

// Many right-hand sides (k <= KC columns): X <- L^-1 X or U^-1 X, X in block
// batch layout (matrix m's block at xoff = voff*KC... given by xstride: the
// block of matrix m starts at X + d.voff * ldk, column q at + q * d.ld).
template <typename T, bool UPPER, int KC>
__global__ __launch_bounds__(256) void k_trsm_multi(const MatDesc* __restrict__ desc,
                                                    const int32_t* __restrict__ items, const T* __restrict__ A,
                                                    const T* __restrict__ Ainv, double* X, int ldk, int k,
                                                    unsigned* sync, unsigned* flags, DevErr* err) {
  constexpr int H = KC / 2;
  __shared__ double xs[NB * KC];   // [c][q]
  __shared__ int s_t;
  __shared__ unsigned s_epoch;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_t = (int)atomicAdd(&sync[0], 1u);
    s_epoch = __hip_atomic_load(&sync[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  const int m = items[2 * s_t], I = items[2 * s_t + 1];
  const unsigned epoch = s_epoch;
  const MatDesc d = desc[m];
  double* Xm = X + d.voff * (int64_t)ldk;
  const int r = tid & (NB - 1), g = tid >> 7;
  double acc[H];
  // acc = -inv(D_II) B_I first (solve form of the factor, see k_qblocks)
  for (int idx = tid; idx < NB * KC; idx += 256) {
    int rr = idx & (NB - 1), q = idx >> 7;
    xs[rr * KC + q] = q < k ? Xm[(int64_t)q * d.ld + (int64_t)I * NB + rr] : 0.0;
  }
  __syncthreads();
  {
    const T* inv = Ainv + d.inv_off + ((UPPER ? d.nblk : 0) + (int64_t)I) * NB * NB;
#pragma unroll
    for (int q = 0; q < H; ++q) acc[q] = 0.0;
    for (int c = 0; c < NB; ++c) {
      const double l = (double)inv[(int64_t)c * NB + r];
#pragma unroll
      for (int q = 0; q < H; ++q) acc[q] -= l * xs[c * KC + g * H + q];
    }
  }
  __syncthreads();
  __shared__ int s_front;
  const int J0 = UPPER ? d.nblk - 1 : 0, Jend = UPPER ? I : I, dir = UPPER ? -1 : 1;
  if (tid == 0) s_front = J0;
  for (int J = J0; J != Jend; J += dir) {
    if (tid == 0 && J == s_front) s_front = wait_frontier(flags + d.flag_off, J, Jend, dir, epoch, err);
    __syncthreads();
    for (int idx = tid; idx < NB * KC; idx += 256) {
      int rr = idx & (NB - 1), q = idx >> 7;
      xs[rr * KC + q] = q < k ? load_coherent(Xm + (int64_t)q * d.ld + (int64_t)J * NB + rr) : 0.0;
    }
    __syncthreads();
    const T* col = A + d.off + (int64_t)J * NB * d.ld + (int64_t)I * NB + r;
    for (int c = 0; c < NB; ++c) {
      const double l = (double)col[(int64_t)c * d.ld];
#pragma unroll
      for (int q = 0; q < H; ++q) acc[q] += l * xs[c * KC + g * H + q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < H; ++q) {
    const int qq = g * H + q;
    if (qq < k) store_coherent(Xm + (int64_t)qq * d.ld + (int64_t)I * NB + r, -acc[q]);
  }
  __syncthreads();
  if (tid == 0) publish(flags + d.flag_off + I, epoch);
}

// FP64 many-right-hand-side solve on MFMA: the block products
// Q(I,J) X_J (128 x 128 by 128 x 32) run as v_mfma_f64_16x16x4 tiles, wave
// w owning rows 32w..32w+31 and all 32 columns; X_J is staged in LDS.
template <bool UPPER>
__global__ __launch_bounds__(256) void k_trsm_multi_mfma(const MatDesc* __restrict__ desc,
                                                         const int32_t* __restrict__ items,
                                                         const double* __restrict__ A,
                                                         const double* __restrict__ Ainv,
                                                         const double* __restrict__ Xin, double* Xout, int ldk, int k,
                                                         unsigned* sync, DevErr* err, int qform) {
  constexpr int KC = 32, XP = KC + 1;
  __shared__ double xs[NB * XP];   // [row][column]
  __shared__ int s_t;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  if (tid == 0) s_t = (int)atomicAdd(&sync[0], 1u);
  __syncthreads();
  const int m = items[2 * s_t], I = items[2 * s_t + 1];
  const MatDesc d = desc[m];
  const double* Xm = Xin + d.voff * (int64_t)ldk;   // right-hand sides
  double* Ym = Xout + d.voff * (int64_t)ldk;        // results (preset pending, polled by later blocks)
  d4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4_t{0, 0, 0, 0};
  // acc += Ablk (128 x 128, element (r, c) at Ablk[c * lda + r]) times xs (128 x 32)
  auto block_product = [&](const double* __restrict__ Ablk, int64_t lda) {
    const double* Ar = Ablk + 32 * w + lr;
    for (int kk = 0; kk < NB; kk += 4) {
      const double a0 = Ar[(int64_t)(kk + lk) * lda], a1 = Ar[(int64_t)(kk + lk) * lda + 16];
      const double b0 = xs[(kk + lk) * XP + lr], b1 = xs[(kk + lk) * XP + 16 + lr];
      acc[0][0] = mfma16(a0, b0, acc[0][0]);
      acc[0][1] = mfma16(a0, b1, acc[0][1]);
      acc[1][0] = mfma16(a1, b0, acc[1][0]);
      acc[1][1] = mfma16(a1, b1, acc[1][1]);
    }
  };
  const double* inv = Ainv + d.inv_off + ((UPPER ? d.nblk : 0) + (int64_t)I) * NB * NB;
  if (qform) {
    // -c_I = -inv(D_II) B_I
    for (int idx = tid; idx < NB * KC; idx += 256) {
      const int rr = idx & (NB - 1), q = idx >> 7;
      xs[rr * XP + q] = q < k ? -Xm[(int64_t)q * d.ld + (int64_t)I * NB + rr] : 0.0;
    }
    __syncthreads();
    block_product(inv, NB);
  }
  const int J0 = UPPER ? d.nblk - 1 : 0, Jend = I, dir = UPPER ? -1 : 1;
  constexpr int PER = NB * KC / 256;   // values of X_J per thread
  for (int J = J0; J != Jend; J += dir) {
    __syncthreads();   // every wave is done with the previous xs
    // all loads in flight at once; only values still pending are polled again
    double vals[PER];
    const double* yj = Ym + (int64_t)J * NB;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = tid + 256 * u, rr = idx & (NB - 1), q = idx >> 7;
      vals[u] = q < k ? load_coherent(yj + (int64_t)q * d.ld + rr) : 0.0;
    }
    for (unsigned spins = 0;; ++spins) {
      bool pend = false;
#pragma unroll
      for (int u = 0; u < PER; ++u) pend |= __builtin_bit_cast(uint64_t, vals[u]) == kPending;
      if (!pend) break;
      if (spins > kSpinLimit) {
        set_err(err, GENEO_ESYNC, -1, -1);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = tid + 256 * u, rr = idx & (NB - 1), q = idx >> 7;
        if (__builtin_bit_cast(uint64_t, vals[u]) == kPending) vals[u] = load_coherent(yj + (int64_t)q * d.ld + rr);
      }
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = tid + 256 * u, rr = idx & (NB - 1), q = idx >> 7;
      xs[rr * XP + q] = vals[u];
    }
    __syncthreads();
    block_product(A + d.off + (int64_t)J * NB * d.ld + (int64_t)I * NB, d.ld);
  }
  if (!qform) {
    // plain form: X_I = inv(D_II) (B_I - acc)
    __syncthreads();   // every wave is done with the last X_J in xs
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 32 * w + 16 * i + acc_row<double>(lane, v);
          const int col = 16 * j + lr;
          xs[row * XP + col] = col < k ? Xm[(int64_t)col * d.ld + (int64_t)I * NB + row] - acc[i][j][v] : 0.0;
          acc[i][j][v] = 0.0;
        }
    __syncthreads();
    block_product(inv, NB);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[i][j][v] = -acc[i][j][v];
  }
  // X_I = -acc
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 32 * w + 16 * i + acc_row<double>(lane, v);
        const int col = 16 * j + lr;
        if (col < k) store_coherent(Ym + (int64_t)col * d.ld + (int64_t)I * NB + row, -acc[i][j][v]);
      }
}

// marks the k columns of the solve's blocks pending (many right-hand sides)
__global__ void k_pending_multi(const MatDesc* __restrict__ desc, const int32_t* __restrict__ items, double* X,
                                int ldk, int k) {
  const int m = items[2 * blockIdx.x], I = items[2 * blockIdx.x + 1];
  const MatDesc d = desc[m];
  for (int idx = threadIdx.x; idx < NB * k; idx += blockDim.x)
    X[d.voff * (int64_t)ldk + (int64_t)(idx >> 7) * d.ld + (int64_t)I * NB + (idx & (NB - 1))] =
        __builtin_bit_cast(double, kPending);
}

template <typename T>
static void mirror_impl(const FactorPlan& P, T* A, hipStream_t st) {
  if (P.mirror_tiles > 0)
    k_mirror<T><<<dim3((unsigned)P.mirror_tiles), dim3(256), 0, st>>>(P.d_desc.p, P.d_order.p, P.d_mirror_prefix.p,
                                                                      P.nmat, A, P.sparse ? P.d_lower_pairs.p : nullptr);
}

template <typename T>
static void qblocks_impl(const FactorPlan& P, T* A, const T* Ainv, hipStream_t st) {
  if (P.mirror_tiles > 0)
    k_qblocks<T><<<dim3((unsigned)P.mirror_tiles), dim3(256), 0, st>>>(P.d_desc.p, P.d_order.p, P.d_mirror_prefix.p,
                                                                       P.nmat, A, Ainv,
                                                                       P.sparse ? P.d_lower_pairs.p : nullptr);
  HIP_CHECK(hipGetLastError());
}

template <typename T>
static void solve_impl(const FactorPlan& P, const T* A, const T* Ainv, double* x, unsigned* sync, DevErr* err,
                       hipStream_t st) {
  if (P.n_items == 0) return;
  double* y = P.d_y.p;   // forward result, backward input
  const unsigned ni = (unsigned)P.n_items;
  for (int dir = 0; dir < 2; ++dir) {
    const bool split = P.sparse;
    const int32_t* items = split ? P.d_sitems[dir].p : (dir == 0 ? P.d_items_fwd.p : P.d_items_bwd.p);
    const unsigned nw = split ? (unsigned)P.n_sitems[dir] : ni;
    const int32_t* dptr = P.sparse ? (dir == 0 ? P.d_dep_fwd_ptr.p : P.d_dep_bwd_ptr.p) : nullptr;
    const int32_t* dl = P.sparse ? (dir == 0 ? P.d_dep_fwd.p : P.d_dep_bwd.p) : nullptr;
    const int32_t* hr = split ? P.d_help_rng[dir].p : nullptr;
    const int32_t* rlo = split ? P.d_row_lo[dir].p : nullptr;
    const int32_t* rh = split ? P.d_row_help[dir].p : nullptr;
    double* xin = dir == 0 ? x : y;
    double* xout = dir == 0 ? y : x;
    k_pending<<<ni, NB, 0, st>>>(P.d_desc.p, P.d_items_fwd.p, xout);
    if (split && P.n_help[dir] > 0) k_pending_slots<<<(unsigned)P.n_help[dir], NB, 0, st>>>(P.d_part.p);
    k_solve_begin<<<1, 1, 0, st>>>(sync);
    if (dir == 0)
      k_trsv<T, false><<<nw, dim3(kTrsvThreads), 0, st>>>(P.d_desc.p, items, A, Ainv, xin, xout, sync, err, dptr, dl,
                                                           hr, rlo, rh, P.d_part.p, P.solve_form ? 1 : 0);
    else
      k_trsv<T, true><<<nw, dim3(kTrsvThreads), 0, st>>>(P.d_desc.p, items, A, Ainv, xin, xout, sync, err, dptr, dl,
                                                          hr, rlo, rh, P.d_part.p, P.solve_form ? 1 : 0);
  }
  HIP_CHECK(hipGetLastError());
}

template <typename T>
static void solve_multi_impl(const FactorPlan& P, const T* A, const T* Ainv, double* X, int ldk, int k,
                             unsigned* sync, unsigned* flags, DevErr* err, hipStream_t st) {
  if (P.n_items == 0 || k == 0) return;
  if (k > 32) throw Error(GENEO_EUNSUPPORTED, "more than 32 right-hand sides");
  k_solve_begin<<<1, 1, 0, st>>>(sync);
  k_trsm_multi<T, false, 32><<<dim3((unsigned)P.n_items), dim3(256), 0, st>>>(P.d_desc.p, P.d_items_fwd.p, A, Ainv,
                                                                              X, ldk, k, sync, flags, err);
  k_solve_begin<<<1, 1, 0, st>>>(sync);
  k_trsm_multi<T, true, 32><<<dim3((unsigned)P.n_items), dim3(256), 0, st>>>(P.d_desc.p, P.d_items_bwd.p, A, Ainv,
                                                                             X, ldk, k, sync, flags, err);
  HIP_CHECK(hipGetLastError());
}

void mirror(const FactorPlan& P, double* A, hipStream_t st) { mirror_impl<double>(P, A, st); }
void mirror(const FactorPlan& P, float* A, hipStream_t st) { mirror_impl<float>(P, A, st); }

void solve(const FactorPlan& P, const double* A, const double* Ainv, double* x, unsigned* sync, DevErr* err,
           hipStream_t st) {
  solve_impl<double>(P, A, Ainv, x, sync, err, st);
}
void solve(const FactorPlan& P, const float* A, const float* Ainv, double* x, unsigned* sync, DevErr* err,
           hipStream_t st) {
  solve_impl<float>(P, A, Ainv, x, sync, err, st);
}
void solve_multi(const FactorPlan& P, const double* A, const double* Ainv, double* X, int ldk, int k,
                 unsigned* sync, unsigned* flags, DevErr* err, hipStream_t st) {
  static const bool valu = [] {
    const char* e = std::getenv("GENEO_TRSM_MULTI");
    return e && std::string(e) == "valu";
  }();
  if (valu) {
    if (!P.solve_form) throw Error(GENEO_EUNSUPPORTED, "VALU many-RHS solve needs a factor in solve form");
    solve_multi_impl<double>(P, A, Ainv, X, ldk, k, sync, flags, err, st);
    return;
  }
  if (P.n_items == 0 || k == 0) return;
  if (k > 32 || ldk < k) throw Error(GENEO_EUNSUPPORTED, "more than 32 right-hand sides");
  if (P.sparse) throw Error(GENEO_EUNSUPPORTED, "many right-hand sides on a block-sparse factor");
  // intermediate block (forward result, backward input), one per plan
  const int64_t need = P.d_y.n * (int64_t)ldk;
  if ((int64_t)P.d_ym.n < need) P.d_ym.alloc(need);
  double* Y = P.d_ym.p;
  const unsigned ni = (unsigned)P.n_items;
  const int qf = P.solve_form ? 1 : 0;
  k_pending_multi<<<ni, 256, 0, st>>>(P.d_desc.p, P.d_items_fwd.p, Y, ldk, k);
  k_solve_begin<<<1, 1, 0, st>>>(sync);
  k_trsm_multi_mfma<false><<<ni, 256, 0, st>>>(P.d_desc.p, P.d_items_fwd.p, A, Ainv, X, Y, ldk, k, sync, err, qf);
  k_pending_multi<<<ni, 256, 0, st>>>(P.d_desc.p, P.d_items_fwd.p, X, ldk, k);
  k_solve_begin<<<1, 1, 0, st>>>(sync);
  k_trsm_multi_mfma<true><<<ni, 256, 0, st>>>(P.d_desc.p, P.d_items_bwd.p, A, Ainv, Y, X, ldk, k, sync, err, qf);
  HIP_CHECK(hipGetLastError());
  (void)flags;
}
void solve_multi(const FactorPlan& P, const float* A, const float* Ainv, double* X, int ldk, int k,
                 unsigned* sync, unsigned* flags, DevErr* err, hipStream_t st) {
  if (!P.solve_form) throw Error(GENEO_EUNSUPPORTED, "FP32 many-RHS solve needs a factor in solve form");
  solve_multi_impl<float>(P, A, Ainv, X, ldk, k, sync, flags, err, st);
}

}  // namespace geneo
