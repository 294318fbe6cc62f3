// Local generalised eigenproblems of the GenEO coarse space, all subdomains
// at once (Section 3.2, GEVP "tauthresholdAS", eq. (eigAtildeBAS)):
//   Atilde_j V = lambda B_j V,  Atilde_j = (I - xi_j)^T D_j A_j D_j (I - xi_j),
//   B_j = A_j^Neu,  xi_j = G_j S_j^-1 G_j^T A_j,  S_j = G_j^T A_j G_j,
// keep lambda > tau (at most nev_max), coarse vectors D_j (I - xi_j) V.
//
// Solver: block LOBPCG for the largest eigenvalues, preconditioned with
// B_j^-1 (dense Cholesky of the Neumann matrix: with this preconditioner the
// iterates stay B-orthogonal to span(G_j), which is the lambda = 0
// eigenspace; the start block is B-orthogonally projected out of span(G_j)
// with H_j = G_j^T B_j G_j).  Rayleigh-Ritz in FP64 on [X, W, P] through
// an eigendecomposition of the B-Gram matrix (columns that are numerically
// dependent are dropped) followed by a Jacobi eigensolver, one workgroup per
// subdomain in LDS.  Residual of a Ritz pair: ||Atilde x - theta B x|| /
// (|theta| ||B x||).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <numeric>

#include "model.h"

namespace geneo {

static inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

__device__ inline int find_seg(const int64_t* __restrict__ off, int n, int64_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------ operators
// Neumann values: local nonzero k of subdomain j sums the element entries of
// its global slot whose tet lies in a cell of Omega_j.
__global__ void k_neumann_vals(int64_t nnz, int nsub, const int64_t* __restrict__ nnz_off,
                               const int32_t* __restrict__ lslot, const int32_t* __restrict__ cptr,
                               const int32_t* __restrict__ cidx, const double* __restrict__ elem,
                               const int32_t* __restrict__ tet_cell, const uint32_t* __restrict__ cellbits,
                               int64_t words, double* __restrict__ bval) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int j = find_seg(nnz_off, nsub, k);
  const uint32_t* bits = cellbits + (int64_t)j * words;
  const int32_t s = lslot[k];
  double acc = 0.0;
  for (int32_t c = cptr[s]; c < cptr[s + 1]; ++c) {
    const int32_t e = cidx[c];
    const int32_t cell = tet_cell[e / 36];
    if ((bits[cell >> 5] >> (cell & 31)) & 1u) acc += elem[e];
  }
  bval[k] = acc;
}

__global__ void k_gather_vals(int64_t nnz, const int32_t* __restrict__ lslot, const double* __restrict__ gval,
                              double* __restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < nnz) out[t] = gval[lslot[t]];
}

// N = G^T X : node block (p_pad rows per subdomain), one thread per (node row, column)
__global__ void k_gt(int64_t plen, int k, const int32_t* __restrict__ node_sub, const int64_t* __restrict__ poff,
                     const int32_t* __restrict__ pl, const int64_t* __restrict__ voff,
                     const int64_t* __restrict__ ne_off, const int32_t* __restrict__ ne_ptr,
                     const int32_t* __restrict__ ne_edge, const int8_t* __restrict__ ne_sign,
                     const double* __restrict__ X, double* __restrict__ N) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= plen * k) return;
  const int64_t b = idx % plen;
  const int q = (int)(idx / plen);
  const int j = node_sub[b];
  const int64_t a = b - poff[j];
  const int64_t pld = poff[j + 1] - poff[j];
  const int64_t ld = voff[j + 1] - voff[j];
  double acc = 0.0;
  if (a < pl[j]) {
    const int32_t* ptr = ne_ptr + ne_off[j];
    const double* x = X + voff[j] * k + (int64_t)q * ld;
    for (int32_t t = ptr[a]; t < ptr[a + 1]; ++t) acc += (double)ne_sign[t] * x[ne_edge[t]];
  }
  N[poff[j] * k + (int64_t)q * pld + a] = acc;
}

// out = [base -] scale .* (G N) : edge block; G row r = -node(na) + node(nb)
__global__ void k_g(int64_t len, int k, const int32_t* __restrict__ row_sub, const int64_t* __restrict__ voff,
                    const int32_t* __restrict__ nloc, const int64_t* __restrict__ poff,
                    const int32_t* __restrict__ ena, const int32_t* __restrict__ enb, const double* __restrict__ N,
                    const double* __restrict__ base, const double* __restrict__ scale, double* __restrict__ out) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= len * k) return;
  const int64_t b = idx % len;
  const int q = (int)(idx / len);
  const int j = row_sub[b];
  const int64_t r = b - voff[j];
  const int64_t ld = voff[j + 1] - voff[j];
  const int64_t pld = poff[j + 1] - poff[j];
  const int64_t o = voff[j] * k + (int64_t)q * ld + r;
  double v = 0.0;
  if (r < nloc[j]) {
    const double* n = N + poff[j] * k + (int64_t)q * pld;
    const int32_t a = ena[b], c = enb[b];
    if (a >= 0) v -= n[a];
    if (c >= 0) v += n[c];
  }
  double t = base ? base[o] - v : v;
  out[o] = scale ? t * scale[b] : t;
}

// R = AX - BX diag(theta) (into W); also per-(subdomain, column) squared norms of R and BX
// Shifts of column q of subdomain j's block (one workgroup per column):
// without LtX, theta = (Bx)^T (Ax) / ||Bx||^2, the shift that minimises
// ||Ax - theta Bx|| (no cancellation: Ax and Bx are nearly parallel);
// with LtX (the block L_B^T X, B = L_B L_B^T) the Rayleigh quotient
// x^T (A x) / ||L_B^T x||^2, whose denominator is a sum of squares (rounding
// relative to itself) where x^T (B x) cancels (B ill conditioned,
// x^T B x << ||B|| ||x||^2) and carries u ||B|| ||x||^2.
__global__ __launch_bounds__(256) void k_rq(int k, const int64_t* __restrict__ voff, const double* __restrict__ X,
                                            const double* __restrict__ AX, const double* __restrict__ BX,
                                            const double* __restrict__ LtX, double* __restrict__ theta) {
  const int j = blockIdx.x / k, q = blockIdx.x % k;
  const int64_t ld = voff[j + 1] - voff[j];
  const int64_t o = voff[j] * k + (int64_t)q * ld;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t r = threadIdx.x; r < ld; r += 256) {
    if (LtX) {
      const double y = LtX[o + r];
      s1 += X[o + r] * AX[o + r];
      s2 += y * y;
    } else {
      const double bx = BX[o + r];
      s1 += bx * AX[o + r];
      s2 += bx * bx;
    }
  }
  __shared__ double a1[256], a2[256];
  a1[threadIdx.x] = s1;
  a2[threadIdx.x] = s2;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      a1[threadIdx.x] += a1[threadIdx.x + st];
      a2[threadIdx.x] += a2[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && a2[0] > 0.0) theta[j * k + q] = a1[0] / a2[0];
}

// Y = L^T X on every subdomain (L: the lower Cholesky factor of the batched
// local matrices, column-major, ld = n_pad; only its lower triangle is read):
// Y[I-block rows, q] = sum over rows r >= 128 I of L[r, 128 I + i] X[r, q].
// One workgroup per (subdomain, 128-row block I), rows staged through LDS in
// chunks of 32.  blk[g] = (subdomain, I) of workgroup g.
constexpr int kLtChunk = 32;
__global__ __launch_bounds__(256) void k_ltx(int k, const MatDesc* __restrict__ desc,
                                             const int32_t* __restrict__ blk, const int64_t* __restrict__ voff,
                                             const double* __restrict__ L, const double* __restrict__ X,
                                             double* __restrict__ Y) {
  __shared__ double lt[kLtChunk][NB + 1];
  __shared__ double xt[kLtChunk][33];
  const int j = blk[2 * blockIdx.x], I = blk[2 * blockIdx.x + 1];
  const MatDesc d = desc[j];
  const int64_t ld = voff[j + 1] - voff[j];   // = d.ld
  const double* Xj = X + voff[j] * k;
  const int tid = threadIdx.x;
  const int i = tid & (NB - 1), qh = tid >> 7;   // column of the block column; half of the right-hand sides
  const int64_t c0 = (int64_t)I * NB;
  double acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = 0.0;
  // chunk r0: L[r0 .. r0 + 31, c0 .. c0 + 127] (lower triangle only) and
  // X[r0 .. r0 + 31, 0 .. k - 1], read into registers one chunk ahead of the
  // one staged in LDS, so the loads overlap the products
  constexpr int LPT = kLtChunk * NB / 256, XPT = kLtChunk * 32 / 256;
  double lreg[LPT], xreg[XPT];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      const int e = tid + 256 * u;
      const int rr = e & (kLtChunk - 1), cc = e >> 5;
      const int64_t r = r0 + rr, c = c0 + cc;
      lreg[u] = r >= c ? L[d.off + c * d.ld + r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < XPT; ++u) {
      const int e = tid + 256 * u;
      const int rr = e & (kLtChunk - 1), q = e >> 5;
      xreg[u] = q < k ? Xj[(int64_t)q * ld + r0 + rr] : 0.0;
    }
  };
  fetch(c0);
  for (int64_t r0 = c0; r0 < d.ld; r0 += kLtChunk) {
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      const int e = tid + 256 * u;
      lt[e & (kLtChunk - 1)][e >> 5] = lreg[u];
    }
#pragma unroll
    for (int u = 0; u < XPT; ++u) {
      const int e = tid + 256 * u;
      xt[e & (kLtChunk - 1)][e >> 5] = xreg[u];
    }
    __syncthreads();
    if (r0 + kLtChunk < d.ld) fetch(r0 + kLtChunk);
#pragma unroll 4
    for (int rr = 0; rr < kLtChunk; ++rr) {
      const double l = lt[rr][i];
#pragma unroll
      for (int t = 0; t < 16; ++t) acc[t] += l * xt[rr][2 * t + qh];
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int q = 2 * t + qh;
    if (q < k) Y[voff[j] * k + (int64_t)q * ld + c0 + i] = acc[t];
  }
}

__global__ __launch_bounds__(256) void k_residual(int k, const int64_t* __restrict__ voff, const double* __restrict__ AX,
                                                  const double* __restrict__ BX, const double* __restrict__ theta,
                                                  double* __restrict__ R, double* __restrict__ nrm,
                                                  double* __restrict__ R2) {
  const int j = blockIdx.x / k, q = blockIdx.x % k;
  const int64_t ld = voff[j + 1] - voff[j];
  const int64_t o = voff[j] * k + (int64_t)q * ld;
  const double th = theta[j * k + q];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t r = threadIdx.x; r < ld; r += 256) {
    const double bx = BX[o + r];
    const double v = AX[o + r] - th * bx;
    R[o + r] = v;
    if (R2) R2[o + r] = v;
    s1 += v * v;
    s2 += bx * bx;
  }
  __shared__ double a1[256], a2[256];
  a1[threadIdx.x] = s1;
  a2[threadIdx.x] = s2;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      a1[threadIdx.x] += a1[threadIdx.x + st];
      a2[threadIdx.x] += a2[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    nrm[2 * (j * k + q)] = a1[0];
    nrm[2 * (j * k + q) + 1] = a2[0];
  }
}

// Per column (j, q): eta[2 (j k + q)] = r^T W = r^T B^-1 r (R the residual
// block, W = B^-1 R) and eta[2 (j k + q) + 1] = x^T B x.
__global__ __launch_bounds__(256) void k_eta(int k, const int64_t* __restrict__ voff, const double* __restrict__ R,
                                             const double* __restrict__ W, const double* __restrict__ X,
                                             const double* __restrict__ BX, double* __restrict__ eta) {
  const int j = blockIdx.x / k, q = blockIdx.x % k;
  const int64_t ld = voff[j + 1] - voff[j];
  const int64_t o = voff[j] * k + (int64_t)q * ld;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t r = threadIdx.x; r < ld; r += 256) {
    s1 += R[o + r] * W[o + r];
    s2 += X[o + r] * BX[o + r];
  }
  __shared__ double a1[256], a2[256];
  a1[threadIdx.x] = s1;
  a2[threadIdx.x] = s2;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      a1[threadIdx.x] += a1[threadIdx.x + st];
      a2[threadIdx.x] += a2[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    eta[2 * (j * k + q)] = a1[0];
    eta[2 * (j * k + q) + 1] = a2[0];
  }
}

// Gram partials: for row range [r0, r0 + 512) of subdomain j,
//   GA[a][b] = sum_r L[r][a] RA[r][b],  GB[a][b] = sum_r L[r][a] RB[r][b]
// where the "left" block is [L0 L1 L2] (nl blocks of k columns) and the right
// blocks likewise.  Partials land in part[(chunk) * 2 m^2 ...].
// 32-row slices of the three blocks are staged in LDS (columns padded with
// zeros to mp = 16 ceil(m / 16)); the products run on v_mfma_f64_16x16x4,
// wave w owning output tiles w, w + 4, ... of both GA and GB (the L operand
// is shared by the two).
constexpr int kGramRows = 512, kGramSub = 32;

typedef double gd4_t __attribute__((ext_vector_type(4)));

// MAXT: output tiles per wave (1 for m <= 32, 7 for m <= 80); PER: staged
// entries per thread and block (32 mp / 256).  The next slice is fetched
// into registers while the current one runs on the MFMAs.
template <int MAXT, int PER>
__global__ __launch_bounds__(256) void k_gram(int k, int nl, const int64_t* __restrict__ voff,
                                              const int64_t* __restrict__ chunk_off, int nsub,
                                              const double* __restrict__ L0, const double* __restrict__ L1,
                                              const double* __restrict__ L2, const double* __restrict__ A0,
                                              const double* __restrict__ A1, const double* __restrict__ A2,
                                              const double* __restrict__ B0, const double* __restrict__ B1,
                                              const double* __restrict__ B2, double* __restrict__ part) {
  extern __shared__ double sm[];
  const int m = nl * k;
  const int nt = (m + 15) >> 4, mp = nt * 16;
  double* ls = sm;                          // [kGramSub][mp]
  double* as = ls + kGramSub * mp;
  double* bs = as + kGramSub * mp;
  const int j = find_seg(chunk_off, nsub, blockIdx.x);
  const int64_t chunk = blockIdx.x - chunk_off[j];
  const int64_t ld = voff[j + 1] - voff[j];
  const int64_t base = voff[j] * k;
  const int64_t rbeg = chunk * kGramRows, rend = min((int64_t)ld, rbeg + kGramRows);
  const double* Ls[3] = {L0, L1, L2};
  const double* As[3] = {A0, A1, A2};
  const double* Bs[3] = {B0, B1, B2};
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lr = lane & 15, lk = lane >> 4;
  const int ntt = nt * nt;
  // this thread's staged entries: slice row rr, column c (fixed per slice)
  int ublk[PER];
  int64_t uoff[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int idx = threadIdx.x + 256 * u, c = idx >> 5;
    const bool ok = idx < kGramSub * mp && c < m;
    const int bl = ok ? c / k : -1;
    ublk[u] = bl;
    uoff[u] = ok ? base + (int64_t)(c - bl * k) * ld + (idx & (kGramSub - 1)) : 0;
  }
  double pl[PER], pa[PER], pb[PER];
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = threadIdx.x + 256 * u;
      const bool ok = ublk[u] >= 0 && r0 + (idx & (kGramSub - 1)) < rend;
      pl[u] = ok ? Ls[ublk[u]][uoff[u] + r0] : 0.0;
      pa[u] = ok ? As[ublk[u]][uoff[u] + r0] : 0.0;
      pb[u] = ok ? Bs[ublk[u]][uoff[u] + r0] : 0.0;
    }
  };
  gd4_t accA[MAXT], accB[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) accA[t] = accB[t] = gd4_t{0, 0, 0, 0};
  fetch(rbeg);
  for (int64_t r0 = rbeg; r0 < rend; r0 += kGramSub) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = threadIdx.x + 256 * u;
      if (idx < kGramSub * mp) {
        const int o = (idx & (kGramSub - 1)) * mp + (idx >> 5);
        ls[o] = pl[u];
        as[o] = pa[u];
        bs[o] = pb[u];
      }
    }
    __syncthreads();
    if (r0 + kGramSub < rend) fetch(r0 + kGramSub);
#pragma unroll 2
    for (int kk = 0; kk < kGramSub; kk += 4) {
      const int ro = (kk + lk) * mp;
#pragma unroll
      for (int q = 0; q < MAXT; ++q) {
        const int t = w + 4 * q;
        if (t < ntt) {
          const int ta = t / nt, tb = t - ta * nt;
          const double l = ls[ro + 16 * ta + lr];
          accA[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(l, as[ro + 16 * tb + lr], accA[q], 0, 0, 0);
          accB[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(l, bs[ro + 16 * tb + lr], accB[q], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // lane holds D[16 ta + lk + 4 v][16 tb + lr]; out is column-major m x m
  const int mm = m * m;
  double* out = part + (int64_t)blockIdx.x * 2 * mm;
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    const int t = w + 4 * q;
    if (t < ntt) {
      const int ta = t / nt, tb = t - ta * nt;
      const int b = 16 * tb + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = 16 * ta + lk + 4 * v;
        if (a < m && b < m) {
          out[a + b * m] = accA[q][v];
          out[mm + a + b * m] = accB[q][v];
        }
      }
    }
  }
}

// sum the Gram partials of each subdomain in chunk order
__global__ void k_gram_reduce(int m, const int64_t* __restrict__ chunk_off, const double* __restrict__ part,
                              double* __restrict__ gram) {
  const int j = blockIdx.y;
  const int mm2 = 2 * m * m;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mm2) return;
  double acc = 0.0;
  for (int64_t c = chunk_off[j]; c < chunk_off[j + 1]; ++c) acc += part[c * mm2 + e];
  gram[(int64_t)j * mm2 + e] = acc;
}

// ---------------------------------------------------- Rayleigh-Ritz (LDS)
constexpr int kMaxM = 72;
constexpr int kRRThreads = 1024;   // threads of the large Rayleigh-Ritz workgroup (m <= kMaxM)
constexpr int kRRSmallM = 32;      // bases up to this size run on kRRSmallThreads threads
constexpr int kRRSmallThreads = 256;

// Jacobi eigendecomposition of the symmetric n x n matrix a (row-major, ld),
// eigenvectors in v; parallel round-robin ordering, all NT threads of the
// block.  Each round rotates ne/2 disjoint pairs (p, q) at once: one pass
// applies A <- J^T A J on the 2 x 2 blocks (rows of one pair, columns of
// another; one thread per block, rows rotated first, then columns) and
// V <- V J on the row pairs of V.  A thread owns the same items in every
// round (no divisions in the passes); with an odd ld the column walks hit
// distinct LDS banks.
template <int NT, int MAXM>
__device__ void jacobi_eig(double* a, double* v, int n, int ld, double* rot_c, double* rot_s, int* pp, int* qq,
                           double* red) {
  constexpr int kHalf = MAXM / 2;
  constexpr int kBlk = (kHalf * kHalf + NT - 1) / NT;
  constexpr int kVit = (kHalf * MAXM + NT - 1) / NT;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < n * n; idx += NT) v[(idx / n) * ld + idx % n] = (idx / n == idx % n) ? 1.0 : 0.0;
  const int ne = n + (n & 1);   // even number of slots; slot n (if odd) is a dummy
  const int half = ne / 2;
  int b_s1[kBlk], b_s2[kBlk], v_slot[kVit], v_row[kVit];
#pragma unroll
  for (int q = 0; q < kBlk; ++q) {
    const int e = tid + q * NT;
    b_s1[q] = e < half * half ? e / half : -1;
    b_s2[q] = e < half * half ? e % half : 0;
  }
#pragma unroll
  for (int q = 0; q < kVit; ++q) {
    const int e = tid + q * NT;
    v_slot[q] = e < half * n ? e / n : -1;
    v_row[q] = e < half * n ? e % n : 0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    // convergence: off-diagonal mass vs diagonal
    double off = 0.0, dia = 0.0;
    for (int idx = tid; idx < n * n; idx += NT) {
      const int i = idx / n, j = idx % n;
      const double x = a[i * ld + j];
      if (i == j) dia += x * x; else off += x * x;
    }
    red[tid] = off;
    red[NT + tid] = dia;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
      if (tid < s) {
        red[tid] += red[tid + s];
        red[NT + tid] += red[NT + tid + s];
      }
      __syncthreads();
    }
    const bool done = red[0] <= 1e-30 * red[NT] || red[0] == 0.0;
    __syncthreads();
    if (done) break;
    for (int round = 0; round < ne - 1; ++round) {
      if (tid < half) {
        int p, q;
        if (tid == 0) {
          p = round;
          q = ne - 1;
        } else {
          p = (round + tid) % (ne - 1);
          q = (round - tid + (ne - 1)) % (ne - 1);
        }
        if (p > q) { int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = a[p * ld + q];
          if (apq != 0.0) {
            const double tau = (a[q * ld + q] - a[p * ld + p]) / (2.0 * apq);
            const double t = tau >= 0.0 ? 1.0 / (tau + sqrt(1.0 + tau * tau)) : -1.0 / (-tau + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        pp[tid] = p;
        qq[tid] = q;
        rot_c[tid] = c;
        rot_s[tid] = s;
      }
      __syncthreads();
      // A <- J^T A J: block (rows p1, q1) x (columns p2, q2); the dummy slot
      // (q = n) has c = 1, s = 0 and no row or column
#pragma unroll
      for (int it = 0; it < kBlk; ++it) {
        const int s1 = b_s1[it];
        if (s1 < 0) continue;
        const int s2 = b_s2[it];
        const int p1 = pp[s1], q1 = qq[s1], p2 = pp[s2], q2 = qq[s2];
        const double c1 = rot_c[s1], sn1 = rot_s[s1], c2 = rot_c[s2], sn2 = rot_s[s2];
        const bool h1 = q1 < n, h2 = q2 < n;
        const double xpp = a[p1 * ld + p2];
        const double xpq = h2 ? a[p1 * ld + q2] : 0.0;
        const double xqp = h1 ? a[q1 * ld + p2] : 0.0;
        const double xqq = h1 && h2 ? a[q1 * ld + q2] : 0.0;
        const double rpp = c1 * xpp - sn1 * xqp, rqp = sn1 * xpp + c1 * xqp;
        const double rpq = c1 * xpq - sn1 * xqq, rqq = sn1 * xpq + c1 * xqq;
        a[p1 * ld + p2] = c2 * rpp - sn2 * rpq;
        if (h2) a[p1 * ld + q2] = sn2 * rpp + c2 * rpq;
        if (h1) {
          a[q1 * ld + p2] = c2 * rqp - sn2 * rqq;
          if (h2) a[q1 * ld + q2] = sn2 * rqp + c2 * rqq;
        }
      }
      // V <- V J
#pragma unroll
      for (int it = 0; it < kVit; ++it) {
        const int slot = v_slot[it];
        if (slot < 0) continue;
        const int p = pp[slot], q = qq[slot], row = v_row[it];
        if (q >= n) continue;
        const double c = rot_c[slot], s = rot_s[slot];
        const double x = v[row * ld + p], y = v[row * ld + q];
        v[row * ld + p] = c * x - s * y;
        v[row * ld + q] = s * x + c * y;
      }
      __syncthreads();
    }
  }
}

// One workgroup per subdomain: solve SA c = theta SB c on the m-dimensional
// basis, write the k largest theta (descending) and coefficients coef (m x k,
// column-major).  Inactive subdomains are skipped.
// svqb != 0: only B-orthonormalise: coef = diag(dsc) U (m x n2, zero columns
// up to k), theta untouched.
template <int NT, int MAXM>
__global__ __launch_bounds__(NT) void k_rayleigh_ritz(int m, int k, const double* __restrict__ gram,
                                                       const int32_t* __restrict__ active, double drop,
                                                       double* __restrict__ theta, double* __restrict__ coef,
                                                       int svqb) {
  const int j = blockIdx.x;
  if (active && !active[j]) return;
  constexpr int LD = MAXM + 1;   // LDS row pitch bound
  __shared__ double A[MAXM * LD], B[MAXM * LD], V[MAXM * LD];
  __shared__ double dsc[MAXM], lam[MAXM], rc[MAXM / 2 + 1], rs[MAXM / 2 + 1], red[2 * NT];
  __shared__ int pp[MAXM / 2 + 1], qq[MAXM / 2 + 1], keep[MAXM], order[MAXM];
  __shared__ int nk;
  const int tid = threadIdx.x;
  const int mm = m * m;
  const int ld = m | 1;   // odd row pitch: column walks hit distinct banks
  const double* GA = gram + (int64_t)j * 2 * mm;
  const double* GB = GA + mm;
  // symmetrise; diagonal scaling of the B-Gram
  for (int idx = tid; idx < mm; idx += NT) {
    const int a = idx % m, b = idx / m;
    A[a * ld + b] = 0.5 * (GA[a + b * m] + GA[b + a * m]);
    B[a * ld + b] = 0.5 * (GB[a + b * m] + GB[b + a * m]);
  }
  __syncthreads();
  if (tid < m) {
    const double d = B[tid * ld + tid];
    dsc[tid] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < mm; idx += NT) {
    const int a = idx / m, b = idx % m;
    A[a * ld + b] *= dsc[a] * dsc[b];
    B[a * ld + b] *= dsc[a] * dsc[b];
  }
  __syncthreads();
  // B-orthonormal coordinates U (m x n2, stored in B, row-major pitch ld):
  // Rayleigh-Ritz bases are B-orthonormal blocks by construction, so the
  // scaled B-Gram is the identity up to rounding and a Cholesky factor
  // B_kk = L L^T of its non-zero columns gives U = L^-T; a pivot below
  // `drop` (near dependence) falls back to the eigen-decomposition of B.
  __shared__ int s_fail;
  if (tid == 0) {
    int c = 0;
    if (!svqb)
      for (int i = 0; i < m; ++i)
        if (dsc[i] > 0.0) keep[c++] = i;
    nk = c;
    s_fail = svqb ? 1 : 0;
  }
  __syncthreads();
  int n2 = nk;
  if (!s_fail) {
    for (int idx = tid; idx < n2 * n2; idx += NT) {
      const int r = idx / n2, c = idx % n2;
      V[r * ld + c] = r >= c ? B[keep[r] * ld + keep[c]] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < n2; ++j) {
      if (tid == 0) {
        const double p = V[j * ld + j];
        if (!(p > drop)) s_fail = 1;
        V[j * ld + j] = p > 0.0 ? sqrt(p) : 1.0;
      }
      __syncthreads();
      if (s_fail) break;
      const double djj = V[j * ld + j];
      for (int i = j + 1 + tid; i < n2; i += NT) V[i * ld + j] /= djj;
      __syncthreads();
      const int t = n2 - j - 1;
      for (int idx = tid; idx < t * t; idx += NT) {
        const int i = j + 1 + idx / t, c = j + 1 + idx % t;
        if (i >= c) V[i * ld + c] -= V[i * ld + j] * V[c * ld + j];
      }
      __syncthreads();
    }
  }
  if (!s_fail) {
    // X = L^-1 (column c by thread c, forward substitution), U[keep[r]][c] = X[c][r]
    for (int idx = tid; idx < m * n2; idx += NT) B[(idx / n2) * ld + idx % n2] = 0.0;
    __syncthreads();
    if (tid < n2) {
      // thread r: column r of X, i.e. row keep[r] of U
      const int r = tid;
      double* urow = B + keep[r] * ld;
      for (int i = r; i < n2; ++i) {
        double sum = i == r ? 1.0 : 0.0;
        for (int t = r; t < i; ++t) sum -= V[i * ld + t] * urow[t];
        urow[i] = sum / V[i * ld + i];
      }
    }
    __syncthreads();
  }
  if (s_fail) {
    jacobi_eig<NT, MAXM>(B, V, m, ld, rc, rs, pp, qq, red);
    if (tid < m) lam[tid] = B[tid * ld + tid];
    __syncthreads();
    if (tid == 0) {
      double mx = 0.0;
      for (int i = 0; i < m; ++i) mx = fmax(mx, lam[i]);
      int c = 0;
      for (int i = 0; i < m; ++i)
        if (lam[i] > drop * mx) keep[c++] = i;
      nk = c;
    }
    __syncthreads();
    n2 = nk;
    // U = V[:, keep] / sqrt(lambda) stored in B (m x n2, row-major pitch ld)
    for (int idx = tid; idx < m * n2; idx += NT) {
      const int r = idx / n2, c = idx % n2;
      const int col = keep[c];
      B[r * ld + c] = V[r * ld + col] / sqrt(lam[col]);
    }
    __syncthreads();
  }
  if (svqb) {
    for (int idx = tid; idx < m * k; idx += NT) {
      const int r = idx % m, c = idx / m;
      coef[(int64_t)j * m * k + (int64_t)c * m + r] = c < n2 ? dsc[r] * B[r * ld + c] : 0.0;
    }
    return;
  }
  // V <- A U (m x n2), then A <- U^T V (n2 x n2)
  for (int idx = tid; idx < m * n2; idx += NT) {
    const int r = idx / n2, c = idx % n2;
    double s = 0.0;
    for (int t = 0; t < m; ++t) s += A[r * ld + t] * B[t * ld + c];
    V[r * ld + c] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < n2 * n2; idx += NT) {
    const int r = idx / n2, c = idx % n2;
    double s = 0.0;
    for (int t = 0; t < m; ++t) s += B[t * ld + r] * V[t * ld + c];
    A[r * ld + c] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < n2 * n2; idx += NT) {
    const int r = idx / n2, c = idx % n2;
    if (r < c) {
      const double s = 0.5 * (A[r * ld + c] + A[c * ld + r]);
      A[r * ld + c] = s;
      A[c * ld + r] = s;
    }
  }
  __syncthreads();
  jacobi_eig<NT, MAXM>(A, V, n2, ld, rc, rs, pp, qq, red);
  if (tid == 0) {
    for (int i = 0; i < n2; ++i) {
      lam[i] = A[i * ld + i];
      order[i] = i;
    }
    for (int i = 1; i < n2; ++i) {   // insertion sort, descending
      int o = order[i];
      int t = i - 1;
      while (t >= 0 && lam[order[t]] < lam[o]) {
        order[t + 1] = order[t];
        --t;
      }
      order[t + 1] = o;
    }
  }
  __syncthreads();
  // coef = diag(dsc) U Y[:, order[0..k)]  (m x k); missing columns -> 0
  for (int idx = tid; idx < m * k; idx += NT) {
    const int r = idx % m, c = idx / m;
    double s = 0.0;
    if (c < n2) {
      const int col = order[c];
      for (int t = 0; t < n2; ++t) s += B[r * ld + t] * V[t * ld + col];
      s *= dsc[r];
    }
    coef[(int64_t)j * m * k + (int64_t)c * m + r] = s;
  }
  if (tid < k) theta[j * k + tid] = tid < n2 ? lam[order[tid]] : -1e300;
}

// One Rayleigh-Ritz (or B-orthonormalisation) launch over the N subdomains:
// bases of up to kRRSmallM vectors on a quarter of the threads (shorter
// barriers, less LDS), larger ones (m <= kMaxM) on kRRThreads.
static void rayleigh_ritz(int N, int m, int k, const double* gram, const int32_t* active, double drop, double* theta,
                          double* coef, int svqb, hipStream_t st) {
  if (m < 1 || m > kMaxM || k > m) throw Error(GENEO_EUNSUPPORTED, "Rayleigh-Ritz basis size out of range");
  if (m <= kRRSmallM)
    k_rayleigh_ritz<kRRSmallThreads, kRRSmallM><<<N, kRRSmallThreads, 0, st>>>(m, k, gram, active, drop, theta, coef,
                                                                              svqb);
  else
    k_rayleigh_ritz<kRRThreads, kMaxM><<<N, kRRThreads, 0, st>>>(m, k, gram, active, drop, theta, coef, svqb);
}

// Block-batch products.  Segments start at multiples of 128 rows, so a
// workgroup of 128 rows lies in one subdomain: its coefficients are uniform
// (scalar loads).  Thread (row rr, half qh) keeps the 16 output columns
// 16 qh .. 16 qh + 15 of its row in registers and reads each input entry
// once, coalesced along the rows.
constexpr int kBR = NB;   // rows per workgroup

// out = [L0 L1 L2][:, cols from coefficient rows c0..m) * coef  (per subdomain, n_pad x k)
// i.e. out[r][q] = sum_{c = c0}^{m-1} Lblk(c)[r][c % k] * coef[c][q]; inactive: out = keep
__global__ __launch_bounds__(256) void k_combine(int64_t len, int k, int m, int c0, const int32_t* __restrict__ row_sub,
                                                 const int64_t* __restrict__ voff, const int32_t* __restrict__ active,
                                                 const double* __restrict__ L0, const double* __restrict__ L1,
                                                 const double* __restrict__ L2, const double* __restrict__ coef,
                                                 const double* __restrict__ keep_src, double* __restrict__ out) {
  const int64_t b0 = (int64_t)blockIdx.x * kBR;
  const int tid = threadIdx.x, rr = tid & (kBR - 1);
  const int qh = __builtin_amdgcn_readfirstlane(tid >> 7);
  const int j = row_sub[b0];
  const int64_t vj = voff[j], ld = voff[j + 1] - vj, r = b0 + rr - vj;
  double* ob = out + vj * k + r;
  if (active && !active[j]) {
    for (int qq = 0; qq < 16; ++qq) {
      const int q = 16 * qh + qq;
      if (q < k) ob[(int64_t)q * ld] = keep_src ? keep_src[vj * k + (int64_t)q * ld + r] : 0.0;
    }
    return;
  }
  const double* cf = coef + (int64_t)j * m * k + (int64_t)16 * qh * m;
  double acc[16];
#pragma unroll
  for (int qq = 0; qq < 16; ++qq) acc[qq] = 0.0;
  const double* L[3] = {L0, L1, L2};
  for (int blk = c0 / k; blk * k < m; ++blk) {
    const double* Lb = L[blk] + vj * k + r;
    for (int cc = blk * k < c0 ? c0 - blk * k : 0; cc < k; ++cc) {
      const int c = blk * k + cc;
      const double x = Lb[(int64_t)cc * ld];
#pragma unroll
      for (int qq = 0; qq < 16; ++qq)
        if (16 * qh + qq < k) acc[qq] += x * cf[qq * m + c];
    }
  }
#pragma unroll
  for (int qq = 0; qq < 16; ++qq)
    if (16 * qh + qq < k) ob[(int64_t)(16 * qh + qq) * ld] = acc[qq];
}

// out -= X C  with C = Gram block (k x k per subdomain, from gram[j] rows 0..k of the A part)
__global__ __launch_bounds__(256) void k_sub_xc(int64_t len, int k, const int32_t* __restrict__ row_sub,
                                                const int64_t* __restrict__ voff, const double* __restrict__ X,
                                                const double* __restrict__ C, int ldc_stride,
                                                double* __restrict__ out) {
  const int64_t b0 = (int64_t)blockIdx.x * kBR;
  const int tid = threadIdx.x, rr = tid & (kBR - 1);
  const int qh = __builtin_amdgcn_readfirstlane(tid >> 7);
  const int j = row_sub[b0];
  const int64_t vj = voff[j], ld = voff[j + 1] - vj, r = b0 + rr - vj;
  const double* cj = C + (int64_t)j * ldc_stride + (int64_t)16 * qh * k;   // column-major k x k
  double acc[16];
#pragma unroll
  for (int qq = 0; qq < 16; ++qq) acc[qq] = 0.0;
  const double* xb = X + vj * k + r;
  for (int c = 0; c < k; ++c) {
    const double x = xb[(int64_t)c * ld];
#pragma unroll
    for (int qq = 0; qq < 16; ++qq)
      if (16 * qh + qq < k) acc[qq] += x * cj[qq * k + c];
  }
  double* ob = out + vj * k + r;
#pragma unroll
  for (int qq = 0; qq < 16; ++qq)
    if (16 * qh + qq < k) ob[(int64_t)(16 * qh + qq) * ld] -= acc[qq];
}

// random start block (counter-based splitmix64 -> standard normal via Box-Muller), pads 0
__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__global__ void k_random_block(int64_t len, int k, const int32_t* __restrict__ row_sub,
                               const int64_t* __restrict__ voff, const int32_t* __restrict__ nloc, uint64_t seed,
                               double* __restrict__ X) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= len * k) return;
  const int64_t b = idx % len;
  const int q = (int)(idx / len);
  const int j = row_sub[b];
  const int64_t r = b - voff[j];
  const int64_t ld = voff[j + 1] - voff[j];
  double v = 0.0;
  if (r < nloc[j]) {
    const uint64_t h1 = splitmix64(seed ^ splitmix64((uint64_t)idx * 2 + 1));
    const uint64_t h2 = splitmix64(h1 + 0x632BE59BD9B4E019ull);
    const double u1 = ((h1 >> 11) + 1.0) * (1.0 / 9007199254740993.0);
    const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
    v = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
  X[voff[j] * k + (int64_t)q * ld + r] = v;
}

__global__ void k_scale_rows(int64_t len, int k, const int32_t* __restrict__ row_sub,
                             const int64_t* __restrict__ voff, const double* __restrict__ s,
                             const double* __restrict__ X, double* __restrict__ out) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= len * k) return;
  const int64_t b = idx % len;
  const int q = (int)(idx / len);
  const int j = row_sub[b];
  const int64_t ld = voff[j + 1] - voff[j];
  const int64_t o = voff[j] * k + (int64_t)q * ld + (b - voff[j]);
  out[o] = s[b] * X[o];
}

// Rows of the subdomains with pick[j] = 1 are taken from the second block set:
// (X, AX, BX) <- (Xs, AXs, BXs) on those subdomains, all k columns.
__global__ void k_take_rows(int64_t len, int k, const int32_t* __restrict__ row_sub, const int64_t* __restrict__ voff,
                            const int32_t* __restrict__ pick, const double* __restrict__ Xs,
                            const double* __restrict__ AXs, const double* __restrict__ BXs, double* __restrict__ X,
                            double* __restrict__ AX, double* __restrict__ BX) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= len) return;
  const int j = row_sub[b];
  if (!pick[j]) return;
  const int64_t ld = voff[j + 1] - voff[j];
  const int64_t o = voff[j] * k + (b - voff[j]);
  for (int q = 0; q < k; ++q) {
    const int64_t i = o + (int64_t)q * ld;
    X[i] = Xs[i];
    AX[i] = AXs[i];
    BX[i] = BXs[i];
  }
}

// Knuth's two-sum: s + e = a + b exactly (contraction off so that no fused
// form changes it)
__device__ inline void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// dense p x p G^T M G (M = local A or B values), one thread per (subdomain, node row a).
// The entries are sums of M's entries with signs that cancel down to M G ~
// gamma (the gradients' mass part) for interior nodes; each is accumulated
// compensated (running sum in S, its rounding errors in Slo, folded by
// k_fold), so that S carries the rounding of its own value only.  An error of
// u |G|^T |M| |G| would move the kernel of the filtered operator off span(G)
// by a relative u |M| / gamma, which the eigensolver's projections out of
// span(G) then fight: its residuals stall (for gamma = 1e-6 near 1e-5).
__global__ void k_gmg(int64_t plen, const int32_t* __restrict__ node_sub, const int64_t* __restrict__ poff,
                      const int32_t* __restrict__ pl, const int64_t* __restrict__ ne_off,
                      const int32_t* __restrict__ ne_ptr, const int32_t* __restrict__ ne_edge,
                      const int8_t* __restrict__ ne_sign, const int64_t* __restrict__ voff,
                      const int64_t* __restrict__ rp_off, const int32_t* __restrict__ lrp,
                      const int32_t* __restrict__ lcol, const int32_t* __restrict__ lslot,
                      const double* __restrict__ gval, const double* __restrict__ lvals,
                      const int32_t* __restrict__ ena, const int32_t* __restrict__ enb,
                      const MatDesc* __restrict__ ndesc, double* __restrict__ S, double* __restrict__ Slo) {
  int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= plen) return;
  const int j = node_sub[b];
  const int64_t a = b - poff[j];
  if (a >= pl[j]) return;
  const MatDesc d = ndesc[j];
  const int32_t* ptr = ne_ptr + ne_off[j];
  const int32_t* rp = lrp + rp_off[j];
  for (int32_t t = ptr[a]; t < ptr[a + 1]; ++t) {
    const int32_t r = ne_edge[t];
    const double sa = (double)ne_sign[t];
    for (int32_t u = rp[r]; u < rp[r + 1]; ++u) {
      const double v = sa * (lvals ? lvals[u] : gval[lslot[u]]);
      const int64_t cb = voff[j] + lcol[u];
      const int32_t na = ena[cb], nbb = enb[cb];
      double hi, e;
      if (na >= 0) {
        const int64_t o = d.off + (int64_t)na * d.ld + a;
        two_sum(S[o], -v, hi, e);
        S[o] = hi;
        Slo[o] += e;
      }
      if (nbb >= 0) {
        const int64_t o = d.off + (int64_t)nbb * d.ld + a;
        two_sum(S[o], v, hi, e);
        S[o] = hi;
        Slo[o] += e;
      }
    }
  }
}

// S += Slo
__global__ void k_fold(int64_t n, double* __restrict__ S, const double* __restrict__ Slo) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) S[i] += Slo[i];
}

// C_j = A_j G_j, one thread per batch row (edge r of subdomain j): entry e of
// the row (node c_node[e]) sums +-A_j(r, c) over the columns c of the row
// with that node as their end (-: first, +: second), compensated (running
// sum in C, rounding errors in Clo; the row's entries belong to the thread).
// For a node whose whole star is in the row's pattern the sum cancels down
// to gamma (M G)(r, node); here it is formed once, from the matrix values,
// instead of cancelling again in every G^T A X and A G c of the eigensolver.
__global__ void k_c_vals(int64_t len, const int32_t* __restrict__ row_sub, const int64_t* __restrict__ voff,
                         const int32_t* __restrict__ nloc, const int64_t* __restrict__ rp_off,
                         const int32_t* __restrict__ lrp, const int32_t* __restrict__ lcol,
                         const double* __restrict__ aval, const int32_t* __restrict__ ena,
                         const int32_t* __restrict__ enb, const int64_t* __restrict__ c_rp,
                         const int32_t* __restrict__ c_node, double* __restrict__ C, double* __restrict__ Clo) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= len) return;
  const int j = row_sub[b];
  const int64_t vj = voff[j], r = b - vj;
  const int64_t e0 = c_rp[b], e1 = c_rp[b + 1];
  for (int64_t e = e0; e < e1; ++e) {
    C[e] = 0.0;
    Clo[e] = 0.0;
  }
  if (r >= nloc[j]) return;
  const int32_t* rp = lrp + rp_off[j];
  for (int32_t t = rp[r]; t < rp[r + 1]; ++t) {
    const double v = aval[t];
    const int64_t cb = vj + lcol[t];
    const int32_t nd[2] = {ena[cb], enb[cb]};
    for (int q = 0; q < 2; ++q) {
      if (nd[q] < 0) continue;
      int64_t e = e0;
      while (e < e1 && c_node[e] != nd[q]) ++e;
      if (e == e1) continue;   // unreachable: the pattern holds every end node of the row's columns
      double hi, lo;
      two_sum(C[e], q ? v : -v, hi, lo);
      C[e] = hi;
      Clo[e] += lo;
    }
  }
  for (int64_t e = e0; e < e1; ++e) C[e] += Clo[e];
}


__global__ void k_dense_scatter_vals(int64_t nnz, const int32_t* __restrict__ lrow, const int32_t* __restrict__ lcol,
                                     const int64_t* __restrict__ nnz_off, int nmat, const MatDesc* __restrict__ desc,
                                     const double* __restrict__ vals, double* __restrict__ A) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int j = find_seg(nnz_off, nmat, k);
  const MatDesc d = desc[j];
  A[d.off + (int64_t)lcol[k] * d.ld + lrow[k]] = vals[k];
}

// dense batch matrices: zero with ones on the padding diagonal; workgroup
// (c, m) writes column c of matrix m (grid (max ld, nmat))
__global__ __launch_bounds__(256) void k_fill_pad_identity(const MatDesc* __restrict__ desc, double* __restrict__ A) {
  const MatDesc d = desc[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= d.ld) return;
  const int64_t col = d.off + (int64_t)c * d.ld;
  for (int r = 2 * threadIdx.x; r < d.ld; r += 512)
    *reinterpret_cast<double2*>(A + col + r) =
        double2{(r == c && r >= d.n) ? 1.0 : 0.0, (r + 1 == c && r + 1 >= d.n) ? 1.0 : 0.0};
}
static dim3 fill_grid(const std::vector<MatDesc>& d) {
  int mx = 1;
  for (const auto& x : d) mx = std::max(mx, x.ld);
  return dim3((unsigned)mx, (unsigned)d.size());
}

// ------------------------------------------------------------- driver

struct EigWork {
  int N = 0, k = 0;
  int64_t len = 0, plen = 0;
  std::vector<int64_t> voff, poff;
  DevBuf<int32_t> row_sub, node_sub, pl, ne_ptr, ne_edge, ena, enb, lrp, nloc;
  DevBuf<int8_t> ne_sign;
  DevBuf<int64_t> voff_d, poff_d, ne_off, rp_off, chunk_off;
  DevBuf<double> bval, aval, LB, LBinv, S, Sinv, H, Hinv;
  FactorPlan node;
  DevBuf<unsigned> flags_node, flags_local;
  DevBuf<double> xrow;   // row-major copy of a block for the sparse products [len x 32] (gather path)
  // C_j = A_j G_j by edge rows (c_*) and by node rows (ct_*)
  DevBuf<int64_t> c_rp, ct_rp;
  DevBuf<int32_t> c_node, ct_row, ct_src;
  DevBuf<double> c_val, ct_val;
  DevBuf<double> nrow;   // row-major copy of a node block [plen x 32]
  std::vector<int64_t> h_c_rp, h_ct_rp;
  std::vector<int32_t> h_c_node, h_ct_row, h_ct_src;
  DevBuf<int32_t> lt_blk;   // (subdomain, 128-row block) pairs of the L^T X products
  int64_t nlt = 0;
  int64_t nchunks = 0;
  // LDS-staged sparse products: per 64-row block the sorted distinct local
  // columns of its rows, and per nonzero its position in that list
  DevBuf<int32_t> ublk_ptr, ucols;
  DevBuf<uint16_t> nz_slot;
  int u_max = 0;
  bool spmm_lds = false;
  std::vector<int32_t> h_ublk_ptr, h_ucols;   // host sources of the uploads (alive until the work ends)
  std::vector<uint16_t> h_nz_slot;
};

// Xt[b][q] = X block entry (row b, column q), rows padded to 32 columns;
// a workgroup transposes 64 rows through LDS so that both the column reads
// and the row writes are contiguous.
__global__ __launch_bounds__(256) void k_block_rowmajor(int64_t len, int k, const int32_t* __restrict__ row_sub,
                                                        const int64_t* __restrict__ voff,
                                                        const double* __restrict__ X, double* __restrict__ Xt) {
  __shared__ double tile[64][33];
  const int64_t b0 = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 32; e += 256) {
    const int q = e >> 6, rr = e & 63;
    const int64_t b = b0 + rr;
    double v = 0.0;
    if (b < len && q < k) {
      const int j = row_sub[b];
      v = X[voff[j] * k + (int64_t)q * (voff[j + 1] - voff[j]) + (b - voff[j])];
    }
    tile[rr][q] = v;
  }
  __syncthreads();
  for (int e = tid; e < 64 * 32; e += 256) {
    const int rr = e >> 5, q = e & 31;
    if (b0 + rr < len) Xt[(b0 + rr) * 32 + q] = tile[rr][q];
  }
}

// Workgroups are dealt to the 8 XCDs round-robin (id mod 8); this maps them
// to contiguous logical ranges per XCD, so that neighbouring row blocks (and
// the rows of X they gather) share one L2.
__device__ inline unsigned xcd_block() {
  const unsigned nb = gridDim.x, id = blockIdx.x, x = id & 7, per = nb >> 3, rem = nb & 7;
  return x * per + (x < rem ? x : rem) + (id >> 3);
}

// Y = [base -] scale .* (A_j X) with X given row-major (Xt, pitch 32).  A
// workgroup owns 64 consecutive batch rows; each wavefront takes two rows
// at a time, one per half-wave, with lane q on column q: a nonzero costs one
// coalesced 256-byte read of an Xt row.  Results go through LDS so that the
// column-major block layout of Y is written in 64-row runs.
__global__ __launch_bounds__(256) void k_spmm_rm(int64_t len, int k, const int32_t* __restrict__ row_sub,
                                                 const int64_t* __restrict__ voff, const int32_t* __restrict__ nloc,
                                                 const int64_t* __restrict__ rp_off, const int32_t* __restrict__ lrp,
                                                 const int32_t* __restrict__ lcol, const double* __restrict__ vals,
                                                 const double* __restrict__ Xt, const double* __restrict__ base,
                                                 const double* __restrict__ scale, double* __restrict__ Y) {
  __shared__ double tile[64][33];
  __shared__ int64_t s_o[64], s_ld[64], s_x[64];
  __shared__ int32_t s_t0[64], s_nnz[64];
  const int64_t b0 = (int64_t)xcd_block() * 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int q = lane & 31, hw = lane >> 5;
  // row metadata for the 64 rows, fetched once in parallel
  if (tid < 64) {
    const int64_t b = b0 + tid;
    int64_t o = -1, ldj = 0, xo = 0;
    int32_t t0 = 0, nnz = 0;
    if (b < len) {
      const int j = row_sub[b];
      const int64_t vj = voff[j], r = b - vj;
      o = vj * k + r;
      ldj = voff[j + 1] - vj;
      xo = vj * 32;
      if (r < nloc[j]) {
        const int32_t* rp = lrp + rp_off[j];
        t0 = rp[r];
        nnz = rp[r + 1] - t0;
      }
    }
    s_o[tid] = o;
    s_ld[tid] = ldj;
    s_x[tid] = xo;
    s_t0[tid] = t0;
    s_nnz[tid] = nnz;
  }
  __syncthreads();
  for (int i = 0; i < 8; ++i) {
    const int rl = 16 * w + 2 * i + hw;
    const int32_t t0 = s_t0[rl], nnz = s_nnz[rl];
    const double* xb = Xt + s_x[rl] + q;
    double acc = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    // the row's column indices and values are fetched one per lane and
    // broadcast inside the half-wave, so the gathers do not wait on them
    for (int cb = 0; cb < nnz; cb += 32) {
      int my_c = 0;
      double my_v = 0.0;
      if (cb + q < nnz) {
        my_c = lcol[t0 + cb + q];
        my_v = vals[t0 + cb + q];
      }
      const int n = min(32, nnz - cb);
      int t = 0;
      for (; t + 3 < n; t += 4) {
        const int c0 = __shfl(my_c, t, 32), c1 = __shfl(my_c, t + 1, 32);
        const int c2 = __shfl(my_c, t + 2, 32), c3 = __shfl(my_c, t + 3, 32);
        const double v0 = __shfl(my_v, t, 32), v1 = __shfl(my_v, t + 1, 32);
        const double v2 = __shfl(my_v, t + 2, 32), v3 = __shfl(my_v, t + 3, 32);
        acc += v0 * xb[(int64_t)c0 * 32];
        a1 += v1 * xb[(int64_t)c1 * 32];
        a2 += v2 * xb[(int64_t)c2 * 32];
        a3 += v3 * xb[(int64_t)c3 * 32];
      }
      for (; t < n; ++t) acc += __shfl(my_v, t, 32) * xb[(int64_t)__shfl(my_c, t, 32) * 32];
    }
    acc += a1 + a2 + a3;
    if (scale && nnz > 0) acc *= scale[b0 + rl];
    tile[rl][q] = acc;
  }
  __syncthreads();
  for (int e = tid; e < 64 * k; e += 256) {
    const int rl = e & 63, qq = e >> 6;
    const int64_t o = s_o[rl];
    if (o < 0) continue;
    const int64_t oq = o + (int64_t)qq * s_ld[rl];
    Y[oq] = base ? base[oq] - tile[rl][qq] : tile[rl][qq];
  }
}

// Products with C_j = A_j G_j, lane q on column q of a row-major block
// (pitch 32): NODE_ROWS: Y = C_j^T X, rows are the node rows of the node
// block (node_sub / poff, p_j live rows), the row's entries index edge rows
// of Xt (at voff); else Y = base - C_j N, rows are the edge rows of the edge
// block (row_sub / voff, n_j live rows), entries index node rows of Nt (at
// poff).  Workgroup = 64 rows, one per half-wave at a time; results staged
// through LDS and written in column runs, as in k_spmm_rm.
template <bool NODE_ROWS>
__global__ __launch_bounds__(256) void k_csr_rm(int64_t nrows, int k, const int32_t* __restrict__ rsub,
                                                const int64_t* __restrict__ roff, const int32_t* __restrict__ rlive,
                                                const int64_t* __restrict__ xoff, const int64_t* __restrict__ rp,
                                                const int32_t* __restrict__ cidx, const double* __restrict__ vals,
                                                const double* __restrict__ Xt, const double* __restrict__ base,
                                                double* __restrict__ Y) {
  __shared__ double tile[64][33];
  __shared__ int64_t s_o[64], s_ld[64], s_x[64], s_t0[64];
  __shared__ int32_t s_nnz[64];
  const int64_t b0 = (int64_t)xcd_block() * 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int q = lane & 31, hw = lane >> 5;
  if (tid < 64) {
    const int64_t b = b0 + tid;
    int64_t o = -1, ldj = 0, xo = 0, t0 = 0;
    int32_t nnz = 0;
    if (b < nrows) {
      const int j = rsub[b];
      const int64_t rj = roff[j], r = b - rj;
      o = rj * k + r;
      ldj = roff[j + 1] - rj;
      xo = xoff[j] * 32;
      if (r < rlive[j]) {
        t0 = rp[b];
        nnz = (int32_t)(rp[b + 1] - t0);
      }
    }
    s_o[tid] = o;
    s_ld[tid] = ldj;
    s_x[tid] = xo;
    s_t0[tid] = t0;
    s_nnz[tid] = nnz;
  }
  __syncthreads();
  for (int i = 0; i < 8; ++i) {
    const int rl = 16 * w + 2 * i + hw;
    const int64_t t0 = s_t0[rl];
    const int32_t nnz = s_nnz[rl];
    const double* xb = Xt + s_x[rl] + q;
    double acc = 0.0, a1 = 0.0;
    for (int cb = 0; cb < nnz; cb += 32) {
      int my_c = 0;
      double my_v = 0.0;
      if (cb + q < nnz) {
        my_c = cidx[t0 + cb + q];
        my_v = vals[t0 + cb + q];
      }
      const int n = min(32, nnz - cb);
      int t = 0;
      for (; t + 1 < n; t += 2) {
        const int c0 = __shfl(my_c, t, 32), c1 = __shfl(my_c, t + 1, 32);
        const double v0 = __shfl(my_v, t, 32), v1 = __shfl(my_v, t + 1, 32);
        acc += v0 * xb[(int64_t)c0 * 32];
        a1 += v1 * xb[(int64_t)c1 * 32];
      }
      if (t < n) acc += __shfl(my_v, t, 32) * xb[(int64_t)__shfl(my_c, t, 32) * 32];
    }
    tile[rl][q] = acc + a1;
  }
  __syncthreads();
  for (int e = tid; e < 64 * k; e += 256) {
    const int rl = e & 63, qq = e >> 6;
    const int64_t o = s_o[rl];
    if (o < 0) continue;
    const int64_t oq = o + (int64_t)qq * s_ld[rl];
    Y[oq] = NODE_ROWS ? tile[rl][qq] : base[oq] - tile[rl][qq];
  }
}

// Y = [base -] scale .* (A_j X), X in its column-major block layout.  A
// workgroup owns 64 consecutive batch rows (one subdomain: segments are
// multiples of 128 rows).  It first copies the X rows of the block's
// distinct columns into LDS (column by column, reading runs of the sorted
// column list), then each wavefront takes two rows at a time, one per
// half-wave, lane q on column q, every nonzero read from LDS; the sums run
// in the same order as the gather kernel's.  Results are kept in registers,
// then staged through the same LDS so that Y is written in 64-row runs.
constexpr int kSpmmThreads = 512;
constexpr int kSpmmRows = 64 / (kSpmmThreads / 32);   // rows per half-wave
__global__ __launch_bounds__(kSpmmThreads) void k_spmm_lds(int64_t len, int k, int pitch, const int32_t* __restrict__ row_sub,
                                                  const int64_t* __restrict__ voff, const int32_t* __restrict__ nloc,
                                                  const int64_t* __restrict__ rp_off, const int32_t* __restrict__ lrp,
                                                  const uint16_t* __restrict__ nz_slot,
                                                  const double* __restrict__ vals,
                                                  const int32_t* __restrict__ ublk_ptr,
                                                  const int32_t* __restrict__ ucols, const double* __restrict__ X,
                                                  const double* __restrict__ base, const double* __restrict__ scale,
                                                  double* __restrict__ Y) {
  extern __shared__ double xs[];   // [U * pitch], later the 64 x 33 output tile
  __shared__ int32_t s_t0[64], s_nnz[64];
  const int64_t blk = (int64_t)xcd_block();
  const int64_t b0 = blk * 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int q = lane & 31, hw = lane >> 5;
  const int j = row_sub[b0];
  const int64_t vj = voff[j], ldj = voff[j + 1] - vj, r0 = b0 - vj;
  const double* Xj = X + vj * k;
  const int u0 = ublk_ptr[blk], U = ublk_ptr[blk + 1] - u0;
  {
    // at most kSpmmThreads distinct columns; eight columns of X in flight per row
    const bool hA = tid < U;
    const int64_t cA = hA ? ucols[u0 + tid] : 0;
    for (int c0 = 0; c0 < k; c0 += 8) {
      double va[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) va[i] = hA && c0 + i < k ? Xj[(int64_t)(c0 + i) * ldj + cA] : 0.0;
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (hA && c0 + i < k) xs[tid * pitch + c0 + i] = va[i];
    }
  }
  if (tid < 64) {
    int32_t t0 = 0, nnz = 0;
    const int64_t r = r0 + tid;
    if (r < nloc[j]) {
      const int32_t* rp = lrp + rp_off[j];
      t0 = rp[r];
      nnz = rp[r + 1] - t0;
    }
    s_t0[tid] = t0;
    s_nnz[tid] = nnz;
  }
  __syncthreads();
  const bool live = q < k;
  double res[kSpmmRows];
#pragma unroll
  for (int i = 0; i < kSpmmRows; ++i) {
    const int rl = 2 * kSpmmRows * w + 2 * i + hw;
    const int32_t t0 = s_t0[rl], nnz = s_nnz[rl];
    double acc = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int cb = 0; cb < nnz; cb += 32) {
      int my_s = 0;
      double my_v = 0.0;
      if (cb + q < nnz) {
        my_s = nz_slot[t0 + cb + q];
        my_v = vals[t0 + cb + q];
      }
      const int n = min(32, nnz - cb);
      int t = 0;
      for (; t + 3 < n; t += 4) {
        const int c0 = __shfl(my_s, t, 32), c1 = __shfl(my_s, t + 1, 32);
        const int c2 = __shfl(my_s, t + 2, 32), c3 = __shfl(my_s, t + 3, 32);
        const double v0 = __shfl(my_v, t, 32), v1 = __shfl(my_v, t + 1, 32);
        const double v2 = __shfl(my_v, t + 2, 32), v3 = __shfl(my_v, t + 3, 32);
        if (live) {
          acc += v0 * xs[c0 * pitch + q];
          a1 += v1 * xs[c1 * pitch + q];
          a2 += v2 * xs[c2 * pitch + q];
          a3 += v3 * xs[c3 * pitch + q];
        }
      }
      for (; t < n; ++t) {
        const int c0 = __shfl(my_s, t, 32);
        const double v0 = __shfl(my_v, t, 32);
        if (live) acc += v0 * xs[c0 * pitch + q];
      }
    }
    acc += a1 + a2 + a3;
    if (scale && nnz > 0) acc *= scale[b0 + rl];
    res[i] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kSpmmRows; ++i) xs[(2 * kSpmmRows * w + 2 * i + hw) * 33 + q] = res[i];
  __syncthreads();
  for (int e = tid; e < 64 * k; e += kSpmmThreads) {
    const int rl = e & 63, qq = e >> 6;
    if (b0 + rl >= len) continue;
    const int64_t oq = vj * k + (int64_t)qq * ldj + r0 + rl;
    Y[oq] = base ? base[oq] - xs[rl * 33 + qq] : xs[rl * 33 + qq];
  }
}

// lvals == nullptr selects the local A_j values
static void spmm(const geneo_precond* pc, EigWork& w, const double* lvals, const double* X, const double* base,
                 const double* scale, double* Y, hipStream_t st) {
  if (w.spmm_lds) {
    const int pitch = w.k | 1;
    const size_t lds = sizeof(double) * std::max<size_t>((size_t)w.u_max * pitch, 64 * 33);
    k_spmm_lds<<<(unsigned)(w.len / 64), kSpmmThreads, lds, st>>>(w.len, w.k, pitch, w.row_sub.p, w.voff_d.p, w.nloc.p,
                                                         w.rp_off.p, w.lrp.p, w.nz_slot.p,
                                                         lvals ? lvals : w.aval.p, w.ublk_ptr.p, w.ucols.p, X, base,
                                                         scale, Y);
    return;
  }
  if (!w.xrow.p) w.xrow.alloc((size_t)w.len * 32);
  k_block_rowmajor<<<(unsigned)((w.len + 63) / 64), 256, 0, st>>>(w.len, w.k, w.row_sub.p, w.voff_d.p, X, w.xrow.p);
  k_spmm_rm<<<(unsigned)((w.len + 63) / 64), 256, 0, st>>>(w.len, w.k, w.row_sub.p, w.voff_d.p, w.nloc.p,
                                                          w.rp_off.p, w.lrp.p, pc->d_lcol.p,
                                                          lvals ? lvals : w.aval.p, w.xrow.p, base, scale, Y);
}
static void gt(EigWork& w, const double* X, double* Nn, hipStream_t st) {
  k_gt<<<nb256(w.plen * w.k), 256, 0, st>>>(w.plen, w.k, w.node_sub.p, w.poff_d.p, w.pl.p, w.voff_d.p, w.ne_off.p,
                                            w.ne_ptr.p, w.ne_edge.p, w.ne_sign.p, X, Nn);
}
// Nn = C_j^T X (X through its row-major copy)
static void ctx_mul(EigWork& w, const double* X, double* Nn, hipStream_t st) {
  if (!w.xrow.p) w.xrow.alloc((size_t)w.len * 32);
  k_block_rowmajor<<<(unsigned)((w.len + 63) / 64), 256, 0, st>>>(w.len, w.k, w.row_sub.p, w.voff_d.p, X, w.xrow.p);
  k_csr_rm<true><<<(unsigned)((w.plen + 63) / 64), 256, 0, st>>>(w.plen, w.k, w.node_sub.p, w.poff_d.p, w.pl.p,
                                                                 w.voff_d.p, w.ct_rp.p, w.ct_row.p, w.ct_val.p,
                                                                 w.xrow.p, nullptr, Nn);
}
// out = base - C_j Nn (Nn through its row-major copy)
static void cn_mul(EigWork& w, const double* Nn, const double* base, double* out, hipStream_t st) {
  if (!w.nrow.p) w.nrow.alloc((size_t)w.plen * 32);
  k_block_rowmajor<<<(unsigned)((w.plen + 63) / 64), 256, 0, st>>>(w.plen, w.k, w.node_sub.p, w.poff_d.p, Nn,
                                                                   w.nrow.p);
  k_csr_rm<false><<<(unsigned)((w.len + 63) / 64), 256, 0, st>>>(w.len, w.k, w.row_sub.p, w.voff_d.p, w.nloc.p,
                                                                 w.poff_d.p, w.c_rp.p, w.c_node.p, w.c_val.p,
                                                                 w.nrow.p, base, out);
}
static void gmul(EigWork& w, const double* Nn, const double* base, const double* scale, double* out, hipStream_t st) {
  k_g<<<nb256(w.len * w.k), 256, 0, st>>>(w.len, w.k, w.row_sub.p, w.voff_d.p, w.nloc.p, w.poff_d.p, w.ena.p, w.enb.p,
                                          Nn, base, scale, out);
}

// out = Atilde X  (tmp1, tmp2: edge blocks; nt: node block); with the
// classical pencil out = D A D X.  G^T A X and A G c go through C = A G
// (k_c_vals): formed as G^T (A X) and A (G c) their sums cancel (A G ~
// gamma M G for interior nodes while A's entries are of the curl-curl
// size) and the FP64 rounding, amplified by S^-1 ~ 1 / gamma, makes the
// operator non-linear at a level that stalls the eigensolver on strongly
// heterogeneous subdomains.
static void apply_atilde(geneo_ctx* ctx, const geneo_precond* pc, EigWork& w, const double* X, double* out,
                         double* t1, double* t2, double* nt) {
  hipStream_t st = ctx->stream;
  const double* D = pc->d_bpou.p;
  if (pc->opts.classical) {
    k_scale_rows<<<nb256(w.len * w.k), 256, 0, st>>>(w.len, w.k, w.row_sub.p, w.voff_d.p, D, X, t1);
    spmm(pc, w, nullptr, t1, nullptr, D, out, st);                   // D A D X
    return;
  }
  ctx_mul(w, X, nt, st);                                             // G^T A X = C^T X
  solve_multi(w.node, w.S.p, w.Sinv.p, nt, w.k, w.k, ctx->d_sync, w.flags_node.p, ctx->d_err, st);
  gmul(w, nt, X, D, t1, st);                                         // D (X - G S^-1 G^T A X)
  spmm(pc, w, nullptr, t1, nullptr, D, t2, st);                      // y = D A D u
  gt(w, t2, nt, st);
  solve_multi(w.node, w.S.p, w.Sinv.p, nt, w.k, w.k, ctx->d_sync, w.flags_node.p, ctx->d_err, st);
  cn_mul(w, nt, t2, out, st);                                        // y - A G S^-1 G^T y = y - C c
}

static void gram(EigWork& w, int nl, const double* L0, const double* L1, const double* L2, const double* A0,
                 const double* A1, const double* A2, const double* B0, const double* B1, const double* B2,
                 DevBuf<double>& part, DevBuf<double>& g, hipStream_t st) {
  const int m = nl * w.k;
  const size_t lds = sizeof(double) * 3 * kGramSub * ((m + 15) / 16 * 16);
  if (m > 16 * 5) throw Error(GENEO_EUNSUPPORTED, "Gram blocks wider than 80 columns");
  if (m <= 32)
    k_gram<1, 4><<<dim3((unsigned)w.nchunks), 256, lds, st>>>(w.k, nl, w.voff_d.p, w.chunk_off.p, w.N, L0, L1, L2,
                                                              A0, A1, A2, B0, B1, B2, part.p);
  else
    k_gram<7, 10><<<dim3((unsigned)w.nchunks), 256, lds, st>>>(w.k, nl, w.voff_d.p, w.chunk_off.p, w.N, L0, L1, L2,
                                                               A0, A1, A2, B0, B1, B2, part.p);
  dim3 grid((unsigned)((2 * m * m + 255) / 256), (unsigned)w.N);
  k_gram_reduce<<<grid, 256, 0, st>>>(m, w.chunk_off.p, part.p, g.p);
}

void solve_local_gevps(geneo_ctx* ctx, geneo_precond* pc) {
  HostClock hc;
  hc.tag = "gevp";
  hipStream_t st = ctx->stream;
  const geneo_system* s = pc->sys;
  const geneo_decomp* dec = pc->dec;
  const int N = pc->N;
  const int nev = pc->opts.nev_max;
  const int k = std::min(32, nev + std::max(0, pc->opts.lobpcg_guard));
  if (nev < 1) return;
  if (3 * k > kMaxM) throw Error(GENEO_EUNSUPPORTED, "nev_max + guard must be <= 24");
  EigWork w;
  w.N = N;
  w.k = k;
  w.voff = pc->voff;
  w.len = pc->batch_len;
  // ---- host structures: row -> subdomain, local rowptr, G incidence, node layout
  std::vector<int32_t> row_sub(w.len), nloc(N);
  std::vector<int64_t> rp_off(N + 1, 0);
  std::vector<int32_t> lrp;
  for (int j = 0; j < N; ++j) {
    for (int64_t b = w.voff[j]; b < w.voff[j + 1]; ++b) row_sub[b] = j;
    const int64_t n = dec->dofs_ptr[j + 1] - dec->dofs_ptr[j];
    nloc[j] = (int32_t)n;
    rp_off[j] = (int64_t)lrp.size();
    // local nnz of subdomain j are in row order, absolute indices from lnnz_off[j]
    lrp.resize(lrp.size() + n + 1);
    rp_off[j + 1] = (int64_t)lrp.size();
  }
  {
    const auto& hrow = pc->h_lrow;
    parallel_for(N, [&](int j) {   // each subdomain writes its own segment of lrp
      const int64_t n = nloc[j];
      int32_t* rp = lrp.data() + rp_off[j];
      for (int64_t r = 0; r <= n; ++r) rp[r] = (int32_t)pc->lnnz_off[j];
      for (int64_t t = pc->lnnz_off[j]; t < pc->lnnz_off[j + 1]; ++t) rp[hrow[t] + 1]++;
      for (int64_t r = 0; r < n; ++r) rp[r + 1] += rp[r] - (int32_t)pc->lnnz_off[j];
      // rp[r] now = lnnz_off[j] + count of rows < r  (absolute)
    });
  }
  {
    // distinct local columns of every 64-row block (the LDS-staged products
    // stage those rows of X once per block); host work only, planned before
    // the first upload, which waits for the local factorisation queued ahead
    const auto& hcol = pc->h_lcol;
    std::vector<uint16_t> slot(hcol.size(), 0);
    std::vector<std::vector<int32_t>> ub(N), ucnt(N);
    std::vector<int> submax(N, 0);
    parallel_for(N, [&](int j) {
      const int64_t n = nloc[j];
      const int64_t nb = (w.voff[j + 1] - w.voff[j]) / 64;
      std::vector<int32_t> pos(std::max<int64_t>(n, 1), -1), list;
      const int32_t* rp = lrp.data() + rp_off[j];
      for (int64_t bb = 0; bb < nb; ++bb) {
        list.clear();
        const int64_t ra = bb * 64, rb = std::min<int64_t>(n, ra + 64);
        for (int64_t r = ra; r < rb; ++r)
          for (int32_t t = rp[r]; t < rp[r + 1]; ++t)
            if (pos[hcol[t]] < 0) {
              pos[hcol[t]] = 0;
              list.push_back(hcol[t]);
            }
        std::sort(list.begin(), list.end());
        for (size_t u = 0; u < list.size(); ++u) pos[list[u]] = (int32_t)u;
        for (int64_t r = ra; r < rb; ++r)
          for (int32_t t = rp[r]; t < rp[r + 1]; ++t) slot[t] = (uint16_t)std::min(pos[hcol[t]], 65535);
        for (int32_t c : list) pos[c] = -1;
        ucnt[j].push_back((int32_t)list.size());
        ub[j].insert(ub[j].end(), list.begin(), list.end());
        submax[j] = std::max(submax[j], (int)list.size());
      }
    });
    w.u_max = N ? *std::max_element(submax.begin(), submax.end()) : 0;
    const int pitch = w.k | 1;
    // dynamic LDS of one workgroup stays within 64 KiB; wider blocks take the gather kernel
    w.spmm_lds = w.len % 64 == 0 && w.u_max <= kSpmmThreads && (size_t)w.u_max * pitch * sizeof(double) <= 65536;
    if (w.spmm_lds) {
      w.h_ublk_ptr.assign(1, 0);
      for (int j = 0; j < N; ++j) {
        for (int32_t c : ucnt[j]) w.h_ublk_ptr.push_back(w.h_ublk_ptr.back() + c);
        w.h_ucols.insert(w.h_ucols.end(), ub[j].begin(), ub[j].end());
      }
      w.h_nz_slot = std::move(slot);
    }
  }
  w.poff.assign(N + 1, 0);
  std::vector<int32_t> pl(N), node_sub, ne_ptr, ne_edge, ena(w.len, -1), enb(w.len, -1);
  std::vector<int8_t> ne_sign;
  std::vector<int64_t> ne_off(N + 1, 0);
  std::vector<MatDesc> ndesc(N);
  {
    int64_t off = 0, inv_off = 0, voff = 0;
    int32_t flag_off = 0;
    for (int j = 0; j < N; ++j) {
      const int64_t p = dec->gn_ptr[j + 1] - dec->gn_ptr[j];
      pl[j] = (int32_t)p;
      const int64_t pp = round_up(std::max<int64_t>(p, 1), NB);
      ndesc[j] = MatDesc{off, inv_off, -1, voff, (int32_t)pp, (int32_t)(pp / NB), flag_off, (int32_t)p};
      off += pp * pp;
      inv_off += 2 * pp * NB;
      w.poff[j] = voff;
      voff += pp;
      flag_off += (int32_t)(pp / NB);
    }
    // node -> incident local edges (sign -1 at the edge's first node, +1 at its
    // second), per subdomain in parallel, then packed in subdomain order
    std::vector<std::vector<int32_t>> ptr_j(N), edge_j(N);
    std::vector<std::vector<int8_t>> sign_j(N);
    parallel_for(N, [&](int j) {
      thread_local std::vector<int32_t> gl;   // free node -> local node, reset after use
      if ((int64_t)gl.size() < s->n_free_nodes) gl.assign(s->n_free_nodes, -1);
      const int64_t gb = dec->gn_ptr[j], ge = dec->gn_ptr[j + 1];
      const int64_t p = ge - gb;
      for (int64_t t = gb; t < ge; ++t) gl[dec->gnodes[t]] = (int32_t)(t - gb);
      std::vector<int32_t>& cnt = ptr_j[j];
      cnt.assign(p + 1, 0);
      const int64_t d0 = dec->dofs_ptr[j], d1 = dec->dofs_ptr[j + 1];
      for (int64_t r = d0; r < d1; ++r) {
        const int32_t lr = (int32_t)(r - d0);
        const int32_t e = s->free_edges[dec->dofs[r]];
        const int32_t fa = s->node_to_free[s->edges[2 * (int64_t)e]];
        const int32_t fb = s->node_to_free[s->edges[2 * (int64_t)e + 1]];
        const int32_t la = fa >= 0 ? gl[fa] : -1, lb = fb >= 0 ? gl[fb] : -1;
        ena[w.voff[j] + lr] = la;
        enb[w.voff[j] + lr] = lb;
        if (la >= 0) cnt[la + 1]++;
        if (lb >= 0) cnt[lb + 1]++;
      }
      for (int64_t a = 0; a < p; ++a) cnt[a + 1] += cnt[a];
      std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
      edge_j[j].resize(cnt[p]);
      sign_j[j].resize(cnt[p]);
      for (int64_t r = d0; r < d1; ++r) {   // in edge order, as each node's list
        const int32_t lr = (int32_t)(r - d0);
        const int32_t la = ena[w.voff[j] + lr], lb = enb[w.voff[j] + lr];
        if (la >= 0) {
          edge_j[j][pos[la]] = lr;
          sign_j[j][pos[la]++] = -1;
        }
        if (lb >= 0) {
          edge_j[j][pos[lb]] = lr;
          sign_j[j][pos[lb]++] = 1;
        }
      }
      for (int64_t t = gb; t < ge; ++t) gl[dec->gnodes[t]] = -1;
    });
    for (int j = 0; j < N; ++j) {
      ne_off[j] = (int64_t)ne_ptr.size();
      ne_ptr.insert(ne_ptr.end(), ptr_j[j].begin(), ptr_j[j].end());
      ne_edge.insert(ne_edge.end(), edge_j[j].begin(), edge_j[j].end());
      ne_sign.insert(ne_sign.end(), sign_j[j].begin(), sign_j[j].end());
    }
    w.poff[N] = voff;
    w.plen = voff;
    node_sub.resize(w.plen);
    for (int j = 0; j < N; ++j)
      for (int64_t b = w.poff[j]; b < w.poff[j + 1]; ++b) node_sub[b] = j;
    // edge offsets in ne_edge are per subdomain: ne_ptr indexes from ne_off-relative starts
    // (ne_ptr segment of subdomain j starts at ne_off[j] and its values index ne_edge
    //  relative to the first edge of the segment) -> make them absolute
    int64_t base = 0;
    for (int j = 0; j < N; ++j) {
      for (int64_t a = 0; a <= pl[j]; ++a) ne_ptr[ne_off[j] + a] += (int32_t)base;
      base += ne_ptr[ne_off[j] + pl[j]] - ne_ptr[ne_off[j]];
    }
    ne_off[N] = (int64_t)ne_ptr.size();
    w.node.build(ndesc, st);
    // plain form: S_j = G^T A_j G is ill conditioned for small gamma (2e8 at gamma = 1e-4), and
    // premultiplying the off-diagonal blocks by explicit diagonal-block inverses loses accuracy
    // the Rayleigh quotients of the filtered operator see
    w.node.solve_form = false;
    w.S.alloc(off);
    w.H.alloc(off);
    w.Sinv.alloc(inv_off);
    w.Hinv.alloc(inv_off);
    w.flags_node.alloc(flag_off);
    HIP_CHECK(hipMemsetAsync(w.flags_node.p, 0, sizeof(unsigned) * flag_off, st));
  }
  // ---- patterns of C_j = A_j G_j: the entries of edge row r are the distinct
  // end nodes of the row's columns; by node rows, the transpose (edge row,
  // entry index)
  {
    const auto& hcol = pc->h_lcol;
    std::vector<std::vector<int32_t>> rowlen(N), nodes(N), trow(N), tsrc(N);
    std::vector<std::vector<int64_t>> tpre(N);
    parallel_for(N, [&](int j) {
      const int64_t n = nloc[j], p = pl[j];
      const int32_t* rp = lrp.data() + rp_off[j];
      const int64_t vj = w.voff[j];
      auto& rl = rowlen[j];
      auto& nd = nodes[j];
      rl.assign(n, 0);
      std::vector<int32_t> cand;
      for (int64_t r = 0; r < n; ++r) {
        cand.clear();
        for (int32_t t = rp[r]; t < rp[r + 1]; ++t) {
          const int64_t cb = vj + hcol[t];
          if (ena[cb] >= 0) cand.push_back(ena[cb]);
          if (enb[cb] >= 0) cand.push_back(enb[cb]);
        }
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        rl[r] = (int32_t)cand.size();
        nd.insert(nd.end(), cand.begin(), cand.end());
      }
      auto& pre = tpre[j];
      pre.assign(p + 1, 0);
      for (int32_t a : nd) pre[a + 1]++;
      for (int64_t a = 0; a < p; ++a) pre[a + 1] += pre[a];
      trow[j].assign(nd.size(), 0);
      tsrc[j].assign(nd.size(), 0);
      std::vector<int64_t> f(pre.begin(), pre.end() - 1);
      int64_t e = 0;
      for (int64_t r = 0; r < n; ++r)
        for (int32_t q = 0; q < rl[r]; ++q, ++e) {
          const int32_t a = nd[e];
          trow[j][f[a]] = (int32_t)r;
          tsrc[j][f[a]++] = (int32_t)e;
        }
    });
    int64_t tot = 0;
    for (int j = 0; j < N; ++j) tot += (int64_t)nodes[j].size();
    if (tot >= (int64_t)INT32_MAX) throw Error(GENEO_EUNSUPPORTED, "pattern of A_j G_j beyond 2^31 entries");
    w.h_c_rp.assign(w.len + 1, 0);
    w.h_ct_rp.assign(w.plen + 1, 0);
    w.h_c_node.reserve(tot);
    w.h_ct_row.reserve(tot);
    w.h_ct_src.reserve(tot);
    int64_t e_base = 0;
    for (int j = 0; j < N; ++j) {
      const int64_t vj = w.voff[j];
      for (int64_t r = 0; r < nloc[j]; ++r) w.h_c_rp[vj + r + 1] = rowlen[j][r];
      for (int64_t a = 0; a < pl[j]; ++a) w.h_ct_rp[w.poff[j] + a + 1] = tpre[j][a + 1] - tpre[j][a];
      w.h_c_node.insert(w.h_c_node.end(), nodes[j].begin(), nodes[j].end());
      w.h_ct_row.insert(w.h_ct_row.end(), trow[j].begin(), trow[j].end());
      for (int32_t e : tsrc[j]) w.h_ct_src.push_back((int32_t)(e_base + e));
      e_base += (int64_t)nodes[j].size();
    }
    for (int64_t b = 0; b < w.len; ++b) w.h_c_rp[b + 1] += w.h_c_rp[b];
    for (int64_t b = 0; b < w.plen; ++b) w.h_ct_rp[b + 1] += w.h_ct_rp[b];
  }
  hc.mark("host planning");
  w.c_rp.upload(w.h_c_rp, st);
  w.c_node.upload(w.h_c_node, st);
  w.ct_rp.upload(w.h_ct_rp, st);
  w.ct_row.upload(w.h_ct_row, st);
  w.ct_src.upload(w.h_ct_src, st);
  w.row_sub.upload(row_sub, st);
  w.nloc.upload(nloc, st);
  w.rp_off.upload(rp_off, st);
  w.lrp.upload(lrp, st);
  if (w.spmm_lds) {
    w.ublk_ptr.upload(w.h_ublk_ptr, st);
    w.ucols.upload(w.h_ucols, st);
    w.nz_slot.upload(w.h_nz_slot, st);
  }
  w.voff_d.upload(w.voff, st);
  w.poff_d.upload(w.poff, st);
  w.pl.upload(pl, st);
  w.node_sub.upload(node_sub, st);
  w.ne_off.upload(ne_off, st);
  w.ne_ptr.upload(ne_ptr, st);
  w.ne_edge.upload(ne_edge, st);
  w.ne_sign.upload(ne_sign, st);
  w.ena.upload(ena, st);
  w.enb.upload(enb, st);
  hc.mark("uploads");
  std::vector<int64_t> chunk_off(N + 1, 0);
  for (int j = 0; j < N; ++j) chunk_off[j + 1] = chunk_off[j] + (w.voff[j + 1] - w.voff[j] + kGramRows - 1) / kGramRows;
  w.nchunks = chunk_off[N];
  w.chunk_off.upload(chunk_off, st);

  // ---- Neumann values, dense B_j, factor
  const int64_t lnnz = pc->lnnz_off[N];
  {
    const int64_t words = (s->n_cells + 31) / 32;
    std::vector<uint32_t> bits((size_t)words * N, 0u);
    for (int j = 0; j < N; ++j)
      for (int64_t t = dec->cells_ptr[j]; t < dec->cells_ptr[j + 1]; ++t) {
        const int32_t c = dec->cells[t];
        bits[(size_t)j * words + (c >> 5)] |= 1u << (c & 31);
      }
    DevBuf<uint32_t> dbits;
    dbits.upload(bits, st);
    w.bval.alloc(lnnz);
    w.aval.alloc(lnnz);
    k_gather_vals<<<nb256(lnnz), 256, 0, st>>>(lnnz, pc->d_lslot.p, s->d_val.p, w.aval.p);
    k_neumann_vals<<<nb256(lnnz), 256, 0, st>>>(lnnz, N, pc->d_lnnz_off.p, pc->d_lslot.p, s->d_contrib_ptr.p,
                                                 s->d_contrib.p, s->d_elem.p, s->d_tet_cell.p, dbits.p, words,
                                                 w.bval.p);
    // C_j = A_j G_j, then its values in node-row order
    const int64_t nc = (int64_t)w.h_c_node.size();
    w.c_val.alloc(std::max<int64_t>(nc, 1));
    w.ct_val.alloc(std::max<int64_t>(nc, 1));
    DevBuf<double> clo;
    clo.alloc(std::max<int64_t>(nc, 1));
    k_c_vals<<<nb256(w.len), 256, 0, st>>>(w.len, w.row_sub.p, w.voff_d.p, w.nloc.p, w.rp_off.p, w.lrp.p,
                                           pc->d_lcol.p, w.aval.p, w.ena.p, w.enb.p, w.c_rp.p, w.c_node.p,
                                           w.c_val.p, clo.p);
    if (nc) k_gather_vals<<<nb256(nc), 256, 0, st>>>(nc, w.ct_src.p, w.c_val.p, w.ct_val.p);
    HIP_CHECK(hipStreamSynchronize(st));
  }
  const auto& ld = pc->local.h_desc;
  const int64_t dense_total = ld.back().off + (int64_t)ld.back().ld * ld.back().ld;
  w.LB.alloc(dense_total);
  w.LBinv.alloc(pc->dLinv.n ? pc->dLinv.n : pc->fLinv.n);
  hc.mark("host plans");
  k_fill_pad_identity<<<fill_grid(ld), 256, 0, st>>>(pc->local.d_desc.p, w.LB.p);
  k_dense_scatter_vals<<<nb256(lnnz), 256, 0, st>>>(lnnz, pc->d_lrow.p, pc->d_lcol.p, pc->d_lnnz_off.p, N,
                                                     pc->local.d_desc.p, w.bval.p, w.LB.p);
  factor(pc->local, w.LB.p, w.LBinv.p, nullptr, 0.0, nullptr, ctx->d_err, st);
  {
    std::vector<int32_t> lb;
    for (int j = 0; j < N; ++j)
      for (int I = 0; I < ld[j].nblk; ++I) {
        lb.push_back(j);
        lb.push_back(I);
      }
    w.nlt = (int64_t)lb.size() / 2;
    w.lt_blk.upload(lb, st);
  }
  w.flags_local.alloc(pc->d_flags_local.n);
  HIP_CHECK(hipMemsetAsync(w.flags_local.p, 0, sizeof(unsigned) * pc->d_flags_local.n, st));

  // ---- S_j = G^T A_j G, H_j = G^T B_j G, factor
  {
    k_fill_pad_identity<<<fill_grid(ndesc), 256, 0, st>>>(w.node.d_desc.p, w.S.p);
    k_fill_pad_identity<<<fill_grid(ndesc), 256, 0, st>>>(w.node.d_desc.p, w.H.p);
    DevBuf<double> lo;   // rounding errors of the compensated sums (S, then H)
    lo.alloc(w.S.n);
    HIP_CHECK(hipMemsetAsync(lo.p, 0, sizeof(double) * lo.n, st));
    k_gmg<<<nb256(w.plen), 256, 0, st>>>(w.plen, w.node_sub.p, w.poff_d.p, w.pl.p, w.ne_off.p, w.ne_ptr.p,
                                         w.ne_edge.p, w.ne_sign.p, w.voff_d.p, w.rp_off.p, w.lrp.p, pc->d_lcol.p,
                                         pc->d_lslot.p, s->d_val.p, nullptr, w.ena.p, w.enb.p, w.node.d_desc.p,
                                         w.S.p, lo.p);
    k_fold<<<nb256((int64_t)lo.n), 256, 0, st>>>((int64_t)lo.n, w.S.p, lo.p);
    HIP_CHECK(hipMemsetAsync(lo.p, 0, sizeof(double) * lo.n, st));
    k_gmg<<<nb256(w.plen), 256, 0, st>>>(w.plen, w.node_sub.p, w.poff_d.p, w.pl.p, w.ne_off.p, w.ne_ptr.p,
                                         w.ne_edge.p, w.ne_sign.p, w.voff_d.p, w.rp_off.p, w.lrp.p, pc->d_lcol.p,
                                         pc->d_lslot.p, s->d_val.p, w.bval.p, w.ena.p, w.enb.p, w.node.d_desc.p,
                                         w.H.p, lo.p);
    k_fold<<<nb256((int64_t)lo.n), 256, 0, st>>>((int64_t)lo.n, w.H.p, lo.p);
    factor(w.node, w.S.p, w.Sinv.p, nullptr, 0.0, nullptr, ctx->d_err, st);
    factor(w.node, w.H.p, w.Hinv.p, nullptr, 0.0, nullptr, ctx->d_err, st);
    check_device_error(ctx);
  }

  // ---- LOBPCG
  const int64_t blk = w.len * k;
  if (w.len % kBR) throw Error(GENEO_EINVAL, "batch length not a multiple of the block size");
  const unsigned grows = (unsigned)(w.len / kBR);   // 128-row workgroups of the block-batch products
  DevBuf<double> X, Wb, P, AX, AW, AP, BX, BW, BP, Xn, Pn, T1, T2, Tv, Tb, NT, part, g, coef, theta, nrm;
  for (auto* b : {&X, &Wb, &P, &AX, &AW, &AP, &BX, &BW, &BP, &Xn, &Pn, &T1, &T2, &Tv, &Tb}) b->alloc(blk);
  NT.alloc(w.plen * k);
  const int mmax = 3 * k;
  part.alloc((size_t)w.nchunks * 2 * mmax * mmax);
  g.alloc((size_t)N * 2 * mmax * mmax);
  coef.alloc((size_t)N * mmax * k);
  theta.alloc((size_t)N * k);
  nrm.alloc((size_t)N * k * 2);
  std::vector<int32_t> active(N, 1);
  DevBuf<int32_t> d_active;
  d_active.upload(active, st);
  for (const void* kf : {(const void*)k_gram<1, 4>, (const void*)k_gram<7, 10>})
    HIP_CHECK(hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(sizeof(double) * 3 * kGramSub * ((mmax + 15) / 16 * 16))));

  // start block: warm start if given, else random; B-orthogonal projection out of span(G_j)
  int learned = 0;
  if (pc->opts.warm_start) {
    std::vector<double> h(blk, 0.0);
    k_random_block<<<nb256(blk), 256, 0, st>>>(w.len, k, w.row_sub.p, w.voff_d.p, w.nloc.p, pc->opts.seed, X.p);
    HIP_CHECK(hipMemcpy(h.data(), X.p, sizeof(double) * blk, hipMemcpyDeviceToHost));
    int64_t src = 0;
    for (int j = 0; j < N; ++j) {   // first nev columns from the warm start, guard columns random
      const int64_t ldj = w.voff[j + 1] - w.voff[j];
      for (int q = 0; q < std::min(k, nev); ++q)
        for (int64_t r = 0; r < nloc[j]; ++r) h[w.voff[j] * k + q * ldj + r] = pc->opts.warm_start[src + (int64_t)q * nloc[j] + r];
      src += (int64_t)nloc[j] * nev;
    }
    HIP_CHECK(hipMemcpy(X.p, h.data(), sizeof(double) * blk, hipMemcpyHostToDevice));
  } else {
    k_random_block<<<nb256(blk), 256, 0, st>>>(w.len, k, w.row_sub.p, w.voff_d.p, w.nloc.p, pc->opts.seed, X.p);
    if (pc->opts.model) {
      // the random block stays as the competing candidate (P is unused until the first iteration)
      HIP_CHECK(hipMemcpyAsync(P.p, X.p, sizeof(double) * blk, hipMemcpyDeviceToDevice, st));
      learned = model_warm_start(ctx, pc->opts.model, pc, k, nev, X.p);
      hc.mark("model start block");
    }
  }

  const double drop = 1e-12;
  const int32_t* act = d_active.p;
  auto bmul = [&](const double* V, double* BV) { spmm(pc, w, w.bval.p, V, nullptr, nullptr, BV, st); };
  // V <- V - U (U^T B V), BV recomputed by the caller
  auto orth = [&](const double* U, double* V, const double* BV) {
    gram(w, 1, U, nullptr, nullptr, BV, nullptr, nullptr, BV, nullptr, nullptr, part, g, st);
    k_sub_xc<<<grows, 256, 0, st>>>(w.len, k, w.row_sub.p, w.voff_d.p, U, g.p, 2 * k * k, V);
  };
  // B-orthonormalise V (numerically dependent columns become zero), twice; th receives the
  // Gram eigenvalues (scratch)
  auto svqb2 = [&](DevBuf<double>& V, DevBuf<double>& BV, const int32_t* a, double* th) {
    for (int t = 0; t < 2; ++t) {
      gram(w, 1, V.p, nullptr, nullptr, BV.p, nullptr, nullptr, BV.p, nullptr, nullptr, part, g, st);
      rayleigh_ritz(N, k, k, g.p, a, drop, th, coef.p, 1, st);
      k_combine<<<grows, 256, 0, st>>>(w.len, k, k, 0, w.row_sub.p, w.voff_d.p, a, V.p, nullptr, nullptr,
                                            coef.p, V.p, Tv.p);
      k_combine<<<grows, 256, 0, st>>>(w.len, k, k, 0, w.row_sub.p, w.voff_d.p, a, BV.p, nullptr, nullptr,
                                            coef.p, BV.p, Tb.p);
      V.swap(Tv);
      BV.swap(Tb);
    }
  };
  // V <- V - G_j H_j^-1 G_j^T B V: the B-orthogonal projection out of span(G_j), the kernel of
  // the filtered operator, in which no eigenvector with lambda > 0 has a component
  auto deflate = [&](double* V) {
    if (pc->opts.classical) return;   // the classical pencil is not restricted to the complement of span(G_j)
    spmm(pc, w, w.bval.p, V, nullptr, nullptr, T1.p, st);          // B V
    gt(w, T1.p, NT.p, st);
    solve_multi(w.node, w.H.p, w.Hinv.p, NT.p, k, k, ctx->d_sync, w.flags_node.p, ctx->d_err, st);
    gmul(w, NT.p, V, nullptr, V, st);
  };
  // start block V: projected out of span(G_j) in the B inner product, B-orthonormalised, one
  // Rayleigh-Ritz step (Ritz values into th); AV and BV are the products of the resulting block
  auto start_block = [&](DevBuf<double>& V, DevBuf<double>& AV, DevBuf<double>& BV, DevBuf<double>& Vn,
                         double* th) {
    deflate(V.p);
    bmul(V.p, BV.p);
    svqb2(V, BV, nullptr, th);
    apply_atilde(ctx, pc, w, V.p, AV.p, T1.p, T2.p, NT.p);
    gram(w, 1, V.p, nullptr, nullptr, AV.p, nullptr, nullptr, BV.p, nullptr, nullptr, part, g, st);
    rayleigh_ritz(N, k, k, g.p, nullptr, drop, th, coef.p, 0, st);
    k_combine<<<grows, 256, 0, st>>>(w.len, k, k, 0, w.row_sub.p, w.voff_d.p, nullptr, V.p, nullptr, nullptr,
                                          coef.p, nullptr, Vn.p);
    V.swap(Vn);
    // products are recomputed from the basis after every update (tracking them
    // through the Rayleigh-Ritz coefficients drifts once the basis becomes
    // ill-conditioned near convergence)
    apply_atilde(ctx, pc, w, V.p, AV.p, T1.p, T2.p, NT.p);
    bmul(V.p, BV.p);
  };
  start_block(X, AX, BX, Xn, theta.p);
  hc.mark("start block queued");
  pc->info.learned_candidates = learned;
  if (learned > 0) {
    // The model's block is judged by its eigen-residuals: both candidates take
    // the first Rayleigh-Ritz step, and a subdomain keeps the learned block only
    // if the largest residual of its top min(k, nev) Ritz pairs is below half
    // that of the random block; otherwise it continues from the random block,
    // exactly as the cold start would.
    DevBuf<double> theta_r, nrm_r;
    theta_r.alloc((size_t)N * k);
    nrm_r.alloc((size_t)N * k * 2);
    start_block(P, AP, BP, Pn, theta_r.p);
    k_residual<<<N * k, 256, 0, st>>>(k, w.voff_d.p, AX.p, BX.p, theta.p, Wb.p, nrm.p, nullptr);
    k_residual<<<N * k, 256, 0, st>>>(k, w.voff_d.p, AP.p, BP.p, theta_r.p, Wb.p, nrm_r.p, nullptr);
    std::vector<double> th_l(N * k), th_r(N * k), n_l(N * k * 2), n_r(N * k * 2);
    HIP_CHECK(hipMemcpyAsync(th_l.data(), theta.p, sizeof(double) * N * k, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipMemcpyAsync(th_r.data(), theta_r.p, sizeof(double) * N * k, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipMemcpyAsync(n_l.data(), nrm.p, sizeof(double) * N * k * 2, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipMemcpyAsync(n_r.data(), nrm_r.p, sizeof(double) * N * k * 2, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    // Compared: the largest residual over the pairs that decide the coarse space, the Ritz values
    // above tau (at most nev) of either candidate plus the next one.  A column without B-norm
    // (dropped as dependent) has no residual: infinitely bad.
    const double tau_sel = pc->opts.tau;
    const int kq = std::min(k, nev);
    auto nabove = [&](const std::vector<double>& th, int j) {
      int c = 0;
      while (c < kq && th[j * k + c] > tau_sel) ++c;
      return c;
    };
    auto worst = [&](const std::vector<double>& th, const std::vector<double>& nr, int j, int m) {
      double r = 0.0;
      for (int q = 0; q < m; ++q) {
        const double a = nr[2 * (j * k + q)], b = nr[2 * (j * k + q) + 1];
        const double den = std::fabs(th[j * k + q]) * std::sqrt(b);
        r = std::max(r, den > 0.0 ? std::sqrt(a) / den : HUGE_VAL);
      }
      return r;
    };
    std::vector<int32_t> pick(N, 0);
    int kept = 0;
    for (int j = 0; j < N; ++j) {
      const int m = std::min(kq, std::max(nabove(th_l, j), nabove(th_r, j)) + 1);
      const bool keep = worst(th_l, n_l, j, m) < 0.5 * worst(th_r, n_r, j, m);
      pick[j] = keep ? 0 : 1;
      kept += keep ? 1 : 0;
      if (!keep) std::copy(th_r.begin() + j * k, th_r.begin() + (j + 1) * k, th_l.begin() + j * k);
    }
    learned = kept;
    if (kept < N) {
      DevBuf<int32_t> d_pick;
      d_pick.upload(pick, st);
      k_take_rows<<<nb256(w.len), 256, 0, st>>>(w.len, k, w.row_sub.p, w.voff_d.p, d_pick.p, P.p, AP.p, BP.p, X.p,
                                                AX.p, BX.p);
      HIP_CHECK(hipMemcpyAsync(theta.p, th_l.data(), sizeof(double) * N * k, hipMemcpyHostToDevice, st));
      HIP_CHECK(hipStreamSynchronize(st));
    }
  }
  pc->info.learned_starts = learned;
  hc.mark("start blocks judged");
  const double tol = pc->opts.lobpcg_tol, tau = pc->opts.tau;
  const bool verbose = std::getenv("GENEO_VERBOSE") != nullptr;
  const double cert_tol = std::max(tol, 1e-4);
  constexpr double kCertRough = 1e-2;
  std::vector<double> h_theta(N * k), h_nrm(N * k * 2), h_eta(N * k * 2);
  DevBuf<double> eta;
  eta.alloc((size_t)N * k * 2);
  std::vector<double> best(N, 1e300);
  std::vector<int> best_it(N, 0);
  bool have_p = false;
  int it = 0, unconv = 0;
  const int maxit = std::max(1, pc->opts.lobpcg_maxit);
  // device time of the iteration loop, and of one application of B^-1 to the
  // k-column block (both triangular sweeps over every local factor), timed on
  // the second iteration
  struct LoopEvents {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    ~LoopEvents() {
      for (auto& x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } lt;
  for (auto& x : lt.e) HIP_CHECK(hipEventCreate(&x));
  bool solve_timed = false;
  HIP_CHECK(hipEventRecord(lt.e[0], st));
  for (it = 1; it <= maxit; ++it) {
    // residual shifts of the current block (the projection out of span(G_j)
    // after the update moves it off the Rayleigh-Ritz vectors): the shifts that
    // minimise each residual
    if (it > 1) k_rq<<<N * k, 256, 0, st>>>(k, w.voff_d.p, X.p, AX.p, BX.p, nullptr, theta.p);
    k_residual<<<N * k, 256, 0, st>>>(k, w.voff_d.p, AX.p, BX.p, theta.p, Wb.p, nrm.p, T1.p);
    // W = B^-1 R (used below when the loop goes on) and the B^-1-norms of
    // the residuals (r^T W, R kept in T1) for the certification bound
    if (it == 2) HIP_CHECK(hipEventRecord(lt.e[2], st));
    solve_multi(pc->local, w.LB.p, w.LBinv.p, Wb.p, k, k, ctx->d_sync, w.flags_local.p, ctx->d_err, st);
    if (it == 2) {
      HIP_CHECK(hipEventRecord(lt.e[3], st));
      solve_timed = true;
    }
    k_eta<<<N * k, 256, 0, st>>>(k, w.voff_d.p, T1.p, Wb.p, X.p, BX.p, eta.p);
    HIP_CHECK(hipMemcpyAsync(h_theta.data(), theta.p, sizeof(double) * N * k, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipMemcpyAsync(h_nrm.data(), nrm.p, sizeof(double) * N * k * 2, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipMemcpyAsync(h_eta.data(), eta.p, sizeof(double) * N * k * 2, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    int n_active = 0, n_cert = 0, n_bound = 0;
    double worst_sel = 0.0, worst_cert = 0.0;
    unconv = 0;
    for (int j = 0; j < N; ++j) {
      const double* th = h_theta.data() + j * k;
      auto resid = [&](int q) {
        return std::sqrt(h_nrm[2 * (j * k + q)]) / (std::fabs(th[q]) * std::sqrt(h_nrm[2 * (j * k + q) + 1]) + 1e-300);
      };
      int nsel = 0;
      while (nsel < k && nsel < nev && th[nsel] > tau) ++nsel;
      double rsel = 0.0;
      for (int q = 0; q < nsel; ++q) rsel = std::max(rsel, resid(q));
      // a subdomain whose residual sits at its rounding floor (within 100 tol
      // and no halving over 5 iterations) counts as converged
      if (rsel < best[j] * 0.5) {
        best[j] = rsel;
        best_it[j] = it;
      }
      if (it == 1)
        for (int q = 0; q < std::min(k, nev); ++q) pc->info.start_residual = std::max(pc->info.start_residual, resid(q));
      const bool stalled = rsel <= 100.0 * tol && it - best_it[j] >= 5;
      bool conv = rsel <= tol || stalled;
      if (!conv) unconv += 1;
      // the first Ritz value below tau must be settled too: its residual is
      // below 1e-4, or the pair is roughly converged (residual below 1e-2,
      // after the first iteration) and the interval theta +- ||r||_B^-1 /
      // ||x||_B, which holds an eigenvalue of the pencil for any shift theta,
      // lies below tau.  The interval alone says nothing about eigenvalues
      // the block has not yet found (from a random start every Ritz value is
      // small and its interval below tau).
      auto below_tau = [&](int q) {
        const double e1 = h_eta[2 * (j * k + q)], e2 = h_eta[2 * (j * k + q) + 1];
        return it >= 2 && resid(q) <= kCertRough && e2 > 0.0 && th[q] + std::sqrt(std::max(e1, 0.0) / e2) < tau;
      };
      if (nsel < nev && nsel < k && !(resid(nsel) <= cert_tol)) {
        if (below_tau(nsel)) {
          ++n_bound;
        } else {
          if (conv) ++n_cert;
          conv = false;
          worst_cert = std::max(worst_cert, resid(nsel));
        }
      }
      if (rsel > tol) worst_sel = std::max(worst_sel, rsel);
      active[j] = conv ? 0 : 1;
      n_active += active[j];
      if (verbose && (!conv || it == 1) && (it % 10 == 1 || it == maxit)) {
        double rmax = 0.0;
        for (int q = 0; q < std::min(k, nsel + 1); ++q) rmax = std::max(rmax, resid(q));
        std::fprintf(stderr, "[lobpcg] it %d sub %d nsel %d theta0 %.6g theta_k-1 %.6g maxres %.3g conv %d\n", it, j,
                     nsel, th[0], th[k - 1], rmax, (int)conv);
      }
    }
    if (verbose)
      std::fprintf(stderr,
                   "[lobpcg] it %d active %d (certification only %d, certified by the interval %d) worst selected "
                   "res %.3g worst cert res %.3g\n",
                   it, n_active, n_cert, n_bound, worst_sel, worst_cert);
    if (n_active == 0 || it == maxit) break;
    HIP_CHECK(hipMemcpyAsync(d_active.p, active.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, st));
    // W = B^-1 R, B-orthogonal to span(G_j) and X, B-orthonormal.  In exact arithmetic
    // G_j^T B W = G_j^T Atilde X = 0 already; B^-1 amplifies the rounding errors of R along the
    // near-kernel of B (gradients, eigenvalues ~ gamma), so W is projected again (as are the
    // updated X and P below).
    deflate(Wb.p);
    for (int t = 0; t < 2; ++t) {
      bmul(Wb.p, BW.p);
      orth(X.p, Wb.p, BW.p);
    }
    bmul(Wb.p, BW.p);
    svqb2(Wb, BW, act, theta.p);
    if (have_p) {   // P B-orthogonal to X and W, B-orthonormal
      for (int t = 0; t < 2; ++t) {
        bmul(P.p, BP.p);
        orth(X.p, P.p, BP.p);
        bmul(P.p, BP.p);
        orth(Wb.p, P.p, BP.p);
      }
      bmul(P.p, BP.p);
      svqb2(P, BP, act, theta.p);
      apply_atilde(ctx, pc, w, P.p, AP.p, T1.p, T2.p, NT.p);
    }
    apply_atilde(ctx, pc, w, Wb.p, AW.p, T1.p, T2.p, NT.p);
    const int nl = have_p ? 3 : 2;
    const int m = nl * k;
    gram(w, nl, X.p, Wb.p, have_p ? P.p : nullptr, AX.p, AW.p, have_p ? AP.p : nullptr, BX.p, BW.p,
         have_p ? BP.p : nullptr, part, g, st);
    rayleigh_ritz(N, m, k, g.p, act, drop, theta.p, coef.p, 0, st);
    k_combine<<<grows, 256, 0, st>>>(w.len, k, m, 0, w.row_sub.p, w.voff_d.p, act, X.p, Wb.p,
                                          have_p ? P.p : nullptr, coef.p, X.p, Xn.p);
    k_combine<<<grows, 256, 0, st>>>(w.len, k, m, k, w.row_sub.p, w.voff_d.p, act, X.p, Wb.p,
                                          have_p ? P.p : nullptr, coef.p, have_p ? P.p : nullptr, Pn.p);
    X.swap(Xn);
    P.swap(Pn);
    // the Ritz update mixes blocks whose gradient components rounding keeps
    // re-creating; without this projection the residual of small-gamma
    // problems stalls far above the rounding floor of the filtered operator
    deflate(X.p);
    deflate(P.p);
    apply_atilde(ctx, pc, w, X.p, AX.p, T1.p, T2.p, NT.p);
    bmul(X.p, BX.p);
    have_p = true;
    HIP_CHECK(hipGetLastError());
  }
  // the eigenvalues: Rayleigh quotients of the final block with the factored denominator
  k_ltx<<<(unsigned)w.nlt, 256, 0, st>>>(k, pc->local.d_desc.p, w.lt_blk.p, w.voff_d.p, w.LB.p, X.p, T2.p);
  k_rq<<<N * k, 256, 0, st>>>(k, w.voff_d.p, X.p, AX.p, BX.p, T2.p, theta.p);
  HIP_CHECK(hipEventRecord(lt.e[1], st));
  HIP_CHECK(hipMemcpyAsync(h_theta.data(), theta.p, sizeof(double) * N * k, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  check_device_error(ctx);
  {
    float ms = 0.0f;
    HIP_CHECK(hipEventElapsedTime(&ms, lt.e[0], lt.e[1]));
    pc->info.t_lobpcg_loop_ms = ms;
    if (solve_timed) {
      HIP_CHECK(hipEventElapsedTime(&ms, lt.e[2], lt.e[3]));
      pc->info.lobpcg_solve_ms = ms;
    }
    double bytes = 0.0;
    for (int j = 0; j < N; ++j) bytes += (double)nloc[j] * ((double)nloc[j] + 1.0) * 8.0;
    pc->info.lobpcg_solve_bytes = bytes;
  }
  hc.mark("iterations done");
  pc->info.lobpcg_iters = it > maxit ? maxit : it;
  pc->info.lobpcg_unconverged = unconv;

  if (pc->opts.keep_ritz) {
    pc->d_ritz.alloc(blk);
    HIP_CHECK(hipMemcpyAsync(pc->d_ritz.p, X.p, sizeof(double) * blk, hipMemcpyDeviceToDevice, st));
    pc->ritz_k = k;
  }

  // ---- selection and coarse vectors D_j (I - xi_j) X_sel
  std::vector<int32_t> sel(N, 0);
  for (int j = 0; j < N; ++j) {
    const double* th = h_theta.data() + j * k;
    pc->eigs[j].assign(th, th + k);
    int c = 0;
    while (c < k && c < nev && th[c] > tau) ++c;
    sel[j] = c;
    pc->eig_sel[j] = c;
  }
  // u = D (X - G S^-1 G^T A X) into T1 (all k columns), then pack the selected ones
  ctx_mul(w, X.p, NT.p, st);
  solve_multi(w.node, w.S.p, w.Sinv.p, NT.p, k, k, ctx->d_sync, w.flags_node.p, ctx->d_err, st);
  gmul(w, NT.p, X.p, pc->d_bpou.p, T1.p, st);
  check_device_error(ctx);
  pc->gen_cnt = sel;
  pc->w_off.assign(N + 1, 0);
  for (int j = 0; j < N; ++j) pc->w_off[j + 1] = pc->w_off[j] + (w.voff[j + 1] - w.voff[j]) * sel[j];
  pc->d_W.alloc(std::max<int64_t>(pc->w_off[N], 1));
  for (int j = 0; j < N; ++j)
    if (sel[j])
      HIP_CHECK(hipMemcpyAsync(pc->d_W.p + pc->w_off[j], T1.p + w.voff[j] * k,
                               sizeof(double) * (w.voff[j + 1] - w.voff[j]) * sel[j], hipMemcpyDeviceToDevice, st));
  std::vector<int64_t> goff(N + 1, 0);
  for (int j = 0; j < N; ++j) goff[j + 1] = goff[j] + sel[j];
  pc->d_gen_off.upload(goff, st);
  pc->d_gen_cnt.upload(sel, st);
  pc->d_w_off.upload(pc->w_off, st);
  pc->d_voff.upload(w.voff, st);
  pc->d_n.upload(nloc, st);
  HIP_CHECK(hipStreamSynchronize(st));
}

}  // namespace geneo
