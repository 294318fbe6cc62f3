// Setup and application of the two-level additive Schwarz preconditioner
//   M^-1 r = Z E^-1 Z^T r + (I - P_0) sum_i R_i^T A_i^-1 R_i (I - P_0^T) r,
// and preconditioned conjugate gradients.
//
// Batch vectors: the restrictions R_i r of all subdomains side by side, each
// padded to n_pad; gathers use the batch -> free-edge map, and the sum of
// extensions R_i^T uses the inverse map (free edge -> batch positions) in a
// fixed order, so results are bitwise reproducible.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <exception>
#include <numeric>
#include <thread>
#include <string>

#include "precond.h"

namespace geneo {

// ---------------------------------------------------------- small kernels
// Dense batch matrices: zero, with ones on the diagonal of the padding rows
// (r >= n).  Workgroup (c, m) writes column c of matrix m with 16-byte stores
// (launch: grid (max ld, nmat)); lower != 0: only rows r >= c (rounded down
// to even), the part a factorisation reads.
__global__ __launch_bounds__(256) void k_fill_identity_pad(const MatDesc* __restrict__ desc, double* __restrict__ A,
                                                           float* __restrict__ Af, int lower = 0) {
  const MatDesc d = desc[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= d.ld) return;
  const int64_t col = d.off + (int64_t)c * d.ld;
  for (int r = (lower ? (c & ~1) : 0) + 2 * threadIdx.x; r < d.ld; r += 512) {
    const double v0 = (r == c && r >= d.n) ? 1.0 : 0.0, v1 = (r + 1 == c && r + 1 >= d.n) ? 1.0 : 0.0;
    if (A) *reinterpret_cast<double2*>(A + col + r) = double2{v0, v1};
    if (Af) *reinterpret_cast<float2*>(Af + col + r) = float2{(float)v0, (float)v1};
  }
}
static dim3 fill_grid(const std::vector<MatDesc>& d) {
  int mx = 1;
  for (const auto& x : d) mx = std::max(mx, x.ld);
  return dim3((unsigned)mx, (unsigned)d.size());
}

// dense A_i from the global CSR values through the local CSR triplets
__global__ void k_dense_scatter(int64_t nnz, const int32_t* __restrict__ lrow, const int32_t* __restrict__ lcol,
                                const int32_t* __restrict__ lslot, const int64_t* __restrict__ nnz_off, int nmat,
                                const MatDesc* __restrict__ desc, const double* __restrict__ val,
                                double* __restrict__ A, float* __restrict__ Af) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  int lo = 0, hi = nmat - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (nnz_off[mid] <= k) lo = mid; else hi = mid - 1;
  }
  const MatDesc d = desc[lo];
  int64_t pos = d.off + (int64_t)lcol[k] * d.ld + lrow[k];
  double v = val[lslot[k]];
  if (A) A[pos] = v;
  if (Af) Af[pos] = (float)v;
}

__global__ void k_gather(int64_t len, const int32_t* __restrict__ bmap, const double* __restrict__ g,
                         double* __restrict__ b) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= len) return;
  int32_t e = bmap[k];
  b[k] = e >= 0 ? g[e] : 0.0;
}

// out[e] = (base ? base[e] : 0) + sign * sum_{k in inv(e)} b[k]
__global__ void k_scatter_add(int64_t n, const int32_t* __restrict__ ip, const int32_t* __restrict__ ii,
                              const double* __restrict__ b, const double* __restrict__ base, double sign,
                              double* __restrict__ out) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  double acc = 0.0;
  for (int32_t k = ip[e]; k < ip[e + 1]; ++k) acc += b[ii[k]];
  out[e] = (base ? base[e] : 0.0) + sign * acc;
}

// t[c] = sum over the entries of sparse column c: val * r[row]
__global__ void k_csc_t(int64_t ncol, const int32_t* __restrict__ cp, const int32_t* __restrict__ ri,
                        const double* __restrict__ cv, const double* __restrict__ r, double* __restrict__ t) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  double acc = 0.0;
  for (int32_t k = cp[c]; k < cp[c + 1]; ++k) acc += cv[k] * r[ri[k]];
  t[c] = acc;
}

// u[e] = sum over the entries of sparse row e: val * c[col]  (+ add[e] if given)
__global__ void k_csr(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                      const double* __restrict__ v, const double* __restrict__ c, const double* __restrict__ add,
                      double* __restrict__ u) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  double acc = add ? add[e] : 0.0;
  for (int32_t k = rp[e]; k < rp[e + 1]; ++k) acc += v[k] * c[ci[k]];
  u[e] = acc;
}

// GenEO columns, transpose: t[gen_off_j + k] = W_j(:,k) . b_j (one wave per column)
__global__ void k_w_t(int nsub, const int32_t* __restrict__ gcnt, const int64_t* __restrict__ goff,
                      const int64_t* __restrict__ woff, const int64_t* __restrict__ voff,
                      const int32_t* __restrict__ nloc, const double* __restrict__ W, const double* __restrict__ b,
                      double* __restrict__ t, int64_t total_cols) {
  const int64_t col = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (col >= total_cols) return;
  int lo = 0, hi = nsub - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (goff[mid] <= col) lo = mid; else hi = mid - 1;
  }
  const int64_t k = col - goff[lo];
  const int n = nloc[lo];
  const int64_t ld = voff[lo + 1] - voff[lo];
  const double* w = W + woff[lo] + k * ld;
  const double* bb = b + voff[lo];
  double acc = 0.0;
  for (int r = lane; r < n; r += 64) acc += w[r] * bb[r];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) t[col] = acc;
}

// GenEO columns, forward: b_j = W_j c_j (batch vector; pads get 0)
__global__ void k_w_n(int64_t len, int nsub, const int64_t* __restrict__ voff, const int32_t* __restrict__ gcnt,
                      const int64_t* __restrict__ goff, const int64_t* __restrict__ woff,
                      const double* __restrict__ W, const double* __restrict__ c, double* __restrict__ b) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= len) return;
  int lo = 0, hi = nsub - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (voff[mid] <= k) lo = mid; else hi = mid - 1;
  }
  const int64_t r = k - voff[lo];
  const int64_t ld = voff[lo + 1] - voff[lo];
  const double* w = W + woff[lo] + r;
  const double* cc = c + goff[lo];
  double acc = 0.0;
  for (int j = 0; j < gcnt[lo]; ++j) acc += w[j * ld] * cc[j];
  b[k] = acc;
}

__global__ void k_unit_diag(int64_t m, const int32_t* __restrict__ pos, double* __restrict__ E, int64_t ld) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < m) E[(int64_t)pos[t] * ld + pos[t]] = 1.0;
}

__global__ void k_copy(int64_t n, const double* __restrict__ x, double* __restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = x[i];
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double bcoef, const double* __restrict__ y,
                        double* __restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * x[i] + bcoef * (y ? y[i] : 0.0);
}

__global__ void k_copy_diag(const MatDesc* __restrict__ desc, const double* __restrict__ A, double* __restrict__ od) {
  const MatDesc d = desc[blockIdx.y];
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < d.ld) od[d.diag_off + i] = A[d.off + i * d.ld + i];
}

// E (SNK x SNK) = Z^T A Z, one thread per coarse column c1 (writes column c1 only; with perm,
// natural column c sits at row / column perm[c])
__global__ void k_coarse_snk(int64_t nsnk, const int32_t* __restrict__ zc_ptr, const int32_t* __restrict__ zc_row,
                             const double* __restrict__ zc_val, const int32_t* __restrict__ rp,
                             const int32_t* __restrict__ ci, const double* __restrict__ av,
                             const int32_t* __restrict__ zr_ptr, const int32_t* __restrict__ zr_col,
                             const double* __restrict__ zr_val, const int32_t* __restrict__ perm,
                             double* __restrict__ E, int64_t ld, uint8_t* __restrict__ tiles, int nbt) {
  int64_t c1 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c1 >= nsnk) return;
  const int64_t pc1 = perm ? perm[c1] : c1;
  double* col = E + pc1 * ld;
  int64_t last = -1;   // last tile marked (consecutive writes mostly share one)
  for (int32_t k1 = zc_ptr[c1]; k1 < zc_ptr[c1 + 1]; ++k1) {
    const int32_t e = zc_row[k1];
    const double z1 = zc_val[k1];
    for (int32_t s = rp[e]; s < rp[e + 1]; ++s) {
      const int32_t f = ci[s];
      const double a = av[s] * z1;
      for (int32_t k2 = zr_ptr[f]; k2 < zr_ptr[f + 1]; ++k2) {
        const int32_t c2 = zr_col[k2];
        const int64_t pr = perm ? perm[c2] : c2;
        const double v = a * zr_val[k2];
        col[pr] += v;
        if (tiles && pr >= pc1 && v != 0.0) {
          const int64_t t = (pr / NB) * nbt + pc1 / NB;
          if (t != last) {
            tiles[t] = 1;
            last = t;
          }
        }
      }
    }
  }
}

// Global GenEO columns: Zg[:, gen_off_j + q] = R_j^T W_j[:, q]; one thread per batch row.
__global__ void k_zg_scatter(int64_t len, int nsub, const int64_t* __restrict__ voff, const int32_t* __restrict__ nloc,
                             const int32_t* __restrict__ gcnt, const int64_t* __restrict__ goff,
                             const int64_t* __restrict__ woff, const int32_t* __restrict__ bmap,
                             const double* __restrict__ W, int64_t n, double* __restrict__ Zg) {
  int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= len) return;
  int lo = 0, hi = nsub - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (voff[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const int64_t r = b - voff[lo];
  if (r >= nloc[lo]) return;
  const int64_t ld = voff[lo + 1] - voff[lo];
  const int32_t e = bmap[b];
  for (int q = 0; q < gcnt[lo]; ++q) Zg[(goff[lo] + q) * n + e] = W[woff[lo] + q * ld + r];
}

// Y = A Z_gen on the rows where it can be non-zero: one thread per ring row
// of a subdomain, computing that row for the subdomain's GenEO columns
// (Z_gen column-major n x ngen, zero outside the column's subdomain).
__global__ void k_spmm_ring(int64_t nring, int nsub, const int32_t* __restrict__ ring_ptr,
                            const int32_t* __restrict__ ring, const int32_t* __restrict__ gcnt,
                            const int64_t* __restrict__ goff, const int32_t* __restrict__ rp,
                            const int32_t* __restrict__ ci, const double* __restrict__ v, int64_t n,
                            const double* __restrict__ Zg, double* __restrict__ Y) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nring) return;
  int lo = 0, hi = nsub - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ring_ptr[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const int32_t e = ring[t];
  const int32_t k0 = rp[e], k1 = rp[e + 1];
  for (int q = 0; q < gcnt[lo]; ++q) {
    const int64_t g = goff[lo] + q;
    const double* z = Zg + g * n;
    double acc = 0.0;
    for (int32_t k = k0; k < k1; ++k) acc += v[k] * z[ci[k]];
    Y[g * n + e] = acc;
  }
}

// Lower triangle of the GenEO columns of E = Z^T Y, Y = A Z_gen (global,
// n x ngen, column-major).  Grid row blockIdx.y = GenEO column g; the
// threads run over the candidate rows c1 of g's subdomain (the columns of
// subdomains whose dofs meet its ring; every other entry is zero).  SNK
// rows use their sparse column; GenEO rows the dense local block of their
// subdomain (a GenEO column lives on one subdomain's edges only).
__global__ void k_coarse_gen(int64_t nsnk, int64_t n, const int32_t* __restrict__ zc_ptr,
                             const int32_t* __restrict__ zc_row, const double* __restrict__ zc_val, int nsub,
                             const int64_t* __restrict__ goff, const int32_t* __restrict__ cand_ptr,
                             const int32_t* __restrict__ cand, const int64_t* __restrict__ voff,
                             const int32_t* __restrict__ nloc, const int64_t* __restrict__ woff,
                             const int32_t* __restrict__ bmap, const double* __restrict__ W,
                             const double* __restrict__ Y, const int32_t* __restrict__ perm,
                             double* __restrict__ E, int64_t ld, uint8_t* __restrict__ tiles, int nbt) {
  // lower-triangle entry (r, c) of the natural order, r >= c, at its place in the factor's order
  // (the tile of a non-zero marked in `tiles`)
  auto put = [&](int64_t r, int64_t c, double v) {
    int64_t pr = perm ? perm[r] : r, pc = perm ? perm[c] : c;
    if (pr < pc) {
      const int64_t t = pr;
      pr = pc;
      pc = t;
    }
    if (tiles && v != 0.0) tiles[(pr / NB) * nbt + pc / NB] = 1;
    E[pc * ld + pr] = v;
  };
  const int64_t g = blockIdx.y;
  int j = 0, hi = nsub - 1;   // subdomain of GenEO column g
  while (j < hi) {
    const int mid = (j + hi + 1) >> 1;
    if (goff[mid] <= g) j = mid; else hi = mid - 1;
  }
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= cand_ptr[j + 1] - cand_ptr[j]) return;
  const int64_t c1 = cand[cand_ptr[j] + t];
  const int64_t cg = nsnk + g;
  const double* y = Y + g * n;
  if (c1 < nsnk) {
    double acc = 0.0;
    for (int32_t k = zc_ptr[c1]; k < zc_ptr[c1 + 1]; ++k) acc += zc_val[k] * y[zc_row[k]];
    put(cg, c1, acc);               // row cg > c1, column c1
    return;
  }
  if (c1 < cg) return;              // upper triangle: not needed
  const int64_t g1 = c1 - nsnk;
  int lo = 0;
  hi = nsub - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (goff[mid] <= g1) lo = mid; else hi = mid - 1;
  }
  const int64_t q = g1 - goff[lo];
  const int64_t lds = voff[lo + 1] - voff[lo];
  const double* w = W + woff[lo] + q * lds;
  const int32_t* bm = bmap + voff[lo];
  double acc = 0.0;
  for (int64_t r = 0; r < nloc[lo]; ++r) acc += w[r] * y[bm[r]];
  put(c1, cg, acc);                 // row c1 >= cg, column cg
}

// Host side of the support restriction (k_spmm_ring / k_coarse_gen).
struct GenSupport {
  std::vector<int32_t> ring, ring_ptr;   // per subdomain j: free edges coupled to dofs(j) through A
  std::vector<int32_t> cand, cand_ptr;   // per subdomain j: coarse columns of subdomains meeting ring_j
  int64_t max_cand = 0;
};

static GenSupport gen_support(const geneo_system* s, const geneo_decomp* dec, const std::vector<int32_t>& gen_cnt,
                              const std::vector<int32_t>& col_sub, int64_t nsnk,
                              const std::vector<int64_t>& gen_off) {
  const int N = dec->N;
  const int64_t n = s->n;
  const int Wd = (N + 63) / 64;
  GenSupport g;
  // subdomains holding each free edge (bit masks)
  std::vector<uint64_t> emask((size_t)n * Wd, 0);
  for (int i = 0; i < N; ++i)
    for (int64_t r = dec->dofs_ptr[i]; r < dec->dofs_ptr[i + 1]; ++r)
      emask[(size_t)dec->dofs[r] * Wd + i / 64] |= 1ull << (i % 64);
  std::vector<uint64_t> adj((size_t)N * Wd, 0);
  std::vector<int32_t> stamp(n, -1);
  g.ring_ptr.assign(N + 1, 0);
  for (int j = 0; j < N; ++j) {
    if (gen_cnt[j] > 0) {
      for (int64_t r = dec->dofs_ptr[j]; r < dec->dofs_ptr[j + 1]; ++r) {
        const int32_t e = dec->dofs[r];
        for (int32_t k = s->rowptr[e]; k < s->rowptr[e + 1]; ++k) {
          const int32_t f = s->colind[k];
          if (stamp[f] == j) continue;
          stamp[f] = j;
          g.ring.push_back(f);
          for (int w = 0; w < Wd; ++w) adj[(size_t)j * Wd + w] |= emask[(size_t)f * Wd + w];
        }
      }
    }
    g.ring_ptr[j + 1] = (int32_t)g.ring.size();
  }
  // coarse columns per subdomain: SNK ranges (subdomain-major), GenEO ranges;
  // columns that belong to no subdomain (global near-kernel, col_sub = -1)
  // are candidates of every GenEO column
  std::vector<int64_t> snk_beg(N + 1, 0);
  std::vector<int32_t> unowned;
  for (int64_t c = 0; c < nsnk; ++c) {
    if (col_sub[c] < 0)
      unowned.push_back((int32_t)c);
    else
      snk_beg[col_sub[c] + 1]++;
  }
  for (int i = 0; i < N; ++i) snk_beg[i + 1] += snk_beg[i];
  if (!unowned.empty() && (int64_t)unowned.size() != nsnk)
    throw Error(GENEO_EINVAL, "coarse columns: owned and global columns mixed");
  g.cand_ptr.assign(N + 1, 0);
  for (int j = 0; j < N; ++j) {
    if (gen_cnt[j] > 0) g.cand.insert(g.cand.end(), unowned.begin(), unowned.end());
    if (gen_cnt[j] > 0)
      for (int i = 0; i < N; ++i) {
        if (!((adj[(size_t)j * Wd + i / 64] >> (i % 64)) & 1)) continue;
        if (unowned.empty())
          for (int64_t c = snk_beg[i]; c < snk_beg[i + 1]; ++c) g.cand.push_back((int32_t)c);
        for (int64_t c = gen_off[i]; c < gen_off[i + 1]; ++c) g.cand.push_back((int32_t)(nsnk + c));
      }
    g.cand_ptr[j + 1] = (int32_t)g.cand.size();
    g.max_cand = std::max<int64_t>(g.max_cand, g.cand_ptr[j + 1] - g.cand_ptr[j]);
  }
  return g;
}


// ---------------------------------------------------------- dot products
constexpr int kDotBlocks = 512;

__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ x, const double* __restrict__ y,
                                                     int64_t n, double* __restrict__ part) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kDotBlocks * 256) acc += x[i] * y[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kDotBlocks) void k_dot_final(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double s[kDotBlocks];
  s[threadIdx.x] = part[threadIdx.x];
  __syncthreads();
  for (int o = kDotBlocks / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

void dot(const double* x, const double* y, int64_t n, double* partial, double* out, hipStream_t st) {
  k_dot_partial<<<kDotBlocks, 256, 0, st>>>(x, y, n, partial);
  k_dot_final<<<1, kDotBlocks, 0, st>>>(partial, out);
}

static inline unsigned nblocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// out = [b -] A_i x on every batch row (FP64), rows with mask 0 give 0;
// out may alias b (each thread reads and writes only its own row).
__global__ void k_local_residual(int64_t len, const int64_t* __restrict__ rp, const int32_t* __restrict__ bcol,
                                 const int32_t* __restrict__ bslot, const double* __restrict__ gval,
                                 const double* b, const double* __restrict__ x, const int8_t* __restrict__ mask,
                                 double* out) {
  const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (row >= len) return;
  double acc = 0.0;
  for (int64_t t = rp[row]; t < rp[row + 1]; ++t) acc += gval[bslot[t]] * x[bcol[t]];
  const double v = (b ? b[row] : 0.0) - acc;
  out[row] = (mask && !mask[row]) ? 0.0 : v;
}

// reproducible pseudo-random start vector in [-1, 1) on real batch rows (splitmix64)
__global__ void k_hash_fill(int64_t len, const int32_t* __restrict__ bmap, uint64_t seed, double* __restrict__ x) {
  const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (row >= len) return;
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(row + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  x[row] = bmap[row] < 0 ? 0.0 : (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

// out[i] = sum of squares of segment i (one block per subdomain, fixed order)
__global__ __launch_bounds__(256) void k_seg_sumsq(const int64_t* __restrict__ voff, const double* __restrict__ x,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int64_t r = voff[i] + threadIdx.x; r < voff[i + 1]; r += 256) acc += x[r] * x[r];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// ---------------------------------------------------------------- setup

void check_device_error(geneo_ctx* ctx) {
  HIP_CHECK(hipMemcpyAsync(ctx->h_err, ctx->d_err, sizeof(DevErr), hipMemcpyDeviceToHost, ctx->stream));
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  DevErr e = *ctx->h_err;
  if (e.code != 0) {
    HIP_CHECK(hipMemsetAsync(ctx->d_err, 0, sizeof(DevErr), ctx->stream));
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    if (e.code == GENEO_ENOTSPD)
      throw Error(GENEO_ENOTSPD, "Cholesky pivot not positive: matrix " + std::to_string(e.mat) + ", column " +
                                     std::to_string(e.idx));
    if (e.code == GENEO_ESYNC) throw Error(GENEO_ESYNC, "device-side wait expired in a triangular solve");
    throw Error(e.code, "device error " + std::to_string(e.code));
  }
}

static float elapsed(geneo_ctx* ctx, int a, int b) {
  HIP_CHECK(hipEventSynchronize(ctx->ev[b]));
  float ms = 0;
  HIP_CHECK(hipEventElapsedTime(&ms, ctx->ev[a], ctx->ev[b]));
  return ms;
}

// Conditioning check before any FP32 work.  The hat function of a node all
// of whose edges lie in Omega_i has the edge coefficients v = G e_node
// (+-1 on those edges); the curl-curl part annihilates it, so its Rayleigh
// quotient in the diagonally scaled matrix D^-1/2 A_i D^-1/2 (D = diag A_i),
//   q = v^T A_i v / v^T D v,
// bounds that matrix's smallest eigenvalue from above.  Its diagonal is 1,
// so 1/q bounds its condition number from below, and Cholesky's rounding
// error follows the condition number of the scaled matrix.  On the measured
// subdomains the refinement radius rho(I - Ahat^-1 A_i) of the FP32 factor
// was at least kFp32RhoPerBound * u32 / q; a subdomain where that exceeds
// fp32_rho_max is flagged (value 2) so the FP32 kernels skip it, and it is
// factored in FP64 directly.  A subdomain without a usable node keeps its
// FP32 attempt.
constexpr double kFp32RhoPerBound = 0.2;
constexpr int kFp32CheckNodes = 32;

struct Fp32Check {
  std::vector<int32_t> smp_off, pair_off, slot;
  std::vector<int8_t> w;   // +-1: off-diagonal term of v^T A v; 2: diagonal (also in v^T D v)
};

static Fp32Check fp32_check_plan(const geneo_system* s, const geneo_decomp* dec) {
  const int64_t n = s->n;
  const int64_t p = (int64_t)s->free_nodes.size();
  // free edges at each free node, with the coefficient of that node's hat gradient
  std::vector<int32_t> nptr(p + 1, 0);
  for (int64_t fe = 0; fe < n; ++fe) {
    const int32_t ge = s->free_edges[fe];
    for (int end = 0; end < 2; ++end) {
      const int32_t fn = s->node_to_free[s->edges[2 * (int64_t)ge + end]];
      if (fn >= 0) nptr[fn + 1]++;
    }
  }
  for (int64_t k = 0; k < p; ++k) nptr[k + 1] += nptr[k];
  std::vector<int32_t> ned(nptr[p]);
  std::vector<int8_t> nsg(nptr[p]);
  {
    std::vector<int32_t> f(nptr.begin(), nptr.end() - 1);
    for (int64_t fe = 0; fe < n; ++fe) {
      const int32_t ge = s->free_edges[fe];
      for (int end = 0; end < 2; ++end) {
        const int32_t fn = s->node_to_free[s->edges[2 * (int64_t)ge + end]];
        if (fn < 0) continue;
        ned[f[fn]] = (int32_t)fe;
        nsg[f[fn]++] = end ? 1 : -1;   // edge (a, b): grad phi_b = +w_e, grad phi_a = -w_e
      }
    }
  }
  const int32_t N = dec->N;
  std::vector<std::vector<int32_t>> cnt(N), sl(N);
  std::vector<std::vector<int8_t>> ww(N);
  parallel_for(N, [&](int i) {
    const int32_t* d0 = dec->dofs.data() + dec->dofs_ptr[i];
    const int32_t* d1 = dec->dofs.data() + dec->dofs_ptr[i + 1];
    const int64_t g0 = dec->gn_ptr[i], ng = dec->gn_ptr[i + 1] - g0;
    const int64_t tries = std::min<int64_t>(ng, 4 * kFp32CheckNodes);
    for (int64_t t = 0; t < tries && (int)cnt[i].size() < kFp32CheckNodes; ++t) {
      const int32_t fn = dec->gnodes[g0 + t * ng / tries];
      bool inside = nptr[fn + 1] > nptr[fn];
      for (int32_t k = nptr[fn]; k < nptr[fn + 1] && inside; ++k) inside = std::binary_search(d0, d1, ned[k]);
      if (!inside) continue;
      int32_t m = 0;
      for (int32_t a = nptr[fn]; a < nptr[fn + 1]; ++a)
        for (int32_t b = nptr[fn]; b < nptr[fn + 1]; ++b) {
          const int32_t e = ned[a], f = ned[b];
          for (int32_t q = s->rowptr[e]; q < s->rowptr[e + 1]; ++q)
            if (s->colind[q] == f) {
              sl[i].push_back(q);
              ww[i].push_back(e == f ? 2 : (int8_t)(nsg[a] * nsg[b]));
              ++m;
              break;
            }
        }
      cnt[i].push_back(m);
    }
  });
  Fp32Check c;
  c.smp_off.assign(N + 1, 0);
  c.pair_off.assign(1, 0);
  for (int32_t i = 0; i < N; ++i) {
    c.smp_off[i + 1] = c.smp_off[i] + (int32_t)cnt[i].size();
    for (int32_t m : cnt[i]) c.pair_off.push_back(c.pair_off.back() + m);
    c.slot.insert(c.slot.end(), sl[i].begin(), sl[i].end());
    c.w.insert(c.w.end(), ww[i].begin(), ww[i].end());
  }
  return c;
}

// One workgroup per subdomain: q of each sampled node, the smallest q, the
// flag and the bound 1/q (0 without a usable node, infinite for q <= 0).
__global__ __launch_bounds__(256) void k_fp32_check(const int32_t* __restrict__ smp_off,
                                                    const int32_t* __restrict__ pair_off,
                                                    const int32_t* __restrict__ slot, const int8_t* __restrict__ w,
                                                    const double* __restrict__ val, double q_floor,
                                                    int32_t* __restrict__ failed, double* __restrict__ kappa_lb) {
  __shared__ double red[256];
  const int i = blockIdx.x, tid = threadIdx.x;
  double q = INFINITY;
  for (int k = smp_off[i] + tid; k < smp_off[i + 1]; k += 256) {
    double num = 0.0, den = 0.0;
    for (int t = pair_off[k]; t < pair_off[k + 1]; ++t) {
      const double a = val[slot[t]];
      if (w[t] == 2) {
        num += a;
        den += a;
      } else {
        num += (double)w[t] * a;
      }
    }
    q = fmin(q, den > 0.0 ? num / den : 0.0);
  }
  red[tid] = q;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] = fmin(red[tid], red[tid + h]);
    __syncthreads();
  }
  if (tid == 0) {
    const double qm = red[0];
    kappa_lb[i] = qm > 0.0 ? (qm == INFINITY ? 0.0 : 1.0 / qm) : INFINITY;
    failed[i] = qm < q_floor ? 2 : 0;
  }
}

// FP32 local factors with one FP64 refinement step apply the map
//   y = yhat + Ahat^-1 (r - A_i yhat),  yhat = Ahat^-1 r,
// i.e. (2 Ahat^-1 - Ahat^-1 A_i Ahat^-1) r, which is symmetric and positive
// definite exactly when rho(I - Ahat^-1 A_i) < 1.  The probe estimates that
// radius per subdomain by power iteration on I - Ahat^-1 A_i (FP64 residual,
// FP32 solve) and refactors in FP64 every subdomain whose estimate exceeds
// fp32_rho_max or is not finite.
constexpr int64_t kFp32MinShare = 8;   // FP32 factors are kept only on at least 1 / 8 of the subdomains

static void fp32_probe(geneo_ctx* ctx, geneo_precond* pc, const std::vector<MatDesc>& descs,
                       const int32_t* d_failed, const double* d_kappa_lb) {
  constexpr int kPowerSteps = 8;
  hipStream_t st = ctx->stream;
  const int32_t N = pc->N;
  const int64_t len = pc->batch_len;
  const geneo_system* s = pc->sys;
  double* v = pc->w_b1.p;
  double* t = pc->w_b2.p;
  DevBuf<double> sq;
  sq.alloc(2 * (int64_t)N);
  DevBuf<int64_t> d_voff;
  d_voff.upload(pc->voff, st);
  std::vector<int32_t> failed(N);
  std::vector<double> klb(N);
  HIP_CHECK(hipMemcpyAsync(failed.data(), d_failed, sizeof(int32_t) * N, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipMemcpyAsync(klb.data(), d_kappa_lb, sizeof(double) * N, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  pc->info.fp32_prechecked = (int32_t)std::count(failed.begin(), failed.end(), 2);
  pc->info.fp32_kappa_lb = klb.empty() ? 0.0 : *std::max_element(klb.begin(), klb.end());
  // the power iteration only matters for factors that completed, and only if
  // at least 1 in kFp32MinShare did: the survivors are among them, so with
  // fewer the share rule below sends every subdomain to FP64 whatever the
  // probe finds
  const int64_t n_ok = std::count(failed.begin(), failed.end(), 0);
  const bool any_ok = n_ok > 0 && n_ok * kFp32MinShare >= N;
  k_hash_fill<<<nblocks(len), 256, 0, st>>>(len, pc->d_bmap.p, pc->opts.seed ^ 0x5eedull, v);
  for (int it = 0; it < (any_ok ? kPowerSteps : 0); ++it) {
    k_local_residual<<<nblocks(len), 256, 0, st>>>(len, pc->d_brp.p, pc->d_bcol.p, pc->d_lslot.p, s->d_val.p,
                                                   nullptr, v, nullptr, t);
    solve(pc->local, pc->fL.p, pc->fLinv.p, t, ctx->d_sync, ctx->d_err, st);
    k_axpby<<<nblocks(len), 256, 0, st>>>(len, 1.0, v, 1.0, t, v);
    if (it >= kPowerSteps - 2) k_seg_sumsq<<<N, 256, 0, st>>>(d_voff.p, v, sq.p + (it - (kPowerSteps - 2)) * N);
  }
  HIP_CHECK(hipGetLastError());
  std::vector<double> h(2 * (size_t)N, 0.0);
  if (any_ok) HIP_CHECK(hipMemcpyAsync(h.data(), sq.p, sizeof(double) * 2 * N, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  check_device_error(ctx);
  std::vector<MatDesc> d32, d64;
  double rho_max = 0.0;
  for (int32_t i = 0; i < N; ++i) {
    double rho = h[i] > 0.0 ? std::sqrt(h[N + i] / h[i]) : (h[N + i] > 0.0 ? INFINITY : 0.0);
    if (failed[i] || !any_ok) rho = INFINITY;
    rho_max = std::max(rho_max, std::isfinite(rho) ? rho : INFINITY);
    (rho <= pc->opts.fp32_rho_max ? d32 : d64).push_back(descs[i]);
  }
  pc->info.fp32_rho_est = rho_max;
  // with fewer than 1 in 8 subdomains left on FP32 factors the mixed apply's
  // fixed cost (the FP64 residual and the second solve pass over the whole
  // batch) exceeds what the FP32 solves save: every subdomain goes to FP64
  if (!d32.empty() && (int64_t)d32.size() * kFp32MinShare < N) {
    d64 = descs;
    d32.clear();
  }
  pc->n_fallback = (int32_t)d64.size();
  pc->info.fp64_fallbacks = pc->n_fallback;
  if (d64.empty()) return;
  auto renumber = [](std::vector<MatDesc>& d) {
    int32_t f = 0;
    for (auto& m : d) {
      m.flag_off = f;
      f += m.nblk;
    }
    return f;
  };
  const int32_t f32 = renumber(d32), f64 = renumber(d64);
  if (!d32.empty()) pc->local32.build(d32, st, GENEO_FP32_REFINE1);
  pc->local64.build(d64, st, GENEO_FP64);
  pc->local32.solve_form = pc->local64.solve_form = false;
  (void)f32;
  (void)f64;
  // FP64 copies of the fallback matrices (extraction of every block is one
  // cheap pass; only the fallback subset is factored)
  const MatDesc& last = descs.back();
  const int64_t total = last.off + (int64_t)last.ld * last.ld;
  const int64_t inv_total = last.inv_off + 2 * (int64_t)last.ld * NB;
  pc->dL.alloc(total);
  pc->dLinv.alloc(inv_total);
  k_fill_identity_pad<<<fill_grid(descs), 256, 0, st>>>(pc->local.d_desc.p, pc->dL.p, nullptr);
  const int64_t nnz = pc->lnnz_off[N];
  if (nnz)
    k_dense_scatter<<<nblocks(nnz), 256, 0, st>>>(nnz, pc->d_lrow.p, pc->d_lcol.p, pc->d_lslot.p, pc->d_lnnz_off.p,
                                                  N, pc->local.d_desc.p, s->d_val.p, pc->dL.p, nullptr);
  HIP_CHECK(hipGetLastError());
  factor(pc->local64, pc->dL.p, pc->dLinv.p, nullptr, 0.0, nullptr, ctx->d_err, st);
  std::vector<int8_t> refine(len, 0);
  for (const auto& m : d32)
    for (int64_t r = 0; r < m.ld; ++r) refine[m.voff + r] = 1;
  pc->d_refine.upload(refine, st);
  HIP_CHECK(hipStreamSynchronize(st));
}

// Columns of one node n, R_i^T D_i G_i(:, n) over the subdomains i that
// contain n, live on the (at most 14) edges at n, and many are linearly
// dependent there (e.g. all D_i constant around n).  Their span is
// unchanged if, group by group, a column whose Gram-Schmidt residual
// against the earlier kept columns of its group is below 1e-8 of its norm
// is left out; the pivoted coarse factorisation then only has to find the
// (few) dependences that span several nodes.  Keeps the original column
// order; rewrites the CSC arrays in place.
static void snk_local_basis(int64_t n_nodes, std::vector<int32_t>& cp, std::vector<int32_t>& ri,
                            std::vector<double>& va, const std::vector<int32_t>& node, std::vector<int32_t>& sub) {
  const int64_t nc = (int64_t)cp.size() - 1;
  std::vector<int64_t> gp(n_nodes + 1, 0);
  for (int64_t c = 0; c < nc; ++c) gp[node[c] + 1]++;
  for (int64_t v = 0; v < n_nodes; ++v) gp[v + 1] += gp[v];
  std::vector<int64_t> gc(nc);
  {
    std::vector<int64_t> f(gp.begin(), gp.end() - 1);
    for (int64_t c = 0; c < nc; ++c) gc[f[node[c]]++] = c;   // ascending column order within a group
  }
  std::vector<uint8_t> keep(nc, 0);
  std::vector<int32_t> edges;
  std::vector<double> basis, u;
  for (int64_t v = 0; v < n_nodes; ++v) {
    const int64_t b = gp[v], e = gp[v + 1];
    if (b == e) continue;
    edges.clear();
    for (int64_t t = b; t < e; ++t)
      for (int32_t k = cp[gc[t]]; k < cp[gc[t] + 1]; ++k) edges.push_back(ri[k]);
    std::sort(edges.begin(), edges.end());
    edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
    const size_t m = edges.size();
    basis.clear();
    int nb = 0;
    for (int64_t t = b; t < e; ++t) {
      const int64_t c = gc[t];
      u.assign(m, 0.0);
      for (int32_t k = cp[c]; k < cp[c + 1]; ++k)
        u[std::lower_bound(edges.begin(), edges.end(), ri[k]) - edges.begin()] += va[k];
      double n0 = 0.0;
      for (double x : u) n0 += x * x;
      if (!(n0 > 0.0)) continue;
      for (int pass = 0; pass < 2; ++pass)
        for (int q = 0; q < nb; ++q) {
          const double* w = basis.data() + (size_t)q * m;
          double d = 0.0;
          for (size_t i = 0; i < m; ++i) d += w[i] * u[i];
          for (size_t i = 0; i < m; ++i) u[i] -= d * w[i];
        }
      double nr = 0.0;
      for (double x : u) nr += x * x;
      if (!(nr > 1e-16 * n0)) continue;   // residual below 1e-8 of the norm
      nr = std::sqrt(nr);
      for (double& x : u) x /= nr;
      basis.insert(basis.end(), u.begin(), u.end());
      ++nb;
      keep[c] = 1;
    }
  }
  std::vector<int32_t> cp2(1, 0), ri2, sub2;
  std::vector<double> va2;
  for (int64_t c = 0; c < nc; ++c) {
    if (!keep[c]) continue;
    sub2.push_back(sub[c]);
    for (int32_t k = cp[c]; k < cp[c + 1]; ++k) {
      ri2.push_back(ri[k]);
      va2.push_back(va[k]);
    }
    cp2.push_back((int32_t)ri2.size());
  }
  cp.swap(cp2);
  ri.swap(ri2);
  va.swap(va2);
  sub.swap(sub2);
}

// Host part of the SNK coarse columns R_i^T D_i G_i: sparse columns (one
// per kept local free node, subdomain-major), exactly dependent ones dropped
// within their node's group, and the row-wise transpose.
struct SnkHost {
  std::vector<int32_t> zc_ptr{0}, zc_row, col_node, col_sub, zr_ptr, zr_col;
  std::vector<double> zc_val, zr_val;
  int32_t n_all = 0;
};

static void build_snk_host(const geneo_system* s, const geneo_decomp* dec, SnkHost& h) {
  const int32_t N = dec->N;
  const int64_t n = s->n;
  std::vector<int32_t>& zc_ptr = h.zc_ptr;
  std::vector<int32_t>& zc_row = h.zc_row;
  std::vector<double>& zc_val = h.zc_val;
  {
    std::vector<int32_t> gl(s->n_free_nodes, -1);
    for (int32_t i = 0; i < N; ++i) {
      const int64_t gb = dec->gn_ptr[i], ge = dec->gn_ptr[i + 1];
      const int32_t base = (int32_t)(zc_ptr.size() - 1);
      for (int64_t k = gb; k < ge; ++k) gl[dec->gnodes[k]] = base + (int32_t)(k - gb);
      const int64_t nk = ge - gb;
      std::vector<std::vector<std::pair<int32_t, double>>> cols(nk);
      for (int64_t r = dec->dofs_ptr[i]; r < dec->dofs_ptr[i + 1]; ++r) {
        const int32_t fe = dec->dofs[r];
        const int32_t e = s->free_edges[fe];
        for (int q = 0; q < 2; ++q) {
          const int32_t fnode = s->node_to_free[s->edges[2 * (int64_t)e + q]];
          if (fnode < 0) continue;
          const int32_t c = gl[fnode];
          if (c < 0) continue;
          const double g = q == 0 ? -1.0 : 1.0;
          cols[c - base].push_back({fe, dec->pou[r] * g});
        }
      }
      for (int64_t k = 0; k < nk; ++k) {
        for (auto& pr : cols[k]) {
          zc_row.push_back(pr.first);
          zc_val.push_back(pr.second);
        }
        zc_ptr.push_back((int32_t)zc_row.size());
        h.col_node.push_back(dec->gnodes[gb + k]);
        h.col_sub.push_back(i);
      }
      for (int64_t k = gb; k < ge; ++k) gl[dec->gnodes[k]] = -1;
    }
  }
  h.n_all = (int32_t)(zc_ptr.size() - 1);
  static const bool local_basis = [] {
    const char* e = std::getenv("GENEO_SNK_LOCAL");
    return !(e && std::string(e) == "0");
  }();
  if (local_basis) snk_local_basis(s->n_free_nodes, zc_ptr, zc_row, zc_val, h.col_node, h.col_sub);
  const int32_t nsnk = (int32_t)(zc_ptr.size() - 1);
  // SNK rows (transpose of the columns)
  h.zr_ptr.assign(n + 1, 0);
  h.zr_col.resize(zc_row.size());
  h.zr_val.resize(zc_row.size());
  for (auto e : zc_row) h.zr_ptr[e + 1]++;
  for (int64_t e = 0; e < n; ++e) h.zr_ptr[e + 1] += h.zr_ptr[e];
  std::vector<int32_t> f(h.zr_ptr.begin(), h.zr_ptr.end() - 1);
  for (int32_t c = 0; c < nsnk; ++c)
    for (int32_t k = zc_ptr[c]; k < zc_ptr[c + 1]; ++k) {
      h.zr_col[f[zc_row[k]]] = c;
      h.zr_val[f[zc_row[k]]++] = zc_val[k];
    }
}

// Host-side phase clock of the setup (GENEO_VERBOSE set: printed to stderr).

// Global near-kernel columns Z = G (Section 4, Numerical results, the NK
// variants): one column per free node, -1 / +1 on the free edges that leave /
// enter it; no subdomain owns a column (col_sub = -1).
static void build_nk_host(const geneo_system* s, SnkHost& h) {
  const int64_t n = s->n, p = s->n_free_nodes;
  std::vector<int32_t> cnt(p + 1, 0);
  for (int64_t fe = 0; fe < n; ++fe) {
    const int32_t e = s->free_edges[fe];
    for (int q = 0; q < 2; ++q) {
      const int32_t v = s->node_to_free[s->edges[2 * (int64_t)e + q]];
      if (v >= 0) cnt[v + 1]++;
    }
  }
  for (int64_t v = 0; v < p; ++v) cnt[v + 1] += cnt[v];
  h.zc_ptr = cnt;
  h.zc_row.assign(cnt[p], 0);
  h.zc_val.assign(cnt[p], 0.0);
  std::vector<int32_t> f(cnt.begin(), cnt.end() - 1);
  for (int64_t fe = 0; fe < n; ++fe) {   // rows ascending within every column
    const int32_t e = s->free_edges[fe];
    for (int q = 0; q < 2; ++q) {
      const int32_t v = s->node_to_free[s->edges[2 * (int64_t)e + q]];
      if (v < 0) continue;
      h.zc_row[f[v]] = (int32_t)fe;
      h.zc_val[f[v]++] = q == 0 ? -1.0 : 1.0;
    }
  }
  h.col_node.resize(p);
  for (int64_t v = 0; v < p; ++v) h.col_node[v] = (int32_t)v;
  h.col_sub.assign(p, -1);
  h.n_all = (int32_t)p;
  h.zr_ptr.assign(n + 1, 0);
  h.zr_col.resize(h.zc_row.size());
  h.zr_val.resize(h.zc_row.size());
  for (auto e : h.zc_row) h.zr_ptr[e + 1]++;
  for (int64_t e = 0; e < n; ++e) h.zr_ptr[e + 1] += h.zr_ptr[e];
  std::vector<int32_t> g(h.zr_ptr.begin(), h.zr_ptr.end() - 1);
  for (int64_t c = 0; c < p; ++c)
    for (int32_t k = h.zc_ptr[c]; k < h.zc_ptr[c + 1]; ++k) {
      h.zr_col[g[h.zc_row[k]]] = (int32_t)c;
      h.zr_val[g[h.zc_row[k]]++] = h.zc_val[k];
    }
}

// Smallest eigenvalue, in the scaling of its diagonal, that the factored
// coarse matrix may have before its dependent columns are eliminated again
// with a larger tolerance: a kept block whose eigenvalue lies below this
// is numerically singular in FP64 (the coarse solve amplifies the rounding
// of its right-hand side by more than 1 / kCoarseLambdaFloor).
constexpr double kCoarseLambdaFloor = 1e-20;
constexpr int kCoarseMaxRefactors = 4;

// y = sqrt(d) .* x (entries with d <= 0: 0)
__global__ void k_sqrt_scale(int64_t n, const double* __restrict__ d, const double* __restrict__ x,
                             double* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = d[i] > 0.0 ? sqrt(d[i]) * x[i] : 0.0;
}
// x[i] = uniform(-1, 1) from a hash of i (start vector of the estimate)
__global__ void k_hash_fill(int64_t n, uint64_t seed, double* __restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  x[i] = (double)(z >> 11) * 0x1p-52 - 1.0;
}

// Estimate of the smallest eigenvalue of S E_kept S (S = diag(E)^-1/2, E_kept:
// the columns the factorisation kept; the others solve to 0): four steps of
// power iteration on its inverse S^-1 E_kept^-1 S^-1, applied with the
// factor's triangular solves; returns 1 / (the last Rayleigh quotient), an
// upper bound of the smallest eigenvalue that is tight once the iteration
// has settled on the inverse's dominant direction.
__global__ void k_scale_dev(int64_t n, const double* __restrict__ ap, int inv, const double* __restrict__ x,
                            double* __restrict__ out);

static double coarse_lambda_min(geneo_ctx* ctx, const geneo_precond* pc, int64_t n0p) {
  hipStream_t st = ctx->stream;
  DevBuf<double> v, w, part, S;
  v.alloc(n0p);
  w.alloc(n0p);
  part.alloc(kDotBlocks);
  S.alloc(2);
  double h[2] = {0.0, 0.0};
  k_hash_fill<<<nblocks(n0p), 256, 0, st>>>(n0p, 0x2311ull, v.p);
  dot(v.p, v.p, n0p, part.p, S.p + 1, st);
  k_scale_dev<<<nblocks(n0p), 256, 0, st>>>(n0p, S.p + 1, 1, v.p, v.p);   // ||v|| = 1
  double rq = 0.0;
  for (int it = 0; it < 4; ++it) {
    // w = S^-1 E^-1 S^-1 v with S^-1 = diag(E)^1/2
    k_sqrt_scale<<<nblocks(n0p), 256, 0, st>>>(n0p, pc->d_odiag.p, v.p, w.p);
    solve(pc->coarse, pc->dE.p, pc->dEinv.p, w.p, ctx->d_sync, ctx->d_err, st);
    k_sqrt_scale<<<nblocks(n0p), 256, 0, st>>>(n0p, pc->d_odiag.p, w.p, w.p);
    dot(v.p, w.p, n0p, part.p, S.p, st);
    dot(w.p, w.p, n0p, part.p, S.p + 1, st);
    HIP_CHECK(hipMemcpyAsync(h, S.p, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    rq = h[0];   // v^T (S^-1 E^-1 S^-1) v, ||v|| = 1
    if (!std::isfinite(h[0]) || !std::isfinite(h[1]) || !(h[1] > 0.0)) return 0.0;
    if (it == 3) break;
    k_scale_dev<<<nblocks(n0p), 256, 0, st>>>(n0p, S.p + 1, 1, w.p, v.p);   // v = w / ||w||
  }
  check_device_error(ctx);
  return rq > 0.0 ? 1.0 / rq : 0.0;
}

void setup_precond(geneo_ctx* ctx, geneo_precond* pc) {
  HostClock hc;
  hipStream_t st = ctx->stream;
  const geneo_system* s = pc->sys;
  const geneo_decomp* dec = pc->dec;
  const int32_t N = dec->N;
  const int64_t n = s->n;
  pc->N = N;
  pc->precision = pc->opts.local_precision;
  if (pc->precision != GENEO_FP64 && pc->precision != GENEO_FP32_REFINE1)
    throw Error(GENEO_EINVAL, "unknown local precision");
  if (pc->opts.coarse < GENEO_COARSE_SNK_GENEO || pc->opts.coarse > GENEO_COARSE_NK_GENEO)
    throw Error(GENEO_EINVAL, "unknown coarse space");
  if (pc->opts.one_level_weight != GENEO_WEIGHT_IDENTITY && pc->opts.one_level_weight != GENEO_WEIGHT_POU)
    throw Error(GENEO_EINVAL, "unknown one-level weight");
  if (pc->opts.classical != 0 && pc->opts.classical != 1) throw Error(GENEO_EINVAL, "classical must be 0 or 1");
  const bool nk = pc->opts.coarse == GENEO_COARSE_NK || pc->opts.coarse == GENEO_COARSE_NK_GENEO;
  const bool with_geneo = pc->opts.coarse == GENEO_COARSE_SNK_GENEO || pc->opts.coarse == GENEO_COARSE_NK_GENEO;

  // ---- batch layout of the local matrices
  std::vector<MatDesc> descs(N);
  int64_t off = 0, inv_off = 0, voff = 0;
  int32_t flag_off = 0;
  pc->voff.assign(N + 1, 0);
  double flops = 0;
  for (int32_t i = 0; i < N; ++i) {
    const int64_t ni = dec->dofs_ptr[i + 1] - dec->dofs_ptr[i];
    const int64_t np = round_up(std::max<int64_t>(ni, 1), NB);
    descs[i] = MatDesc{off, inv_off, -1, voff, (int32_t)np, (int32_t)(np / NB), flag_off, (int32_t)ni};
    off += np * np;
    inv_off += 2 * np * NB;
    pc->voff[i] = voff;
    voff += np;
    flag_off += (int32_t)(np / NB);
    flops += (double)ni * ni * ni / 3.0;
  }
  pc->voff[N] = voff;
  pc->batch_len = voff;
  pc->info.local_factor_flops = flops;
  pc->local.build(descs, st, pc->precision);
  pc->local.solve_form = false;   // bandwidth-bound local solves: no premultiplied blocks
  hc.mark("layout + local plan");
  pc->d_flags_local.alloc(flag_off);
  HIP_CHECK(hipMemsetAsync(pc->d_flags_local.p, 0, sizeof(unsigned) * flag_off, st));

  // batch maps
  std::vector<int32_t> bmap(voff, -1);
  std::vector<double> bpou(voff, 0.0);
  std::vector<int32_t> cnt(n + 1, 0);
  for (int32_t i = 0; i < N; ++i)
    for (int64_t r = dec->dofs_ptr[i]; r < dec->dofs_ptr[i + 1]; ++r) {
      int64_t k = pc->voff[i] + (r - dec->dofs_ptr[i]);
      bmap[k] = dec->dofs[r];
      bpou[k] = dec->pou[r];
      cnt[dec->dofs[r] + 1]++;
    }
  for (int64_t e = 0; e < n; ++e) cnt[e + 1] += cnt[e];
  std::vector<int32_t> inv(cnt[n]);
  {
    std::vector<int32_t> f(cnt.begin(), cnt.end() - 1);
    for (int32_t i = 0; i < N; ++i)
      for (int64_t r = dec->dofs_ptr[i]; r < dec->dofs_ptr[i + 1]; ++r)
        inv[f[dec->dofs[r]]++] = (int32_t)(pc->voff[i] + (r - dec->dofs_ptr[i]));
  }
  pc->d_bmap.upload(bmap, st);
  pc->d_bpou.upload(bpou, st);
  pc->d_inv_ptr.upload(cnt, st);
  pc->d_inv_idx.upload(inv, st);
  hc.mark("batch maps");

  // local CSR triplets: rows/cols local, slot = global CSR position (one
  // pass counts, one fills; subdomains in parallel)
  std::vector<int64_t> lnnz_off(N + 1, 0);
  auto local_triplets = [&](int32_t i, int32_t* lr, int32_t* lc, int32_t* ls) {
    // global -> local map, one per thread, reset to -1 after each subdomain
    thread_local std::vector<int32_t> g2l;
    if ((int64_t)g2l.size() < n) g2l.assign(n, -1);
    const int64_t b = dec->dofs_ptr[i], e = dec->dofs_ptr[i + 1];
    for (int64_t r = b; r < e; ++r) g2l[dec->dofs[r]] = (int32_t)(r - b);
    int64_t cnt = 0;
    for (int64_t r = b; r < e; ++r) {
      const int32_t ge = dec->dofs[r];
      for (int32_t sl = s->rowptr[ge]; sl < s->rowptr[ge + 1]; ++sl) {
        const int32_t c = g2l[s->colind[sl]];
        if (c < 0) continue;
        if (lr) {
          lr[cnt] = (int32_t)(r - b);
          lc[cnt] = c;
          ls[cnt] = sl;
        }
        ++cnt;
      }
    }
    for (int64_t r = b; r < e; ++r) g2l[dec->dofs[r]] = -1;
    return cnt;
  };
  parallel_for(N, [&](int i) { lnnz_off[i + 1] = local_triplets(i, nullptr, nullptr, nullptr); });
  for (int32_t i = 0; i < N; ++i) lnnz_off[i + 1] += lnnz_off[i];
  // every entry is written by the fill pass below (no zero-fill first)
  pc->h_lrow.resize(lnnz_off[N]);
  pc->h_lcol.resize(lnnz_off[N]);
  HostVec<int32_t>& lrow = pc->h_lrow;
  HostVec<int32_t>& lcol = pc->h_lcol;
  HostVec<int32_t> lslot(lnnz_off[N]);
  parallel_for(N, [&](int i) {
    local_triplets(i, lrow.data() + lnnz_off[i], lcol.data() + lnnz_off[i], lslot.data() + lnnz_off[i]);
  });
  pc->lnnz_off = lnnz_off;
  if (pc->precision == GENEO_FP32_REFINE1) {
    // FP64 residuals of the refinement step: the triplets come row by row,
    // batch-row pointers and batch columns (slots are d_lslot)
    std::vector<int64_t> brp(voff + 1, 0);
    HostVec<int32_t> bcol(lrow.size());   // every entry written below
    parallel_for(N, [&](int i) {
      for (int64_t t = lnnz_off[i]; t < lnnz_off[i + 1]; ++t) {
        brp[pc->voff[i] + lrow[t] + 1]++;
        bcol[t] = (int32_t)(pc->voff[i] + lcol[t]);
      }
    });
    for (int64_t r = 0; r < voff; ++r) brp[r + 1] += brp[r];
    pc->d_brp.upload(brp, st);
    pc->d_bcol.upload(bcol, st);
  }
  hc.mark("local triplets");
  pc->d_lrow.upload(lrow, st);
  pc->d_lcol.upload(lcol, st);
  pc->d_lslot.upload(lslot, st);
  pc->d_lnnz_off.upload(lnnz_off, st);
  hc.mark("local triplets uploaded");

  // the SNK columns depend on the mesh and the decomposition only
  SnkHost snk;
  std::exception_ptr snk_err;
  std::thread snk_thread;
  std::vector<std::vector<int32_t>> sub_order;   // elimination order of the subdomain groups of coarse columns
  int nd_levels = 0;
  std::vector<std::vector<int32_t>> sub_adj;   // subdomain coupling graph (for the AUTO choice)
  if (pc->opts.coarse_order != GENEO_ORDER_NESTED_DISSECTION && pc->opts.coarse_order != GENEO_ORDER_NATURAL &&
      pc->opts.coarse_order != GENEO_ORDER_AUTO)
    throw Error(GENEO_EINVAL, "unknown coarse order");
  if (pc->opts.coarse_schedule != GENEO_SCHEDULE_AUTO && pc->opts.coarse_schedule != GENEO_SCHEDULE_STEPS &&
      pc->opts.coarse_schedule != GENEO_SCHEDULE_LEVELS)
    throw Error(GENEO_EINVAL, "unknown coarse schedule");
  if (pc->opts.coarse != GENEO_COARSE_NONE)
    snk_thread = std::thread([&] {
      try {
        if (nk)
          build_nk_host(s, snk);
        else
          build_snk_host(s, dec, snk);
        // NK columns belong to no subdomain: natural order
        if (pc->opts.coarse_order != GENEO_ORDER_NATURAL && !nk)
          sub_order = subdomain_elimination_order(s, dec, &nd_levels, &sub_adj);
      } catch (...) {
        snk_err = std::current_exception();
      }
    });
  struct Joiner {   // joined on every exit path (errors included)
    std::thread& t;
    ~Joiner() {
      if (t.joinable()) t.join();
    }
  } snk_join{snk_thread};

  hc.mark("snk thread start");
  // ---- extraction + factorisation
  const bool fp32 = pc->precision == GENEO_FP32_REFINE1;
  if (fp32) {
    pc->fL.alloc(off);
    pc->fLinv.alloc(inv_off);
  } else {
    pc->dL.alloc(off);
    pc->dLinv.alloc(inv_off);
  }
  // the local phase's events are read only after the eigensolver's host
  // planning, which so runs while the device factors
  struct PhaseEvents {
    hipEvent_t e[3] = {nullptr, nullptr, nullptr};
    ~PhaseEvents() {
      for (auto& x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } lev;
  for (auto& x : lev.e) HIP_CHECK(hipEventCreate(&x));
  hc.mark("local buffers");
  HIP_CHECK(hipEventRecord(lev.e[0], st));
  k_fill_identity_pad<<<fill_grid(pc->local.h_desc), 256, 0, st>>>(pc->local.d_desc.p, fp32 ? nullptr : pc->dL.p,
                                                                   fp32 ? pc->fL.p : nullptr);
  if (!lrow.empty())
    k_dense_scatter<<<nblocks((int64_t)lrow.size()), 256, 0, st>>>((int64_t)lrow.size(), pc->d_lrow.p, pc->d_lcol.p,
                                                                   pc->d_lslot.p, pc->d_lnnz_off.p, N,
                                                                   pc->local.d_desc.p, s->d_val.p,
                                                                   fp32 ? nullptr : pc->dL.p, fp32 ? pc->fL.p : nullptr);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipEventRecord(lev.e[1], st));
  // work vectors
  pc->w_b1.alloc(voff);
  pc->w_b2.alloc(voff);
  pc->w_b3.alloc(voff);
  if (fp32) {
    // an FP32 factor that meets a non-positive pivot is flagged, not fatal:
    // that subdomain falls back to FP64
    DevBuf<int32_t> failed, c_smp, c_pair, c_slot;
    DevBuf<int8_t> c_w;
    DevBuf<double> klb;
    failed.alloc(N);
    klb.alloc(N);
    const Fp32Check chk = fp32_check_plan(s, dec);
    c_smp.upload(chk.smp_off, st);
    c_pair.upload(chk.pair_off, st);
    c_slot.upload(chk.slot, st);
    c_w.upload(chk.w, st);
    const double rho_max = pc->opts.fp32_rho_max;
    const double q_floor = rho_max > 0.0 ? kFp32RhoPerBound * 0x1p-24 / rho_max : INFINITY;
    k_fp32_check<<<N, 256, 0, st>>>(c_smp.p, c_pair.p, c_slot.p, c_w.p, s->d_val.p, q_floor, failed.p, klb.p);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipEventRecord(ctx->ev[2], st));
    factor(pc->local, pc->fL.p, pc->fLinv.p, nullptr, 0.0, nullptr, ctx->d_err, st, failed.p);
    HIP_CHECK(hipEventRecord(ctx->ev[3], st));
    check_device_error(ctx);
    pc->info.t_factor_fp32_ms = elapsed(ctx, 2, 3);
    fp32_probe(ctx, pc, descs, failed.p, klb.p);
  } else {
    factor(pc->local, pc->dL.p, pc->dLinv.p, nullptr, 0.0, nullptr, ctx->d_err, st);
  }
  HIP_CHECK(hipEventRecord(lev.e[2], st));
  hc.mark("local factor queued");

  pc->w_n1.alloc(n);
  pc->w_n2.alloc(n);
  pc->w_n3.alloc(n);
  pc->w_n4.alloc(n);

  // ---- GenEO eigenproblems
  pc->gen_cnt.assign(N, 0);
  pc->gen_off.assign(N + 1, 0);
  pc->eigs.assign(N, {});
  pc->eig_sel.assign(N, 0);
  if (with_geneo) {
    HIP_CHECK(hipEventRecord(ctx->ev[0], st));
    solve_local_gevps(ctx, pc);
    HIP_CHECK(hipEventRecord(ctx->ev[1], st));
    pc->info.t_gevp_ms = elapsed(ctx, 0, 1);
    hc.mark("gevp done");
  }
  {
    float ms = 0;
    HIP_CHECK(hipEventSynchronize(lev.e[2]));
    HIP_CHECK(hipEventElapsedTime(&ms, lev.e[0], lev.e[1]));
    pc->info.t_extract_ms = ms;
    HIP_CHECK(hipEventElapsedTime(&ms, lev.e[1], lev.e[2]));
    pc->info.t_factor_ms = ms;
  }
  check_device_error(ctx);   // a local factor's error surfaces here at the latest
  if (pc->opts.coarse == GENEO_COARSE_NONE) {
    pc->n0 = 0;
    return;
  }

  // ---- coarse space: SNK columns R_i^T D_i G_i (one per kept local free node),
  // built on a host thread while the device ran the factorisations and GEVPs
  snk_thread.join();
  hc.mark("snk thread joined");
  if (snk_err) std::rethrow_exception(snk_err);
  std::vector<int32_t>& zc_ptr = snk.zc_ptr;
  std::vector<int32_t>& zc_row = snk.zc_row;
  std::vector<double>& zc_val = snk.zc_val;
  std::vector<int32_t>& col_sub = snk.col_sub;
  std::vector<int32_t>& zr_ptr = snk.zr_ptr;
  std::vector<int32_t>& zr_col = snk.zr_col;
  std::vector<double>& zr_val = snk.zr_val;
  pc->n_snk_all = snk.n_all;
  pc->n_snk = (int32_t)(zc_ptr.size() - 1);
  pc->info.n0_local_dropped = pc->n_snk_all - pc->n_snk;
  pc->n_gen = 0;
  for (int32_t i = 0; i < N; ++i) {
    pc->gen_off[i] = pc->n_gen;
    pc->n_gen += pc->gen_cnt[i];
  }
  pc->gen_off[N] = pc->n_gen;
  pc->n0 = pc->n_snk + pc->n_gen;
  pc->d_zc_ptr.upload(zc_ptr, st);
  pc->d_zc_row.upload(zc_row, st);
  pc->d_zc_val.upload(zc_val, st);
  pc->d_zr_ptr.upload(zr_ptr, st);
  pc->d_zr_col.upload(zr_col, st);
  pc->d_zr_val.upload(zr_val, st);

  // ---- order of the coarse columns in the factor: the subdomains of every
  // nested-dissection group with their SNK columns, then their GenEO columns;
  // each group starts at a multiple of 128 (unit pad columns in between), so
  // groups that the dissection separates share no 128 x 128 tile
  std::vector<int32_t> pad_pos;
  int64_t n0_fac = pc->n0;          // order size with the pads
  std::vector<int64_t> snk_beg(N + 1, 0);
  if (!sub_order.empty()) {
    for (int32_t c = 0; c < pc->n_snk; ++c) snk_beg[col_sub[c] + 1]++;
    for (int32_t i = 0; i < N; ++i) snk_beg[i + 1] += snk_beg[i];
  }
  if (!sub_order.empty() && pc->opts.coarse_order == GENEO_ORDER_AUTO) {
    // the dependency chain of the solves: the natural order's is its block-row
    // count (every block row meets the previous one); nested dissection's is
    // predicted from the subdomain adjacency.  Dissection is kept where it
    // shortens the chain to 0.6 or less.
    std::vector<int32_t> pos_sub;
    pos_sub.reserve((size_t)pc->n0 + (size_t)NB * sub_order.size());
    for (const auto& grp : sub_order) {
      for (int32_t i : grp) pos_sub.insert(pos_sub.end(), (size_t)(snk_beg[i + 1] - snk_beg[i] + pc->gen_cnt[i]), i);
      while (pos_sub.size() % NB) pos_sub.push_back(-1);
    }
    const int pred = predicted_solve_depth(pos_sub, sub_adj);
    const int64_t natural_rows = (pc->n0 + NB - 1) / NB;
    pc->info.coarse_nd_predicted_depth = pred;
    if ((double)pred > 0.6 * (double)natural_rows) sub_order.clear();
  }
  if (!sub_order.empty()) {
    std::vector<int32_t> perm(pc->n0, -1);
    int64_t pos = 0;
    for (const auto& grp : sub_order) {
      for (int32_t i : grp) {
        for (int64_t c = snk_beg[i]; c < snk_beg[i + 1]; ++c) perm[c] = (int32_t)pos++;
        for (int32_t q = 0; q < pc->gen_cnt[i]; ++q) perm[pc->n_snk + pc->gen_off[i] + q] = (int32_t)pos++;
      }
      while (pos % NB) pad_pos.push_back((int32_t)pos++);
    }
    for (int32_t c = 0; c < pc->n0; ++c)
      if (perm[c] < 0) throw Error(GENEO_EINVAL, "coarse order does not cover every column");
    n0_fac = pos;
    pc->d_cperm.upload(perm, st);
    pc->info.coarse_nd_levels = nd_levels;
  }
  const int32_t* cperm = pc->d_cperm.p;

  // ---- E = Z^T A Z (dense FP64), then Cholesky with dependent columns left out
  const int64_t n0 = pc->n0;
  const int64_t n0p = round_up(std::max<int64_t>(n0_fac, 1), NB);
  std::vector<MatDesc> cd(1, MatDesc{0, 0, 0, 0, (int32_t)n0p, (int32_t)(n0p / NB), 0, (int32_t)n0_fac});
  pc->coarse.build(cd, st);
  pc->dE.alloc(n0p * n0p);
  pc->dEinv.alloc(2 * n0p * NB);
  pc->d_odiag.alloc(n0p);
  pc->d_pivrel.alloc(n0p);
  pc->w_c1.alloc(n0p);
  pc->w_c2.alloc(n0p);
  HIP_CHECK(hipMemsetAsync(pc->w_c1.p, 0, sizeof(double) * n0p, st));
  HIP_CHECK(hipMemsetAsync(pc->w_c2.p, 0, sizeof(double) * n0p, st));
  if (cperm) {
    pc->w_c3.alloc(n0p);
    HIP_CHECK(hipMemsetAsync(pc->w_c3.p, 0, sizeof(double) * n0p, st));
  }
  HIP_CHECK(hipEventRecord(ctx->ev[0], st));
  // block sparsity of E: only subdomains whose columns meet through A couple;
  // the factor touches the tiles of the symbolic fill of that pattern only.
  // The assembly marks every lower 128 x 128 tile it adds a non-zero to (tiles_E); E is
  // zeroed in its lower triangle only (the factorisation reads no other part).
  static const bool coarse_sparse = [] {
    const char* e = std::getenv("GENEO_COARSE_SPARSE");
    return !(e && std::string(e) == "0");
  }();
  const int nbc = (int)(n0p / NB);
  DevBuf<uint8_t> tiles_E;
  if (coarse_sparse && nbc > 1) {
    tiles_E.alloc((size_t)nbc * nbc);
    HIP_CHECK(hipMemsetAsync(tiles_E.p, 0, (size_t)nbc * nbc, st));
  }
  auto fill_E = [&] {
  k_fill_identity_pad<<<fill_grid(cd), 256, 0, st>>>(pc->coarse.d_desc.p, pc->dE.p, nullptr, 1);
  if (!pad_pos.empty()) {   // pad columns between the groups of the order: unit diagonal
    DevBuf<int32_t> d_pad;
    d_pad.upload(pad_pos, st);
    k_unit_diag<<<nblocks((int64_t)pad_pos.size()), 256, 0, st>>>((int64_t)pad_pos.size(), d_pad.p, pc->dE.p, n0p);
    HIP_CHECK(hipStreamSynchronize(st));
  }
  if (pc->n_snk)
    k_coarse_snk<<<nblocks(pc->n_snk), 256, 0, st>>>(pc->n_snk, pc->d_zc_ptr.p, pc->d_zc_row.p, pc->d_zc_val.p,
                                                      s->d_rowptr.p, s->d_colind.p, s->d_val.p, pc->d_zr_ptr.p,
                                                      pc->d_zr_col.p, pc->d_zr_val.p, cperm, pc->dE.p, n0p,
                                                      tiles_E.p, nbc);
  if (pc->n_gen) {
    // global dense GenEO columns and Y = A Z_gen
    DevBuf<double> Zg, Y;
    Zg.alloc((size_t)n * pc->n_gen);
    Y.alloc((size_t)n * pc->n_gen);
    HIP_CHECK(hipMemsetAsync(Zg.p, 0, sizeof(double) * n * pc->n_gen, st));
    k_zg_scatter<<<nblocks(voff), 256, 0, st>>>(voff, N, pc->d_voff.p, pc->d_n.p, pc->d_gen_cnt.p, pc->d_gen_off.p,
                                                pc->d_w_off.p, pc->d_bmap.p, pc->d_W.p, n, Zg.p);
    // supports: a GenEO column of subdomain j lives on its dofs, so A Z_gen
    // is non-zero only on ring_j (the dofs coupled to them through A) and
    // E(c1, g) only for columns c1 of subdomains i whose dofs meet ring_j
    const GenSupport sup = gen_support(s, dec, pc->gen_cnt, col_sub, pc->n_snk, pc->gen_off);
    DevBuf<int32_t> d_ring, d_ring_ptr, d_cand, d_cand_ptr;
    d_ring.upload(sup.ring, st);
    d_ring_ptr.upload(sup.ring_ptr, st);
    d_cand.upload(sup.cand, st);
    d_cand_ptr.upload(sup.cand_ptr, st);
    HIP_CHECK(hipMemsetAsync(Y.p, 0, sizeof(double) * n * pc->n_gen, st));
    if (!sup.ring.empty())
      k_spmm_ring<<<nblocks((int64_t)sup.ring.size()), 256, 0, st>>>(
          (int64_t)sup.ring.size(), N, d_ring_ptr.p, d_ring.p, pc->d_gen_cnt.p, pc->d_gen_off.p, s->d_rowptr.p,
          s->d_colind.p, s->d_val.p, n, Zg.p, Y.p);
    if (sup.max_cand > 0)
      k_coarse_gen<<<dim3((unsigned)((sup.max_cand + 255) / 256), (unsigned)pc->n_gen), 256, 0, st>>>(
          pc->n_snk, n, pc->d_zc_ptr.p, pc->d_zc_row.p, pc->d_zc_val.p, N, pc->d_gen_off.p, d_cand_ptr.p, d_cand.p,
          pc->d_voff.p, pc->d_n.p, pc->d_w_off.p, pc->d_bmap.p, pc->d_W.p, Y.p, cperm, pc->dE.p, n0p, tiles_E.p,
          nbc);
    HIP_CHECK(hipStreamSynchronize(st));
  }
  HIP_CHECK(hipGetLastError());
  {
    dim3 g(nblocks(n0p), 1);
    k_copy_diag<<<g, 256, 0, st>>>(pc->coarse.d_desc.p, pc->dE.p, pc->d_odiag.p);
  }
  };
  fill_E();
  // the coarse plan's diag_off is 0
  HIP_CHECK(hipEventRecord(ctx->ev[1], st));
  pc->info.coarse_factor_flops = (double)n0 * n0 * n0 / 3.0;
  pc->info.coarse_schedule_used = GENEO_SCHEDULE_STEPS;
  // a solve reads every factor tile once per sweep (the diagonal ones as their inverses)
  pc->info.coarse_solve_bytes = 2.0 * ((double)nbc * (nbc + 1) / 2) * NB * NB * sizeof(double);
  if (coarse_sparse && nbc > 1) {
    std::vector<uint8_t> pat((size_t)nbc * nbc);
    HIP_CHECK(hipMemcpyAsync(pat.data(), tiles_E.p, pat.size(), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    hc.mark("coarse E assembled");
    symbolic_fill(nbc, pat);
    hc.mark("coarse symbolic fill");
    pc->coarse.build_sparse(cd[0], pat, st, pc->opts.coarse_schedule);
    hc.mark("coarse plan");
    pc->info.coarse_levels = pc->coarse.n_levels;
    pc->info.coarse_schedule_used = pc->coarse.levels ? GENEO_SCHEDULE_LEVELS : GENEO_SCHEDULE_STEPS;
    pc->info.coarse_factor_flops = pc->coarse.sparse_flops;
    pc->info.coarse_fill = (double)pc->coarse.fill_tiles / ((double)nbc * (nbc + 1) / 2);
    pc->info.coarse_solve_bytes = 2.0 * (double)pc->coarse.fill_tiles * NB * NB * sizeof(double);
    std::vector<int32_t> depth(nbc, 1);
    int32_t dmax = nbc ? 1 : 0;
    for (int I = 0; I < nbc; ++I) {
      for (int J = 0; J < I; ++J)
        if (pat[(size_t)I * nbc + J]) depth[I] = std::max(depth[I], depth[J] + 1);
      dmax = std::max(dmax, depth[I]);
    }
    pc->info.coarse_solve_depth = dmax;
  }
  // Greedy elimination without pivoting is not rank revealing by itself: a
  // run of kept columns, each with a relative Schur pivot just above the
  // tolerance, can leave the kept block with an eigenvalue far below every
  // pivot (the factor's inverse grows along the run), and the coarse solve
  // then returns huge corrections.  The smallest eigenvalue of the kept block
  // in the scaling of E's diagonal is estimated after the factorisation; if
  // it is below kCoarseLambdaFloor the columns are eliminated again with a
  // tenfold tolerance (at most four times, up to 1e4 times the given one).
  double tol = pc->opts.coarse_drop_tol;
  pc->info.coarse_refactors = 0;
  for (int attempt = 0;; ++attempt) {
    factor(pc->coarse, pc->dE.p, pc->dEinv.p, pc->d_odiag.p, tol, pc->d_pivrel.p, ctx->d_err, st);
    if (attempt == 0) {
      HIP_CHECK(hipEventRecord(ctx->ev[2], st));
      hc.mark("coarse factor queued");
      pc->info.t_coarse_build_ms = elapsed(ctx, 0, 1);
      pc->info.t_coarse_factor_ms = elapsed(ctx, 1, 2);
    }
    check_device_error(ctx);
    pc->info.coarse_lambda_min = coarse_lambda_min(ctx, pc, n0p);
    if (tol <= 0.0 || pc->info.coarse_lambda_min >= kCoarseLambdaFloor || attempt == kCoarseMaxRefactors) break;
    tol *= 10.0;
    pc->info.coarse_refactors = attempt + 1;
    fill_E();
  }
  if (pc->info.coarse_refactors) {   // the estimate and the re-eliminations after the first factorisation
    HIP_CHECK(hipEventRecord(ctx->ev[3], st));
    HIP_CHECK(hipEventSynchronize(ctx->ev[3]));
    pc->info.t_coarse_refactor_ms = elapsed(ctx, 2, 3);
  }
  pc->info.coarse_drop_tol_used = tol;
  std::vector<double> piv(n0p);
  HIP_CHECK(hipMemcpy(piv.data(), pc->d_pivrel.p, sizeof(double) * n0p, hipMemcpyDeviceToHost));
  std::vector<int32_t> hperm;
  if (cperm) {
    hperm.resize(n0);
    HIP_CHECK(hipMemcpy(hperm.data(), cperm, sizeof(int32_t) * n0, hipMemcpyDeviceToHost));
  }
  int32_t kept = 0;
  double mink = 1e300, maxd = 0.0;
  for (int64_t c0 = 0; c0 < n0; ++c0) {
    const int64_t c = cperm ? hperm[c0] : c0;   // pivots are in the factor's order
    if (piv[c] > tol) {
      ++kept;
      mink = std::min(mink, piv[c]);
    } else {
      maxd = std::max(maxd, piv[c]);
    }
  }
  pc->info.n0 = pc->n_snk_all + pc->n_gen;
  pc->info.n0_rank = kept;
  pc->info.n_snk = pc->n_snk_all;
  pc->info.n_geneo = pc->n_gen;
  pc->info.min_kept_pivot = kept ? mink : 0.0;
  pc->info.max_dropped_pivot = maxd;
}

// ---------------------------------------------------------------- apply

__global__ void k_fill(int64_t n, double v, double* __restrict__ x) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// y[perm[i]] = x[i] (forward) or x[i] = y[perm[i]] (back), i < n
__global__ void k_permute(int64_t n, const int32_t* __restrict__ perm, int back, double* __restrict__ x,
                          double* __restrict__ y) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (back)
    x[i] = y[perm[i]];
  else
    y[perm[i]] = x[i];
}

static void coarse_solve(geneo_ctx* ctx, const geneo_precond* pc, double* c) {
  // pad rows of the coarse vector carry no data: clear them so that nothing
  // left there by an earlier call (e.g. a non-finite input) reaches the solve
  const int64_t n0p = pc->coarse.h_desc[0].ld;
  hipStream_t st = ctx->stream;
  // the triangular sweeps, timed by events when a PCG run asks for it
  const int t = ctx->cs_timing >= 0 && ctx->cs_timing < 2 ? ctx->cs_timing++ : -1;
  auto sweeps = [&](double* v) {
    if (t >= 0) HIP_CHECK(hipEventRecord(ctx->ev[4 + 2 * t], st));
    solve(pc->coarse, pc->dE.p, pc->dEinv.p, v, ctx->d_sync, ctx->d_err, st);
    if (t >= 0) HIP_CHECK(hipEventRecord(ctx->ev[5 + 2 * t], st));
  };
  if (pc->d_cperm.p) {   // the factor's order, pads between its groups
    double* v = pc->w_c3.p;
    k_fill<<<nblocks(n0p), 256, 0, st>>>(n0p, 0.0, v);
    k_permute<<<nblocks(pc->n0), 256, 0, st>>>(pc->n0, pc->d_cperm.p, 0, c, v);
    sweeps(v);
    k_permute<<<nblocks(pc->n0), 256, 0, st>>>(pc->n0, pc->d_cperm.p, 1, c, v);
    return;
  }
  if (n0p > pc->n0) k_fill<<<nblocks(n0p - pc->n0), 256, 0, st>>>(n0p - pc->n0, 0.0, c + pc->n0);
  sweeps(c);
}

// b <- A_i^-1 b on every segment; FP32 factors get one FP64 refinement step
static void local_solve(geneo_ctx* ctx, const geneo_precond* pc, double* b) {
  hipStream_t st = ctx->stream;
  if (pc->precision != GENEO_FP32_REFINE1) {
    solve(pc->local, pc->dL.p, pc->dLinv.p, b, ctx->d_sync, ctx->d_err, st);
    return;
  }
  const int64_t len = pc->batch_len;
  const FactorPlan& p32 = pc->n_fallback ? pc->local32 : pc->local;
  double* rhs = pc->w_b3.p;
  k_copy<<<nblocks(len), 256, 0, st>>>(len, b, rhs);
  if (p32.nmat) solve(p32, pc->fL.p, pc->fLinv.p, b, ctx->d_sync, ctx->d_err, st);
  if (pc->n_fallback)
    solve(pc->local64, pc->dL.p, pc->dLinv.p, b, ctx->d_sync, ctx->d_err, st);
  if (!p32.nmat) return;
  // rhs <- rhs - A_i yhat on the refined subdomains (0 elsewhere), then the correction
  k_local_residual<<<nblocks(len), 256, 0, st>>>(len, pc->d_brp.p, pc->d_bcol.p, pc->d_lslot.p, pc->sys->d_val.p, rhs,
                                                 b, pc->n_fallback ? pc->d_refine.p : nullptr, rhs);
  solve(p32, pc->fL.p, pc->fLinv.p, rhs, ctx->d_sync, ctx->d_err, st);
  k_axpby<<<nblocks(len), 256, 0, st>>>(len, 1.0, b, 1.0, rhs, b);
}

// t = Z^T g   (g: global vector; uses w_b2 for the GenEO part)
static void z_transpose(const geneo_precond* pc, const double* g, double* t, hipStream_t st) {
  const geneo_system* s = pc->sys;
  if (pc->n_snk)
    k_csc_t<<<nblocks(pc->n_snk), 256, 0, st>>>(pc->n_snk, pc->d_zc_ptr.p, pc->d_zc_row.p, pc->d_zc_val.p, g, t);
  if (pc->n_gen) {
    k_gather<<<nblocks(pc->batch_len), 256, 0, st>>>(pc->batch_len, pc->d_bmap.p, g, pc->w_b2.p);
    k_w_t<<<(unsigned)((pc->n_gen + 3) / 4), 256, 0, st>>>(pc->N, pc->d_gen_cnt.p, pc->d_gen_off.p, pc->d_w_off.p,
                                                           pc->d_voff.p, pc->d_n.p, pc->d_W.p, pc->w_b2.p,
                                                           t + pc->n_snk, pc->n_gen);
  }
  (void)s;
}

// u = Z c (+ add)
static void z_forward(const geneo_precond* pc, const double* c, const double* add, double* u, hipStream_t st) {
  const int64_t n = pc->sys->n;
  const double* base = add;
  if (pc->n_gen) {
    k_w_n<<<nblocks(pc->batch_len), 256, 0, st>>>(pc->batch_len, pc->N, pc->d_voff.p, pc->d_gen_cnt.p,
                                                  pc->d_gen_off.p, pc->d_w_off.p, pc->d_W.p, c + pc->n_snk,
                                                  pc->w_b2.p);
    k_scatter_add<<<nblocks(n), 256, 0, st>>>(n, pc->d_inv_ptr.p, pc->d_inv_idx.p, pc->w_b2.p, add, 1.0, u);
    base = u;
  }
  k_csr<<<nblocks(n), 256, 0, st>>>(n, pc->d_zr_ptr.p, pc->d_zr_col.p, pc->d_zr_val.p, c, base, u);
}

// x <- w .* x (the restricted one-level term: D_i on every local solution)
__global__ void k_mul(int64_t n, const double* __restrict__ w, double* __restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] *= w[i];
}

// b <- A_i^-1 b on every segment, times D_i with the restricted one-level term
static void local_term(geneo_ctx* ctx, const geneo_precond* pc, double* b) {
  local_solve(ctx, pc, b);
  if (pc->opts.one_level_weight == GENEO_WEIGHT_POU)
    k_mul<<<nblocks(pc->batch_len), 256, 0, ctx->stream>>>(pc->batch_len, pc->d_bpou.p, b);
}

void apply_precond(geneo_ctx* ctx, const geneo_precond* pc, const double* r, double* z) {
  hipStream_t st = ctx->stream;
  const int64_t n = pc->sys->n;
  double* y = pc->w_n1.p;
  if (pc->n0 == 0) {
    k_gather<<<nblocks(pc->batch_len), 256, 0, st>>>(pc->batch_len, pc->d_bmap.p, r, pc->w_b1.p);
    local_term(ctx, pc, pc->w_b1.p);
    k_scatter_add<<<nblocks(n), 256, 0, st>>>(n, pc->d_inv_ptr.p, pc->d_inv_idx.p, pc->w_b1.p, nullptr, 1.0, z);
    return;
  }
  double* c = pc->w_c1.p;
  double* c2 = pc->w_c2.p;
  // c = E^-1 Z^T r
  z_transpose(pc, r, c, st);
  coarse_solve(ctx, pc, c);
  // r1 = r - A Z c
  z_forward(pc, c, nullptr, pc->w_n2.p, st);
  launch_spmv(pc->sys, pc->w_n2.p, pc->w_n3.p, st);
  k_axpby<<<nblocks(n), 256, 0, st>>>(n, 1.0, r, -1.0, pc->w_n3.p, pc->w_n2.p);
  // y = sum_i R_i^T A_i^-1 R_i r1
  k_gather<<<nblocks(pc->batch_len), 256, 0, st>>>(pc->batch_len, pc->d_bmap.p, pc->w_n2.p, pc->w_b1.p);
  local_term(ctx, pc, pc->w_b1.p);
  k_scatter_add<<<nblocks(n), 256, 0, st>>>(n, pc->d_inv_ptr.p, pc->d_inv_idx.p, pc->w_b1.p, nullptr, 1.0, y);
  // c2 = E^-1 Z^T A y
  launch_spmv(pc->sys, y, pc->w_n3.p, st);
  z_transpose(pc, pc->w_n3.p, c2, st);
  coarse_solve(ctx, pc, c2);
  // z = y + Z (c - c2)
  k_axpby<<<nblocks(pc->n0), 256, 0, st>>>(pc->n0, 1.0, c, -1.0, c2, c2);
  z_forward(pc, c2, y, z, st);
}

// z = M_AS r + Q (r - A M_AS r), Q = Z E^-1 Z^T: the deflated form
// (I - Q A) M_AS + Q of the two-level preconditioner, one coarse solve per
// application.  PCG with it from x0 = Q b generates, in exact arithmetic,
// the iterates of PCG with M_AS,2 = Q + (I - Q A) M_AS (I - A Q) (eq. (AS2))
// from x0 = 0: every residual then satisfies Z^T r = 0, where the two
// operators agree (the "A-DEF2" form of Tang, Nabben, Vuik and Erlangga,
// 2009); its Q r term keeps rounding from accumulating in span(Z), which the
// form (I - Q A) M_AS alone does not.
static void apply_deflated(geneo_ctx* ctx, const geneo_precond* pc, const double* r, double* z) {
  if (pc->n0 == 0) {
    apply_precond(ctx, pc, r, z);
    return;
  }
  hipStream_t st = ctx->stream;
  const int64_t n = pc->sys->n;
  double* y = pc->w_n1.p;
  double* c = pc->w_c1.p;
  k_gather<<<nblocks(pc->batch_len), 256, 0, st>>>(pc->batch_len, pc->d_bmap.p, r, pc->w_b1.p);
  local_term(ctx, pc, pc->w_b1.p);
  k_scatter_add<<<nblocks(n), 256, 0, st>>>(n, pc->d_inv_ptr.p, pc->d_inv_idx.p, pc->w_b1.p, nullptr, 1.0, y);
  launch_spmv(pc->sys, y, pc->w_n3.p, st);
  k_axpby<<<nblocks(n), 256, 0, st>>>(n, 1.0, r, -1.0, pc->w_n3.p, pc->w_n2.p);   // r - A y
  z_transpose(pc, pc->w_n2.p, c, st);
  coarse_solve(ctx, pc, c);
  z_forward(pc, c, y, z, st);
}

// ---------------------------------------------------------------- PCG
// device scalars: 0 rz, 1 pq, 2 rr, 3 rz_new, 4 bb
__global__ void k_pcg_update(int64_t n, double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
                             const double* __restrict__ q, const double* __restrict__ S) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double alpha = S[0] / S[1];
  x[i] += alpha * p[i];
  r[i] -= alpha * q[i];
}
__global__ void k_pcg_dir(int64_t n, double* __restrict__ p, const double* __restrict__ z, double* __restrict__ S,
                          int first) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  p[i] = first ? z[i] : z[i] + (S[3] / S[0]) * p[i];
}
__global__ void k_pcg_shift(double* S) { S[0] = S[3]; }
// the device error record's status next to ||r||^2, so that one copy per
// iteration brings both to the host
__global__ void k_pcg_status(const DevErr* __restrict__ err, double* S) { S[5] = (double)err->code; }

void pcg(geneo_ctx* ctx, const geneo_system* sys, const geneo_precond* pc, const double* b, double* x,
         const geneo_solve_opts* o, geneo_solve_info* info) {
  const int64_t n = sys->n;
  // Graph mode runs the solve on a library stream of its own (a capture
  // cannot use the legacy default stream): it starts after the work queued
  // on the context stream and the context stream waits for its end.
  const bool use_graph = o->graph != 0;
  hipStream_t user = ctx->stream, gs = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  struct Restore {
    geneo_ctx* ctx;
    hipStream_t user, gs;
    hipEvent_t a, b;
    hipGraph_t& g;
    hipGraphExec_t& e;
    ~Restore() {
      if (gs) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(gs, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
          hipGraph_t tmp = nullptr;
          (void)hipStreamEndCapture(gs, &tmp);
          if (tmp) (void)hipGraphDestroy(tmp);
        }
        (void)hipStreamSynchronize(gs);
      }
      if (e) (void)hipGraphExecDestroy(e);
      if (g) (void)hipGraphDestroy(g);
      ctx->stream = user;
      if (gs) (void)hipStreamDestroy(gs);
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  };
  if (use_graph) {
    HIP_CHECK(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
    HIP_CHECK(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&ev_out, hipEventDisableTiming));
  }
  Restore restore{ctx, user, gs, ev_in, ev_out, graph, exec};
  if (use_graph) {
    HIP_CHECK(hipEventRecord(ev_in, user));
    HIP_CHECK(hipStreamWaitEvent(gs, ev_in, 0));
    ctx->stream = gs;
  }
  hipStream_t st = ctx->stream;
  DevBuf<double> r, z, p, q, part, S;
  r.alloc(n);
  z.alloc(n);
  p.alloc(n);
  q.alloc(n);
  part.alloc(kDotBlocks);
  S.alloc(8);
  double* h = nullptr;
  HIP_CHECK(hipHostMalloc((void**)&h, 8 * sizeof(double), hipHostMallocDefault));
  struct HostFree {
    double* p;
    ~HostFree() { if (p) (void)hipHostFree(p); }
  } hf{h};
  // the deflated form starts from x0 = Q b (r0 = b - A Q b, Z^T r0 = 0); its
  // two coarse solves (this one and the first application's) are timed
  const bool deflated = pc && pc->n0 > 0 && o->pcg_form == GENEO_PCG_DEFLATED;
  ctx->cs_timing = pc && pc->n0 > 0 ? 0 : -1;
  struct TimingOff {   // no later call records the coarse-solve events
    geneo_ctx* c;
    ~TimingOff() { c->cs_timing = -1; }
  } timing_off{ctx};
  HIP_CHECK(hipEventRecord(ctx->ev[0], st));
  if (deflated) {
    z_transpose(pc, b, pc->w_c1.p, st);
    coarse_solve(ctx, pc, pc->w_c1.p);
    z_forward(pc, pc->w_c1.p, nullptr, x, st);
    launch_spmv(sys, x, r.p, st);
    k_axpby<<<nblocks(n), 256, 0, st>>>(n, 1.0, b, -1.0, r.p, r.p);
  } else {
    HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * n, st));
    HIP_CHECK(hipMemcpyAsync(r.p, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  }
  dot(b, b, n, part.p, S.p + 4, st);
  HIP_CHECK(hipMemcpyAsync(h + 4, S.p + 4, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  const double bnorm = std::sqrt(h[4]);
  const double tol = o->rtol * bnorm;
  int it = 0, replays = 0;
  int64_t applies = 0;   // preconditioner applications run (graph captures excluded)
  bool capturing = false;
  double rel = 1.0;
  bool conv = bnorm == 0.0;
  if (!conv) {
    auto precond = [&](const double* in, double* out) {
      if (deflated)
        apply_deflated(ctx, pc, in, out);
      else if (pc)
        apply_precond(ctx, pc, in, out);
      else
        k_copy<<<nblocks(n), 256, 0, st>>>(n, in, out);
    };
    // z = M^-1 r, the new direction (end of one iteration) ...
    auto tail = [&](int first) {
      if (!capturing) ++applies;
      precond(r.p, z.p);
      dot(r.p, z.p, n, part.p, S.p + 3, st);
      k_pcg_dir<<<nblocks(n), 256, 0, st>>>(n, p.p, z.p, S.p, first);
      k_pcg_shift<<<1, 1, 0, st>>>(S.p);
    };
    // ... then q = A p, the step, ||r||^2 to the host (start of the next)
    auto head = [&] {
      launch_spmv(sys, p.p, q.p, st);
      dot(p.p, q.p, n, part.p, S.p + 1, st);
      k_pcg_update<<<nblocks(n), 256, 0, st>>>(n, x, r.p, p.p, q.p, S.p);
      dot(r.p, r.p, n, part.p, S.p + 2, st);
      k_pcg_status<<<1, 1, 0, st>>>(ctx->d_err, S.p);
      HIP_CHECK(hipMemcpyAsync(h + 2, S.p + 2, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    };
    // the first application runs eagerly
    tail(1);
    const int cs_timed = ctx->cs_timing;
    ctx->cs_timing = -1;
    bool fresh = true;    // the next head() follows an explicit tail (first step, or a restart)
    int replaced = 0;
    for (it = 1; it <= o->maxit; ++it) {
      if (fresh || !use_graph) {
        if (!fresh) tail(0);
        head();
        fresh = false;
      } else {
        if (!exec) {
          // one iteration as a graph: kernel nodes and the copy of ||r||^2
          HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
          capturing = true;
          tail(0);
          head();
          capturing = false;
          HIP_CHECK(hipStreamEndCapture(st, &graph));
          HIP_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        }
        HIP_CHECK(hipGraphLaunch(exec, st));
        ++replays;
        ++applies;
      }
      HIP_CHECK(hipGetLastError());
      HIP_CHECK(hipStreamSynchronize(st));
      if (it == 1 && cs_timed == 2) {
        float a = 0.f, b2 = 0.f;
        HIP_CHECK(hipEventElapsedTime(&a, ctx->ev[4], ctx->ev[5]));
        HIP_CHECK(hipEventElapsedTime(&b2, ctx->ev[6], ctx->ev[7]));
        info->coarse_solve_ms = 0.5 * ((double)a + (double)b2);
      }
      // a failed device-side wait (or any kernel error) stops the iteration
      // at once instead of iterating on invalid vectors
      if (h[5] != 0.0) break;
      rel = std::sqrt(h[2]) / bnorm;
      if (std::sqrt(h[2]) <= tol) {
        // the recurrence residual can drift from b - A x (finite precision,
        // an inexactly applied preconditioner): compute the true residual;
        // with opts->true_residual, continue from it with a fresh direction
        // while it misses the tolerance (at most twice)
        // rounding scale of that residual: (m + 1) u || |b| + |A| |x| || with m
        // the largest row length of A (componentwise bound of fl(b - A x) - (b - A x))
        launch_spmv_abs(sys, x, b, z.p, st);
        dot(z.p, z.p, n, part.p, S.p + 7, st);
        launch_spmv(sys, x, q.p, st);
        k_axpby<<<nblocks(n), 256, 0, st>>>(n, 1.0, b, -1.0, q.p, q.p);
        dot(q.p, q.p, n, part.p, S.p + 6, st);
        HIP_CHECK(hipMemcpyAsync(h + 6, S.p + 6, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        info->true_rel_residual = std::sqrt(h[6]) / bnorm;
        int32_t mrow = 0;
        for (int64_t i = 0; i < n; ++i) mrow = std::max(mrow, sys->rowptr[i + 1] - sys->rowptr[i]);
        info->residual_floor = (mrow + 1) * 0x1p-53 * std::sqrt(h[7]) / bnorm;
        conv = true;
        if (!o->true_residual || std::sqrt(h[6]) <= tol) break;
        if (replaced >= 2) {
          conv = false;
          break;
        }
        ++replaced;
        HIP_CHECK(hipMemcpyAsync(r.p, q.p, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        tail(1);
        fresh = true;
        conv = false;
      }
    }
    info->residual_replacements = replaced;
  }
  HIP_CHECK(hipEventRecord(ctx->ev[1], st));
  info->solve_ms = elapsed(ctx, 0, 1);
  info->iterations = std::min(it, o->maxit);
  if (bnorm == 0.0) info->iterations = 0;
  info->rel_residual = bnorm == 0.0 ? 0.0 : rel;
  info->graph_replays = replays;
  // one coarse solve per deflated application plus the start x0 = Q b; two per
  // balanced application
  info->coarse_solves = !(pc && pc->n0 > 0) ? 0 : deflated ? 1 + applies : 2 * applies;
  if (use_graph) {
    HIP_CHECK(hipEventRecord(ev_out, st));
    HIP_CHECK(hipStreamWaitEvent(user, ev_out, 0));
  }
  check_device_error(ctx);
  if (!conv)
    throw Error(GENEO_ENOCONV, info->residual_replacements >= 2
                                   ? "PCG: the true residual stays above rtol after two restarts from it"
                                   : "PCG did not reach rtol in maxit iterations");
}


// ---------------------------------------------------------------- GMRES

// part[c * kDotBlocks + b] = sum over block b's rows of V[:, c] . w, c < kc
__global__ __launch_bounds__(256) void k_gemv_t_partial(int64_t n, int kc, const double* __restrict__ V, int64_t ldv,
                                                        const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double s[256];
  for (int c = 0; c < kc; ++c) {
    const double* v = V + (int64_t)c * ldv;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kDotBlocks * 256) acc += v[i] * w[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)c * kDotBlocks + blockIdx.x] = s[0];
    __syncthreads();
  }
}

// h[c] (+)= sum_b part[c * kDotBlocks + b]; one workgroup per column
__global__ __launch_bounds__(kDotBlocks) void k_gemv_t_final(const double* __restrict__ part, int accumulate,
                                                              double* __restrict__ h) {
  __shared__ double s[kDotBlocks];
  const int c = blockIdx.x;
  s[threadIdx.x] = part[(int64_t)c * kDotBlocks + threadIdx.x];
  __syncthreads();
  for (int o = kDotBlocks / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) h[c] = accumulate ? h[c] + s[0] : s[0];
}

// w = beta w - sum_{c < kc} V[:, c] y[c]   (beta = 1: orthogonalisation; beta = 0: w = -V y)
__global__ void k_gemv_n(int64_t n, int kc, const double* __restrict__ V, int64_t ldv, const double* __restrict__ y,
                         double beta, double* __restrict__ w) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int c = 0; c < kc; ++c) acc += V[(int64_t)c * ldv + i] * y[c];
  w[i] = (beta != 0.0 ? beta * w[i] : 0.0) - acc;
}

// out = a x   (a read from the device scalar *ap, inverted when inv = 1)
__global__ void k_scale_dev(int64_t n, const double* __restrict__ ap, int inv, const double* __restrict__ x,
                            double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = inv ? 1.0 / sqrt(ap[0]) : ap[0];
  out[i] = a * x[i];
}

void gmres(geneo_ctx* ctx, const geneo_system* sys, const geneo_precond* pc, const double* b, double* x,
           const geneo_solve_opts* o, geneo_solve_info* info) {
  const int64_t n = sys->n;
  hipStream_t st = ctx->stream;
  const int m = o->restart > 0 ? std::min(o->restart, o->maxit) : o->maxit;
  DevBuf<double> V, w, z, part, hv, nrm;
  V.alloc((size_t)n * (m + 1));
  w.alloc(n);
  z.alloc(n);
  part.alloc((size_t)kDotBlocks * (m + 1));
  hv.alloc(m + 2);
  nrm.alloc(2);
  std::vector<double> hh(m + 2);
  auto precond = [&](const double* in, double* out) {
    if (pc)
      apply_precond(ctx, pc, in, out);
    else
      k_copy<<<nblocks(n), 256, 0, st>>>(n, in, out);
  };
  auto host_scalar = [&](const double* dev) {
    double v = 0.0;
    HIP_CHECK(hipMemcpyAsync(&v, dev, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    return v;
  };
  HIP_CHECK(hipEventRecord(ctx->ev[0], st));
  HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * n, st));
  dot(b, b, n, part.p, nrm.p, st);
  const double bnorm = std::sqrt(host_scalar(nrm.p));
  const double tol = o->rtol * bnorm;
  int it = 0;
  double res = bnorm;
  bool conv = bnorm == 0.0;
  // H column-major (m+1) x m, Givens cosines / sines, rotated right-hand side
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
  while (!conv && it < o->maxit) {
    // r = b - A x into V[:, 0] (x = 0 on the first cycle: r = b)
    double* v0 = V.p;
    if (it == 0) {
      HIP_CHECK(hipMemcpyAsync(v0, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    } else {
      launch_spmv(sys, x, w.p, st);
      k_axpby<<<nblocks(n), 256, 0, st>>>(n, 1.0, b, -1.0, w.p, v0);
    }
    dot(v0, v0, n, part.p, nrm.p, st);
    // a cycle starts from the true residual; only an exact solution ends it here
    const double beta = std::sqrt(host_scalar(nrm.p));
    res = beta;
    if (beta == 0.0) {
      conv = true;
      break;
    }
    k_scale_dev<<<nblocks(n), 256, 0, st>>>(n, nrm.p, 1, v0, v0);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int kd = 0;
    for (int k = 0; k < m && it < o->maxit; ++k) {
      ++it;
      const double* vk = V.p + (int64_t)k * n;
      precond(vk, z.p);
      launch_spmv(sys, z.p, w.p, st);
      // classical Gram-Schmidt against V[:, 0..k], twice
      for (int pass = 0; pass < 2; ++pass) {
        k_gemv_t_partial<<<kDotBlocks, 256, 0, st>>>(n, k + 1, V.p, n, w.p, part.p);
        k_gemv_t_final<<<k + 1, kDotBlocks, 0, st>>>(part.p, pass, hv.p);
        // w -= V h (the second pass subtracts the correction only: h2 = h_total - h1)
        if (pass == 0) {
          k_gemv_n<<<nblocks(n), 256, 0, st>>>(n, k + 1, V.p, n, hv.p, 1.0, w.p);
          HIP_CHECK(hipMemcpyAsync(hh.data(), hv.p, sizeof(double) * (k + 1), hipMemcpyDeviceToHost, st));
          HIP_CHECK(hipStreamSynchronize(st));
          HIP_CHECK(hipMemsetAsync(hv.p, 0, sizeof(double) * (k + 1), st));
        }
      }
      {
        std::vector<double> h2(k + 1);
        HIP_CHECK(hipMemcpyAsync(h2.data(), hv.p, sizeof(double) * (k + 1), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        k_gemv_n<<<nblocks(n), 256, 0, st>>>(n, k + 1, V.p, n, hv.p, 1.0, w.p);
        for (int j = 0; j <= k; ++j) hh[j] += h2[j];
      }
      dot(w.p, w.p, n, part.p, nrm.p, st);
      const double hn = std::sqrt(host_scalar(nrm.p));
      double* Hk = H.data() + (size_t)k * (m + 1);
      for (int j = 0; j <= k; ++j) Hk[j] = hh[j];
      Hk[k + 1] = hn;
      if (hn > 0.0) k_scale_dev<<<nblocks(n), 256, 0, st>>>(n, nrm.p, 1, w.p, V.p + (int64_t)(k + 1) * n);
      // previous rotations, then a new one that zeroes H[k+1, k]
      for (int j = 0; j < k; ++j) {
        const double t = cs[j] * Hk[j] + sn[j] * Hk[j + 1];
        Hk[j + 1] = -sn[j] * Hk[j] + cs[j] * Hk[j + 1];
        Hk[j] = t;
      }
      const double den = std::hypot(Hk[k], Hk[k + 1]);
      cs[k] = den > 0.0 ? Hk[k] / den : 1.0;
      sn[k] = den > 0.0 ? Hk[k + 1] / den : 0.0;
      Hk[k] = den;
      Hk[k + 1] = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      kd = k + 1;
      res = std::fabs(g[k + 1]);
      HIP_CHECK(hipGetLastError());
      if (res <= tol || hn == 0.0) {
        conv = res <= tol;
        break;
      }
    }
    // y = H[:kd, :kd]^-1 g[:kd] (upper triangular), x += M^-1 V y
    std::vector<double> y(kd);
    for (int i = kd - 1; i >= 0; --i) {
      double s = g[i];
      for (int j = i + 1; j < kd; ++j) s -= H[(size_t)j * (m + 1) + i] * y[j];
      y[i] = s / H[(size_t)i * (m + 1) + i];
    }
    if (kd > 0) {
      HIP_CHECK(hipMemcpyAsync(hv.p, y.data(), sizeof(double) * kd, hipMemcpyHostToDevice, st));
      k_gemv_n<<<nblocks(n), 256, 0, st>>>(n, kd, V.p, n, hv.p, 0.0, w.p);      // w = -V y
      precond(w.p, z.p);
      k_axpby<<<nblocks(n), 256, 0, st>>>(n, 1.0, x, -1.0, z.p, x);              // x += M^-1 V y
      HIP_CHECK(hipStreamSynchronize(st));
    }
    check_device_error(ctx);
  }
  HIP_CHECK(hipEventRecord(ctx->ev[1], st));
  info->solve_ms = elapsed(ctx, 0, 1);
  info->iterations = it;
  info->rel_residual = bnorm == 0.0 ? 0.0 : res / bnorm;
  info->graph_replays = 0;
  check_device_error(ctx);
  if (!conv) throw Error(GENEO_ENOCONV, "GMRES did not reach rtol in maxit iterations");
}

}  // namespace geneo
