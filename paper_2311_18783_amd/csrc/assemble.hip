// Assembly of A = K + gamma M (lowest-order Nedelec edges) and the topology
// it needs: edge table, Dirichlet elimination, CSR structure, the
// deterministic element -> CSR-slot scatter map.
//
// Device work: one thread per tet computes its 6x6 element matrix from the
// Whitney forms (curl w_ab = 2 grad l_a x grad l_b; int l_a l_b = |T|(1+d_ab)/20)
// and one thread per CSR slot sums the element entries that land on it in a
// fixed order (no floating-point atomics, so the result is bitwise
// reproducible).
#include <algorithm>
#include <numeric>

#include "internal.h"

namespace geneo {

__constant__ int c_local_edges[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

__device__ inline void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Element matrix A_e = mu^-1 K_e + gamma eps M_e of every tet, row-major 6x6.
__global__ void k_element(int64_t T, const int32_t* __restrict__ tets, const double* __restrict__ xyz,
                          const double* __restrict__ mu, const double* __restrict__ eps, double gamma,
                          double* __restrict__ elem) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= T) return;
  int v[4];
  double P[4][3];
  for (int k = 0; k < 4; ++k) {
    v[k] = tets[4 * t + k];
    for (int d = 0; d < 3; ++d) P[k][d] = xyz[3 * (int64_t)v[k] + d];
  }
  double r[3][3];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) r[k][d] = P[k + 1][d] - P[0][d];
  // J has rows r0, r1, r2; the columns of J^-1 are (r1 x r2, r2 x r0, r0 x r1) / det
  double g[4][3];
  cross3(r[1], r[2], g[1]);
  cross3(r[2], r[0], g[2]);
  cross3(r[0], r[1], g[3]);
  double det = dot3(r[0], g[1]);
  double inv = 1.0 / det;
  for (int k = 1; k < 4; ++k)
    for (int d = 0; d < 3; ++d) g[k][d] *= inv;
  for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
  double vol = fabs(det) / 6.0;
  int ea[6], eb[6];
  double cu[6][3];
  for (int p = 0; p < 6; ++p) {
    int a = c_local_edges[p][0], b = c_local_edges[p][1];
    if (v[a] > v[b]) { int s = a; a = b; b = s; }
    ea[p] = a;
    eb[p] = b;
    cross3(g[a], g[b], cu[p]);
  }
  double kscale = 4.0 * vol / mu[t];
  double mscale = gamma * eps[t] * vol / 20.0;
  for (int p = 0; p < 6; ++p) {
    for (int q = 0; q < 6; ++q) {
      int a = ea[p], b = eb[p], c = ea[q], d = eb[q];
      double m = (1.0 + (a == c)) * dot3(g[b], g[d]) - (1.0 + (a == d)) * dot3(g[b], g[c]) -
                 (1.0 + (b == c)) * dot3(g[a], g[d]) + (1.0 + (b == d)) * dot3(g[a], g[c]);
      elem[36 * t + 6 * p + q] = kscale * dot3(cu[p], cu[q]) + mscale * m;
    }
  }
}

// val[s] = sum of the element entries mapped to slot s, in stored order.
__global__ void k_scatter(int64_t nnz, const int32_t* __restrict__ cptr, const int32_t* __restrict__ cidx,
                          const double* __restrict__ elem, double* __restrict__ val) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nnz) return;
  double acc = 0.0;
  for (int32_t k = cptr[s]; k < cptr[s + 1]; ++k) acc += elem[cidx[k]];
  val[s] = acc;
}

// y = A x (CSR, one thread per row; rows are short).
__global__ void k_spmv(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                       const double* __restrict__ v, const double* __restrict__ x, double* __restrict__ y) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) acc += v[k] * x[ci[k]];
  y[i] = acc;
}

// y = |b| + |A| |x|: the componentwise scale of the rounding error of b - A x
__global__ void k_spmv_abs(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const double* __restrict__ v, const double* __restrict__ x, const double* __restrict__ b,
                           double* __restrict__ y) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = fabs(b[i]);
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) acc += fabs(v[k] * x[ci[k]]);
  y[i] = acc;
}

void launch_spmv_abs(const geneo_system* s, const double* x, const double* b, double* y, hipStream_t st) {
  if (s->n == 0) return;
  int64_t blocks = (s->n + 255) / 256;
  k_spmv_abs<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(s->n, s->d_rowptr.p, s->d_colind.p, s->d_val.p, x, b, y);
}

void launch_spmv(const geneo_system* s, const double* x, double* y, hipStream_t st) {
  if (s->n == 0) return;
  int64_t blocks = (s->n + 255) / 256;
  k_spmv<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(s->n, s->d_rowptr.p, s->d_colind.p, s->d_val.p, x, y);
}

// ------------------------------------------------------------- host topology

static const int kLocalEdges[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

void build_topology(geneo_system* s, const geneo_mesh* m) {
  const int64_t T = m->n_tets, V = m->n_nodes;
  s->n_tets = T;
  s->n_nodes = V;
  s->xyz.assign(m->xyz, m->xyz + 3 * V);
  s->tets.assign(m->tets, m->tets + 4 * T);
  for (int64_t k = 0; k < 4 * T; ++k)
    if (s->tets[k] < 0 || s->tets[k] >= V) throw Error(GENEO_EINVAL, "tet node id out of range");
  s->cell_of_tet.resize(T);
  if (m->cell_of_tet) {
    s->cell_of_tet.assign(m->cell_of_tet, m->cell_of_tet + T);
  } else {
    std::iota(s->cell_of_tet.begin(), s->cell_of_tet.end(), 0);
  }
  int32_t maxc = -1;
  for (auto c : s->cell_of_tet) {
    if (c < 0) throw Error(GENEO_EINVAL, "negative cell id");
    maxc = std::max(maxc, c);
  }
  s->n_cells = maxc + 1;

  // edge table: unique (low, high) pairs, lexicographic
  std::vector<int64_t> keys(6 * T);
  for (int64_t t = 0; t < T; ++t)
    for (int p = 0; p < 6; ++p) {
      int64_t a = s->tets[4 * t + kLocalEdges[p][0]], b = s->tets[4 * t + kLocalEdges[p][1]];
      if (a > b) std::swap(a, b);
      keys[6 * t + p] = a * V + b;
    }
  std::vector<int64_t> uk(keys);
  std::sort(uk.begin(), uk.end());
  uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
  s->n_edges = (int64_t)uk.size();
  s->edges.resize(2 * uk.size());
  for (size_t e = 0; e < uk.size(); ++e) {
    s->edges[2 * e] = (int32_t)(uk[e] / V);
    s->edges[2 * e + 1] = (int32_t)(uk[e] % V);
  }
  s->tet_edges.resize(6 * T);
  for (int64_t k = 0; k < 6 * T; ++k)
    s->tet_edges[k] = (int32_t)(std::lower_bound(uk.begin(), uk.end(), keys[k]) - uk.begin());

  // Dirichlet nodes and edges: those of triangles flagged Dirichlet
  std::vector<char> dnode(V, 0), dedge(uk.size(), 0);
  for (int64_t f = 0; f < m->n_bfaces; ++f) {
    if (!m->bface_dirichlet || !m->bface_dirichlet[f]) continue;
    int64_t q[3] = {m->bfaces[3 * f], m->bfaces[3 * f + 1], m->bfaces[3 * f + 2]};
    for (int k = 0; k < 3; ++k) {
      if (q[k] < 0 || q[k] >= V) throw Error(GENEO_EINVAL, "boundary face node id out of range");
      dnode[q[k]] = 1;
    }
    const int pr[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (auto& pp : pr) {
      int64_t a = q[pp[0]], b = q[pp[1]];
      if (a > b) std::swap(a, b);
      auto it = std::lower_bound(uk.begin(), uk.end(), a * V + b);
      if (it == uk.end() || *it != a * V + b) throw Error(GENEO_EINVAL, "boundary face edge is not a mesh edge");
      dedge[it - uk.begin()] = 1;
    }
  }
  s->edge_to_free.assign(uk.size(), -1);
  s->free_edges.clear();
  for (size_t e = 0; e < uk.size(); ++e)
    if (!dedge[e]) {
      s->edge_to_free[e] = (int32_t)s->free_edges.size();
      s->free_edges.push_back((int32_t)e);
    }
  s->node_to_free.assign(V, -1);
  s->free_nodes.clear();
  for (int64_t v = 0; v < V; ++v)
    if (!dnode[v]) {
      s->node_to_free[v] = (int32_t)s->free_nodes.size();
      s->free_nodes.push_back((int32_t)v);
    }
  s->n = (int64_t)s->free_edges.size();
  s->n_free_nodes = (int64_t)s->free_nodes.size();
  if (s->n == 0) throw Error(GENEO_EINVAL, "no free edges");
  if (s->n >= (int64_t)1 << 31) throw Error(GENEO_EUNSUPPORTED, "more than 2^31 free edges");

  // CSR structure of A: pairs of free edges sharing a tet
  const int64_t n = s->n;
  std::vector<int64_t> pk;
  pk.reserve(36 * T);
  for (int64_t t = 0; t < T; ++t)
    for (int p = 0; p < 6; ++p) {
      int64_t fe = s->edge_to_free[s->tet_edges[6 * t + p]];
      if (fe < 0) continue;
      for (int q = 0; q < 6; ++q) {
        int64_t ff = s->edge_to_free[s->tet_edges[6 * t + q]];
        if (ff >= 0) pk.push_back(fe * n + ff);
      }
    }
  std::sort(pk.begin(), pk.end());
  pk.erase(std::unique(pk.begin(), pk.end()), pk.end());
  s->nnz = (int64_t)pk.size();
  if (s->nnz >= (int64_t)1 << 31) throw Error(GENEO_EUNSUPPORTED, "more than 2^31 nonzeros");
  s->rowptr.assign(n + 1, 0);
  s->colind.resize(pk.size());
  for (size_t k = 0; k < pk.size(); ++k) {
    s->rowptr[pk[k] / n + 1]++;
    s->colind[k] = (int32_t)(pk[k] % n);
  }
  for (int64_t i = 0; i < n; ++i) s->rowptr[i + 1] += s->rowptr[i];

  // element entry -> slot, then slot -> element entries (counting sort keeps (t,p,q) order)
  std::vector<int32_t> slot_of(36 * T, -1);
  std::vector<int32_t> cnt(s->nnz + 1, 0);
  for (int64_t t = 0; t < T; ++t)
    for (int p = 0; p < 6; ++p) {
      int32_t fe = s->edge_to_free[s->tet_edges[6 * t + p]];
      if (fe < 0) continue;
      const int32_t* b = s->colind.data() + s->rowptr[fe];
      const int32_t* e = s->colind.data() + s->rowptr[fe + 1];
      for (int q = 0; q < 6; ++q) {
        int32_t ff = s->edge_to_free[s->tet_edges[6 * t + q]];
        if (ff < 0) continue;
        int32_t sl = (int32_t)(std::lower_bound(b, e, ff) - s->colind.data());
        slot_of[36 * t + 6 * p + q] = sl;
        cnt[sl + 1]++;
      }
    }
  for (int64_t k = 0; k < s->nnz; ++k) cnt[k + 1] += cnt[k];
  s->contrib_ptr = cnt;
  s->contrib.resize(cnt[s->nnz]);
  std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t k = 0; k < 36 * T; ++k)
    if (slot_of[k] >= 0) s->contrib[fill[slot_of[k]]++] = (int32_t)k;
}

void assemble_device(geneo_ctx* ctx, geneo_system* s, const double* mu, const double* eps, double gamma) {
  hipStream_t st = ctx->stream;
  const int64_t T = s->n_tets;
  for (int64_t t = 0; t < T; ++t) {
    if (!(mu[t] > 0) || !(eps[t] > 0)) throw Error(GENEO_EINVAL, "mu and eps must be > 0");
  }
  if (!(gamma > 0)) throw Error(GENEO_EINVAL, "gamma must be > 0");
  s->gamma = gamma;
  s->d_xyz.upload(s->xyz, st);
  s->d_tets.upload(s->tets, st);
  s->d_tet_cell.upload(s->cell_of_tet, st);
  std::vector<double> hm(mu, mu + T), he(eps, eps + T);
  s->d_mu.upload(hm, st);
  s->d_eps.upload(he, st);
  s->d_rowptr.upload(s->rowptr, st);
  s->d_colind.upload(s->colind, st);
  s->d_contrib_ptr.upload(s->contrib_ptr, st);
  s->d_contrib.upload(s->contrib, st);
  s->d_elem.alloc(36 * T);
  s->d_val.alloc(s->nnz);
  HIP_CHECK(hipEventRecord(ctx->ev[0], st));
  k_element<<<dim3((unsigned)((T + 255) / 256)), dim3(256), 0, st>>>(T, s->d_tets.p, s->d_xyz.p, s->d_mu.p,
                                                                  s->d_eps.p, gamma, s->d_elem.p);
  k_scatter<<<dim3((unsigned)((s->nnz + 255) / 256)), dim3(256), 0, st>>>(s->nnz, s->d_contrib_ptr.p,
                                                                         s->d_contrib.p, s->d_elem.p, s->d_val.p);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipEventRecord(ctx->ev[1], st));
  HIP_CHECK(hipEventSynchronize(ctx->ev[1]));
  float ms = 0;
  HIP_CHECK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
  s->assemble_ms = ms;
}

}  // namespace geneo
