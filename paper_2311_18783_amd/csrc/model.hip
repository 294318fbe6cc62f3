// Learned warm start of the GenEO eigensolver: a three-layer perceptron on
// a canvas description of the subdomain predicts start vectors over the
// canvas edges.  BF16 weights and activations, FP32 accumulation on MFMA
// (v_mfma_f32_16x16x16_bf16), Adam on FP32 master weights.
//
// Canvas: C^3 hexahedral cells, (C+1)^3 nodes; an edge of the six-tetrahedron
// split of a cell runs from a node p to p + d with d one of the seven
// non-zero 0/1 vectors (three axes, three face diagonals, the main
// diagonal).  Edges are oriented from the lower to the higher node, as in
// the mesh (node ids grow with the coordinates), so model rows map onto
// subdomain dofs without sign changes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <fstream>
#include <numeric>
#include <random>

#include "model.h"

namespace geneo {

// ------------------------------------------------------------- BF16
__host__ __device__ inline uint16_t f2bf(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);   // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

static inline unsigned nb(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------------- GEMM
// C[m][n] (+)= sum_k A(m,k) B(k,n),  A(m,k) = A[m sam + k sak],
// B(k,n) = B[k sbk + n sbn] (BF16), C row-major FP32.  64 x 64 tile per
// workgroup, four waves of 32 x 32 (2 x 2 MFMA blocks), K staged through LDS
// in steps of 32.  blockIdx.z splits K into chunks of kchunk, each writing
// its own C slice (split_stride apart) for a fixed-order reduction.
constexpr int GT = 64, GK = 32, GKP = GK + 8;
typedef short s4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const uint16_t* __restrict__ A, int64_t sam,
                                                   int64_t sak, const uint16_t* __restrict__ B, int64_t sbk,
                                                   int64_t sbn, float* __restrict__ C, int64_t ldc,
                                                   int64_t split_stride, int kchunk, int accumulate) {
  __shared__ __align__(16) uint16_t As[GT * GKP];   // [m][k]
  __shared__ __align__(16) uint16_t Bs[GT * GKP];   // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.y * GT, n0 = (int64_t)blockIdx.x * GT;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  f4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
  const bool a_kc = sak == 1, b_kc = sbk == 1;
  for (int k0 = kb; k0 < ke; k0 += GK) {
#pragma unroll
    for (int i = 0; i < GT * GK / 256; ++i) {
      const int e = tid + 256 * i;
      const int mm = a_kc ? e / GK : e % GT, kk = a_kc ? e % GK : e / GT;
      const int64_t gm = m0 + mm;
      const int gk = k0 + kk;
      As[mm * GKP + kk] = (gm < M && gk < ke) ? A[gm * sam + (int64_t)gk * sak] : (uint16_t)0;
      const int nn = b_kc ? e / GK : e % GT, kn = b_kc ? e % GK : e / GT;
      const int64_t gn = n0 + nn;
      const int gk2 = k0 + kn;
      Bs[nn * GKP + kn] = (gn < N && gk2 < ke) ? B[(int64_t)gk2 * sbk + gn * sbn] : (uint16_t)0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GK; ks += 16) {
      s4_t a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *reinterpret_cast<const s4_t*>(&As[(wm + 16 * i + (lane & 15)) * GKP + ks + 4 * (lane >> 4)]);
        b[i] = *reinterpret_cast<const s4_t*>(&Bs[(wn + 16 * i + (lane & 15)) * GKP + ks + 4 * (lane >> 4)]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  float* Cz = C + (int64_t)blockIdx.z * split_stride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm + 16 * i + 4 * (lane >> 4) + v;
        const int64_t col = n0 + wn + 16 * j + (lane & 15);
        if (row < M && col < N) {
          float* c = Cz + row * ldc + col;
          *c = accumulate ? *c + acc[i][j][v] : acc[i][j][v];
        }
      }
}

__global__ void k_reduce_splits(int64_t total, int splits, const float* __restrict__ part, float* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= total) return;
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += part[(int64_t)z * total + i];
  out[i] = s;
}

// C [M x N] row-major; K split in `splits` chunks when > 1 (part holds splits*M*N floats)
static void gemm(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk,
                 int64_t sbn, float* C, hipStream_t st, int splits = 1, float* part = nullptr) {
  if (M == 0 || N == 0) return;
  dim3 grid((unsigned)((N + GT - 1) / GT), (unsigned)((M + GT - 1) / GT), (unsigned)splits);
  if (splits <= 1) {
    k_gemm_bf16<<<grid, 256, 0, st>>>(M, N, K, A, sam, sak, B, sbk, sbn, C, N, 0, std::max(K, 1), 0);
  } else {
    const int kchunk = (int)round_up((K + splits - 1) / splits, GK);
    k_gemm_bf16<<<grid, 256, 0, st>>>(M, N, K, A, sam, sak, B, sbk, sbn, part, N, (int64_t)M * N, kchunk, 0);
    k_reduce_splits<<<nb((int64_t)M * N), 256, 0, st>>>((int64_t)M * N, splits, part, C);
  }
  HIP_CHECK(hipGetLastError());
}

// ------------------------------------------------------------- elementwise
// Z [B x F] += bias; H = BF16(relu(Z)) (or BF16(Z) when relu == 0)
__global__ void k_bias_act(int64_t total, int F, float* __restrict__ Z, const float* __restrict__ bias, int relu,
                           uint16_t* __restrict__ H) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= total) return;
  const float z = Z[i] + bias[i % F];
  Z[i] = z;
  if (H) H[i] = f2bf(relu ? fmaxf(z, 0.f) : z);
}

// dZ = dH where Z > 0 (ReLU), as FP32 and BF16
__global__ void k_relu_back(int64_t total, const float* __restrict__ dH, const float* __restrict__ Z,
                            float* __restrict__ dZ, uint16_t* __restrict__ dZb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= total) return;
  const float g = Z[i] > 0.f ? dH[i] : 0.f;
  dZ[i] = g;
  dZb[i] = f2bf(g);
}

// out[f] = sum_b X[b][f] (bias gradients, fixed order)
__global__ void k_colsum(int B, int64_t F, const float* __restrict__ X, float* __restrict__ out) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= F) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += X[(int64_t)b * F + f];
  out[f] = s;
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ x, uint16_t* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float c1, float c2, float eps,
                       uint16_t* __restrict__ pb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  if (pb) pb[i] = f2bf(pi);
}

// ------------------------------------------------------------- span loss
// Per sample s (one workgroup): G1 = Y^T Y, G2 = V^T Y over the masked rows
// (k x k each, k <= 32), and loss_s = ||G1||^2 - 2 ||G2||^2 + k.
constexpr int kLossRows = 32;
__global__ __launch_bounds__(256) void k_span_gram(int rows, int k, const float* __restrict__ Y,
                                                   const float* __restrict__ V, const uint8_t* __restrict__ mask,
                                                   float* __restrict__ G, double* __restrict__ loss) {
  __shared__ float ys[kLossRows][33], vs[kLossRows][33];
  __shared__ double red[256];
  const int s = blockIdx.x, tid = threadIdx.x;
  const int64_t R = (int64_t)rows * k;
  const float* Ys = Y + s * R;
  const float* Vs = V + s * R;
  const uint8_t* ms = mask + (int64_t)s * rows;
  constexpr int PER = (2 * 32 * 32 + 255) / 256;
  float acc[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) acc[t] = 0.f;
  for (int r0 = 0; r0 < rows; r0 += kLossRows) {
    for (int e = tid; e < kLossRows * k; e += 256) {
      const int rr = e / k, c = e % k, r = r0 + rr;
      const bool on = r < rows && ms[r];
      ys[rr][c] = on ? Ys[(int64_t)r * k + c] : 0.f;
      vs[rr][c] = on ? Vs[(int64_t)r * k + c] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + 256 * t;
      if (e < 2 * k * k) {
        const int which = e / (k * k), d = (e % (k * k)) / k, c = e % k;
        float a = 0.f;
        if (which == 0)
          for (int rr = 0; rr < kLossRows; ++rr) a += ys[rr][d] * ys[rr][c];
        else
          for (int rr = 0; rr < kLossRows; ++rr) a += vs[rr][d] * ys[rr][c];
        acc[t] += a;
      }
    }
    __syncthreads();
  }
  double part = 0.0;
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int e = tid + 256 * t;
    if (e < 2 * k * k) {
      G[(int64_t)s * 2 * k * k + e] = acc[t];
      part += (e < k * k ? 1.0 : -2.0) * (double)acc[t] * (double)acc[t];
    }
  }
  red[tid] = part;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) loss[s] = red[0] + k;
}

// dY = scale * mask * (4 Y G1 - 4 V G2), one thread per output element
__global__ void k_span_dy(int B, int rows, int k, const float* __restrict__ Y, const float* __restrict__ V,
                          const uint8_t* __restrict__ mask, const float* __restrict__ G, float scale,
                          float* __restrict__ dY, uint16_t* __restrict__ dYb) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t R = (int64_t)rows * k;
  if (t >= (int64_t)B * R) return;
  const int64_t s = t / R;
  const int64_t rc = t - s * R;
  const int64_t r = rc / k;
  const int c = (int)(rc - r * k);
  const int64_t base = s * R + r * k;
  const float* G1 = G + s * 2 * k * k;
  const float* G2 = G1 + k * k;
  float a = 0.f;
  for (int d = 0; d < k; ++d) a += Y[base + d] * G1[d * k + c] - V[base + d] * G2[d * k + c];
  const float g = mask[s * rows + r] ? 4.f * scale * a : 0.f;
  dY[t] = g;
  dYb[t] = f2bf(g);
}

// ------------------------------------------------------------- network
struct Net {
  int B = 0;
  DevBuf<uint16_t> X, H1, H2, dYb, dZ1b, dZ2b;
  DevBuf<float> Z1, Z2, Y, V, dY, dH1, dH2, dZ1, dZ2, G, part;
  DevBuf<uint8_t> mask;
  DevBuf<double> loss;
  DevBuf<float> grad[6];
  void alloc(const geneo_model* m, int b, bool train) {
    B = b;
    X.alloc((size_t)b * m->in_dim);
    Z1.alloc((size_t)b * m->hidden);
    Z2.alloc((size_t)b * m->hidden);
    H1.alloc((size_t)b * m->hidden);
    H2.alloc((size_t)b * m->hidden);
    Y.alloc((size_t)b * m->R);
    if (!train) return;
    V.alloc((size_t)b * m->R);
    mask.alloc((size_t)b * m->rows);
    dY.alloc((size_t)b * m->R);
    dYb.alloc((size_t)b * m->R);
    dH1.alloc((size_t)b * m->hidden);
    dH2.alloc((size_t)b * m->hidden);
    dZ1.alloc((size_t)b * m->hidden);
    dZ2.alloc((size_t)b * m->hidden);
    dZ1b.alloc((size_t)b * m->hidden);
    dZ2b.alloc((size_t)b * m->hidden);
    G.alloc((size_t)b * 2 * m->k * m->k);
    loss.alloc(b);
    part.alloc((size_t)kSplits * b * m->hidden);
    for (int i = 0; i < 6; ++i) grad[i].alloc(m->psize[i]);
  }
  static constexpr int kSplits = 128;
};

// Y = f(X) for the B samples in net.X
static void forward(const geneo_model* m, Net& n, hipStream_t st) {
  const int B = n.B, h = m->hidden;
  gemm(B, h, m->in_dim, n.X.p, m->in_dim, 1, m->pbf[0].p, 1, m->in_dim, n.Z1.p, st);
  k_bias_act<<<nb((int64_t)B * h), 256, 0, st>>>((int64_t)B * h, h, n.Z1.p, m->p32[1].p, 1, n.H1.p);
  gemm(B, h, h, n.H1.p, h, 1, m->pbf[2].p, 1, h, n.Z2.p, st);
  k_bias_act<<<nb((int64_t)B * h), 256, 0, st>>>((int64_t)B * h, h, n.Z2.p, m->p32[3].p, 1, n.H2.p);
  gemm(B, (int)m->R, h, n.H2.p, h, 1, m->pbf[4].p, 1, h, n.Y.p, st);
  k_bias_act<<<nb((int64_t)B * m->R), 256, 0, st>>>((int64_t)B * m->R, (int)m->R, n.Y.p, m->p32[5].p, 0, nullptr);
  HIP_CHECK(hipGetLastError());
}

// loss (mean over the batch, returned) and gradients into n.grad; n.V / n.mask hold the targets
static double backward(const geneo_model* m, Net& n, hipStream_t st) {
  const int B = n.B, h = m->hidden, k = m->k, rows = m->rows;
  const int64_t R = m->R;
  k_span_gram<<<B, 256, 0, st>>>(rows, k, n.Y.p, n.V.p, n.mask.p, n.G.p, n.loss.p);
  k_span_dy<<<nb((int64_t)B * R), 256, 0, st>>>(B, rows, k, n.Y.p, n.V.p, n.mask.p, n.G.p, 1.0f / B, n.dY.p,
                                                 n.dYb.p);
  // layer 3: db3, dW3 = dY^T H2, dH2 = dY W3
  k_colsum<<<nb(R), 256, 0, st>>>(B, R, n.dY.p, n.grad[5].p);
  gemm((int)R, h, B, n.dYb.p, 1, R, n.H2.p, h, 1, n.grad[4].p, st);
  gemm(B, h, (int)R, n.dYb.p, R, 1, m->pbf[4].p, h, 1, n.dH2.p, st, Net::kSplits, n.part.p);
  // layer 2
  k_relu_back<<<nb((int64_t)B * h), 256, 0, st>>>((int64_t)B * h, n.dH2.p, n.Z2.p, n.dZ2.p, n.dZ2b.p);
  k_colsum<<<nb(h), 256, 0, st>>>(B, h, n.dZ2.p, n.grad[3].p);
  gemm(h, h, B, n.dZ2b.p, 1, h, n.H1.p, h, 1, n.grad[2].p, st);
  gemm(B, h, h, n.dZ2b.p, h, 1, m->pbf[2].p, h, 1, n.dH1.p, st);
  // layer 1
  k_relu_back<<<nb((int64_t)B * h), 256, 0, st>>>((int64_t)B * h, n.dH1.p, n.Z1.p, n.dZ1.p, n.dZ1b.p);
  k_colsum<<<nb(h), 256, 0, st>>>(B, h, n.dZ1.p, n.grad[1].p);
  gemm(h, m->in_dim, B, n.dZ1b.p, 1, h, n.X.p, m->in_dim, 1, n.grad[0].p, st);
  HIP_CHECK(hipGetLastError());
  std::vector<double> l(B);
  HIP_CHECK(hipMemcpyAsync(l.data(), n.loss.p, sizeof(double) * B, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  double s = 0.0;
  for (double v : l) s += v;
  return s / B;
}

// ------------------------------------------------------------- set-up
static void build_edge_table(geneo_model* m) {
  const int C = m->C, P = C + 1;
  m->edge_id.assign((size_t)7 * P * P * P, -1);
  int32_t row = 0;
  for (int dir = 0; dir < 7; ++dir) {
    const int dx = (dir + 1) & 1, dy = ((dir + 1) >> 1) & 1, dz = ((dir + 1) >> 2) & 1;
    for (int z = 0; z + dz <= C; ++z)
      for (int y = 0; y + dy <= C; ++y)
        for (int x = 0; x + dx <= C; ++x) m->edge_id[(size_t)dir * P * P * P + x + P * (y + P * z)] = row++;
  }
  m->rows = row;
}

void model_init(geneo_model* m, const geneo_model_opts* o, hipStream_t st) {
  if (o->canvas < 1 || o->canvas > 64 || o->hidden < 16 || o->hidden > 4096 || o->k < 1 || o->k > 32)
    throw Error(GENEO_EINVAL, "model options out of range (canvas 1..64, hidden 16..4096, k 1..32)");
  m->C = o->canvas;
  m->hidden = o->hidden;
  m->k = o->k;
  m->seed = o->seed;
  build_edge_table(m);
  m->in_dim = 5 * m->C * m->C * m->C + 2;
  m->R = (int64_t)m->rows * m->k;
  const int64_t h = m->hidden;
  const int64_t sz[6] = {h * m->in_dim, h, h * h, h, m->R * h, m->R};
  std::mt19937_64 rng(o->seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (int i = 0; i < 6; ++i) {
    m->psize[i] = sz[i];
    std::vector<float> v((size_t)sz[i], 0.f);
    if (i % 2 == 0) {
      const int64_t fan_in = i == 0 ? m->in_dim : h;
      const double sd = (i == 4 ? 0.1 : 1.0) * std::sqrt((i == 4 ? 1.0 : 2.0) / (double)fan_in);
      for (auto& x : v) x = bf2f(f2bf((float)(sd * nd(rng))));
    }
    m->p32[i].upload(v, st);
    m->m1[i].alloc(sz[i]);
    m->m2[i].alloc(sz[i]);
    HIP_CHECK(hipMemsetAsync(m->m1[i].p, 0, sizeof(float) * sz[i], st));
    HIP_CHECK(hipMemsetAsync(m->m2[i].p, 0, sizeof(float) * sz[i], st));
    if (i % 2 == 0) {
      m->pbf[i].alloc(sz[i]);
      k_to_bf16<<<nb(sz[i]), 256, 0, st>>>(sz[i], m->p32[i].p, m->pbf[i].p);
    }
  }
  m->adam_t = 0;
  HIP_CHECK(hipStreamSynchronize(st));
}

// ------------------------------------------------------------- canvas
struct Geometry {
  bool ok = false;
  std::vector<int32_t> cell_ijk, node_ijk;   // [3 * cells], [3 * nodes]
  std::vector<float> cell_logmu, cell_logeps, cell_dir;   // per cell
};

static Geometry geometry(const geneo_system* s, hipStream_t st) {
  Geometry g;
  const int64_t T = s->n_tets, nc = s->n_cells, nn = s->n_nodes;
  if (nc <= 0 || (int64_t)s->cell_of_tet.size() != T) return g;
  double o[3] = {1e300, 1e300, 1e300};
  for (int64_t v = 0; v < nn; ++v)
    for (int a = 0; a < 3; ++a) o[a] = std::min(o[a], s->xyz[3 * v + a]);
  // cell size from the first tetrahedron's cell: the smallest non-zero axis gap
  double h = 1e300;
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q)
      for (int a = 0; a < 3; ++a) {
        const double d = std::fabs(s->xyz[3 * s->tets[p] + a] - s->xyz[3 * s->tets[q] + a]);
        if (d > 0) h = std::min(h, d);
      }
  if (!(h < 1e300)) return g;
  g.node_ijk.resize(3 * nn);
  for (int64_t v = 0; v < nn; ++v)
    for (int a = 0; a < 3; ++a) {
      const double x = (s->xyz[3 * v + a] - o[a]) / h;
      const double r = std::round(x);
      if (std::fabs(x - r) > 1e-6) return g;
      g.node_ijk[3 * v + a] = (int32_t)r;
    }
  g.cell_ijk.assign(3 * nc, INT32_MAX);
  for (int64_t t = 0; t < T; ++t) {
    const int32_t c = s->cell_of_tet[t];
    for (int p = 0; p < 4; ++p)
      for (int a = 0; a < 3; ++a) g.cell_ijk[3 * c + a] = std::min(g.cell_ijk[3 * c + a], g.node_ijk[3 * s->tets[4 * t + p] + a]);
  }
  // every node of a cell's tetrahedra lies on that cell's corners
  for (int64_t t = 0; t < T; ++t) {
    const int32_t c = s->cell_of_tet[t];
    for (int p = 0; p < 4; ++p)
      for (int a = 0; a < 3; ++a) {
        const int32_t d = g.node_ijk[3 * s->tets[4 * t + p] + a] - g.cell_ijk[3 * c + a];
        if (d < 0 || d > 1) return g;
      }
  }
  std::vector<double> mu(T), eps(T);
  HIP_CHECK(hipMemcpyAsync(mu.data(), s->d_mu.p, sizeof(double) * T, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipMemcpyAsync(eps.data(), s->d_eps.p, sizeof(double) * T, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  std::vector<double> lm(nc, 0.0), le(nc, 0.0);
  std::vector<int> cnt(nc, 0);
  std::vector<std::vector<int32_t>> cnodes(nc);
  for (int64_t t = 0; t < T; ++t) {
    const int32_t c = s->cell_of_tet[t];
    lm[c] += std::log(mu[t]);
    le[c] += std::log(eps[t]);
    cnt[c]++;
    for (int p = 0; p < 4; ++p) cnodes[c].push_back(s->tets[4 * t + p]);
  }
  g.cell_logmu.resize(nc);
  g.cell_logeps.resize(nc);
  g.cell_dir.resize(nc);
  for (int64_t c = 0; c < nc; ++c) {
    g.cell_logmu[c] = cnt[c] ? (float)(lm[c] / cnt[c]) : 0.f;
    g.cell_logeps[c] = cnt[c] ? (float)(le[c] / cnt[c]) : 0.f;
    auto& v = cnodes[c];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    int d = 0;
    for (int32_t x : v) d += s->node_to_free[x] < 0;
    g.cell_dir[c] = v.empty() ? 0.f : (float)d / (float)v.size();
  }
  g.ok = true;
  return g;
}

// Features of subdomain j [in_dim] and canvas row of each local dof [n_j];
// false if it does not fit the canvas.
static bool canvas_sample(const geneo_model* m, const geneo_system* s, const geneo_decomp* dec, const Geometry& g,
                          int j, float* feat, std::vector<int32_t>& rowmap) {
  if (!g.ok) return false;
  const int C = m->C, P = C + 1;
  int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
  for (int64_t t = dec->cells_ptr[j]; t < dec->cells_ptr[j + 1]; ++t) {
    const int32_t c = dec->cells[t];
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], g.cell_ijk[3 * c + a]);
      hi[a] = std::max(hi[a], g.cell_ijk[3 * c + a]);
    }
  }
  int off[3];
  for (int a = 0; a < 3; ++a) {
    const int e = hi[a] - lo[a] + 1;
    if (e > C || e < 1) return false;
    off[a] = (C - e) / 2 - lo[a];
  }
  const int64_t C3 = (int64_t)C * C * C;
  std::fill(feat, feat + m->in_dim, 0.f);
  for (int64_t t = dec->cells_ptr[j]; t < dec->cells_ptr[j + 1]; ++t) {
    const int32_t c = dec->cells[t];
    const int64_t q = (g.cell_ijk[3 * c] + off[0]) + C * ((g.cell_ijk[3 * c + 1] + off[1]) + (int64_t)C * (g.cell_ijk[3 * c + 2] + off[2]));
    feat[q] = g.cell_logmu[c];
    feat[C3 + q] = g.cell_logeps[c];
    feat[2 * C3 + q] = 1.f;
    feat[3 * C3 + q] = dec->part_of_cell[c] == j ? 1.f : 0.f;
    feat[4 * C3 + q] = g.cell_dir[c];
  }
  feat[5 * C3] = (float)std::log10(s->gamma);
  feat[5 * C3 + 1] = 1.f;
  const int64_t b = dec->dofs_ptr[j], e = dec->dofs_ptr[j + 1];
  rowmap.assign(e - b, -1);
  for (int64_t r = b; r < e; ++r) {
    const int32_t ed = s->free_edges[dec->dofs[r]];
    const int32_t na = s->edges[2 * (int64_t)ed], nb2 = s->edges[2 * (int64_t)ed + 1];
    int d[3], p[3];
    for (int a = 0; a < 3; ++a) {
      d[a] = g.node_ijk[3 * nb2 + a] - g.node_ijk[3 * na + a];
      p[a] = g.node_ijk[3 * na + a] + off[a];
      if (d[a] < 0 || d[a] > 1 || p[a] < 0 || p[a] + d[a] > C) return false;
    }
    const int dir = d[0] + 2 * d[1] + 4 * d[2] - 1;
    if (dir < 0) return false;
    const int32_t row = m->edge_id[(size_t)dir * P * P * P + p[0] + P * (p[1] + (int64_t)P * p[2])];
    if (row < 0) return false;
    rowmap[r - b] = row;
  }
  return true;
}

// ------------------------------------------------------------- warm start
__global__ void k_start_gather(int64_t len, int kb, int nq, int mk, int64_t R, const int32_t* __restrict__ row_sub,
                               const int64_t* __restrict__ voff, const int32_t* __restrict__ slot,
                               const int32_t* __restrict__ rowmap, const float* __restrict__ Y,
                               double* __restrict__ X) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= len) return;
  const int32_t row = rowmap[b];
  if (row < 0) return;
  const int j = row_sub[b];
  const int32_t sl = slot[j];
  if (sl < 0) return;
  const int64_t ld = voff[j + 1] - voff[j];
  const int64_t r = b - voff[j];
  for (int q = 0; q < nq; ++q) {
    double* x = X + voff[j] * kb + (int64_t)q * ld + r;
    *x = (double)Y[(int64_t)sl * R + (int64_t)row * mk + q] + 1e-4 * *x;
  }
}

int model_warm_start(geneo_ctx* ctx, const geneo_model* m, const geneo_precond* pc, int kb, int nev, double* X) {
  hipStream_t st = ctx->stream;
  const geneo_system* s = pc->sys;
  const geneo_decomp* dec = pc->dec;
  const int N = dec->N;
  const Geometry g = geometry(s, st);
  if (!g.ok) return 0;
  std::vector<float> feat;
  std::vector<int32_t> slot(N, -1), rowmap(pc->batch_len, -1), row_sub(pc->batch_len, 0);
  // canvases of all subdomains in parallel, then packed in subdomain order
  std::vector<std::vector<float>> fj(N);
  std::vector<std::vector<int32_t>> rmj(N);
  std::vector<uint8_t> okj(N, 0);
  parallel_for(N, [&](int j) {
    for (int64_t b = pc->voff[j]; b < pc->voff[j + 1]; ++b) row_sub[b] = j;
    fj[j].resize(m->in_dim);
    okj[j] = canvas_sample(m, s, dec, g, j, fj[j].data(), rmj[j]) ? 1 : 0;
  });
  int used = 0;
  for (int j = 0; j < N; ++j) {
    if (!okj[j]) continue;
    slot[j] = used++;
    feat.insert(feat.end(), fj[j].begin(), fj[j].end());
    for (size_t r = 0; r < rmj[j].size(); ++r) rowmap[pc->voff[j] + r] = rmj[j][r];
  }
  if (!used) return 0;
  Net n;
  n.alloc(m, used, false);
  std::vector<uint16_t> xb(feat.size());
  for (size_t i = 0; i < feat.size(); ++i) xb[i] = f2bf(feat[i]);
  HIP_CHECK(hipMemcpyAsync(n.X.p, xb.data(), sizeof(uint16_t) * xb.size(), hipMemcpyHostToDevice, st));
  forward(m, n, st);
  DevBuf<int32_t> d_slot, d_rowmap, d_rowsub;
  DevBuf<int64_t> d_voff;
  d_slot.upload(slot, st);
  d_rowmap.upload(rowmap, st);
  d_rowsub.upload(row_sub, st);
  d_voff.upload(pc->voff, st);
  const int nq = std::min(std::min(m->k, kb), nev);
  k_start_gather<<<nb(pc->batch_len), 256, 0, st>>>(pc->batch_len, kb, nq, m->k, m->R, d_rowsub.p, d_voff.p,
                                                    d_slot.p, d_rowmap.p, n.Y.p, X);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(st));
  return used;
}

// ------------------------------------------------------------- training data
void model_collect(geneo_ctx* ctx, geneo_model* m, const geneo_system* s, const geneo_decomp* dec,
                   const geneo_precond* pc, int holdout) {
  hipStream_t st = ctx->stream;
  if (pc->sys != s || pc->dec != dec) throw Error(GENEO_EINVAL, "preconditioner was built on another system");
  if (!pc->d_ritz.p || pc->ritz_k < 1) throw Error(GENEO_EINVAL, "setup without keep_ritz = 1");
  const Geometry g = geometry(s, st);
  if (!g.ok) throw Error(GENEO_EUNSUPPORTED, "the mesh is not a split hexahedral grid");
  const int N = dec->N, kb = pc->ritz_k;
  std::vector<double> Xh(pc->d_ritz.n);
  HIP_CHECK(hipMemcpyAsync(Xh.data(), pc->d_ritz.p, sizeof(double) * Xh.size(), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  const int kq = std::min(m->k, kb);
  std::vector<float> f(m->in_dim);
  std::vector<int32_t> rm;
  for (int j = 0; j < N; ++j) {
    if (!canvas_sample(m, s, dec, g, j, f.data(), rm)) continue;
    const int64_t nj = (int64_t)rm.size(), ld = pc->voff[j + 1] - pc->voff[j];
    // Ritz vectors, orthonormalised in the Euclidean inner product (twice Gram-Schmidt)
    std::vector<double> Q((size_t)nj * m->k, 0.0);
    int qn = 0;
    for (int q = 0; q < kq; ++q) {
      double* u = Q.data() + (size_t)qn * nj;
      const double* x = Xh.data() + pc->voff[j] * kb + (int64_t)q * ld;
      std::copy(x, x + nj, u);
      for (int pass = 0; pass < 2; ++pass)
        for (int p = 0; p < qn; ++p) {
          const double* w = Q.data() + (size_t)p * nj;
          double d = 0;
          for (int64_t r = 0; r < nj; ++r) d += w[r] * u[r];
          for (int64_t r = 0; r < nj; ++r) u[r] -= d * w[r];
        }
      double nr = 0;
      for (int64_t r = 0; r < nj; ++r) nr += u[r] * u[r];
      nr = std::sqrt(nr);
      if (!(nr > 1e-8)) {
        std::fill(u, u + nj, 0.0);
        continue;
      }
      for (int64_t r = 0; r < nj; ++r) u[r] /= nr;
      ++qn;
    }
    const size_t base_t = m->targ.size(), base_m = m->mask.size();
    m->feat.insert(m->feat.end(), f.begin(), f.end());
    m->targ.resize(base_t + m->R, 0.f);
    m->mask.resize(base_m + m->rows, 0);
    for (int64_t r = 0; r < nj; ++r) {
      m->mask[base_m + rm[r]] = 1;
      for (int q = 0; q < m->k; ++q) m->targ[base_t + (size_t)rm[r] * m->k + q] = (float)Q[(size_t)q * nj + r];
    }
    m->holdout.push_back(holdout ? 1 : 0);
  }
}

// ------------------------------------------------------------- training
struct Batcher {
  DevBuf<uint16_t> X;
  DevBuf<float> V;
  DevBuf<uint8_t> M;
};

__global__ void k_gather_samples(int B, const int32_t* __restrict__ idx, int64_t fx, const uint16_t* __restrict__ X,
                                 int64_t fv, const float* __restrict__ V, int64_t fm, const uint8_t* __restrict__ M,
                                 uint16_t* __restrict__ Xo, float* __restrict__ Vo, uint8_t* __restrict__ Mo) {
  const int b = blockIdx.y;
  const int64_t s = idx[b];
  const int64_t f = fv > fx ? (fv > fm ? fv : fm) : (fx > fm ? fx : fm);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < f; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < fv) Vo[b * fv + i] = V[s * fv + i];
    if (i < fx) Xo[b * fx + i] = X[s * fx + i];
    if (i < fm) Mo[b * fm + i] = M[s * fm + i];
  }
}

static void step_adam(geneo_model* m, Net& n, double lr, hipStream_t st) {
  m->adam_t++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)m->adam_t), c2 = 1.f - std::pow(b2, (float)m->adam_t);
  for (int i = 0; i < 6; ++i)
    k_adam<<<nb(m->psize[i]), 256, 0, st>>>(m->psize[i], m->p32[i].p, n.grad[i].p, m->m1[i].p, m->m2[i].p, (float)lr,
                                             b1, b2, c1, c2, 1e-8f, i % 2 == 0 ? m->pbf[i].p : nullptr);
  HIP_CHECK(hipGetLastError());
}

void model_train(geneo_ctx* ctx, geneo_model* m, const geneo_train_opts* o, geneo_train_info* info) {
  hipStream_t st = ctx->stream;
  if (o->epochs < 0 || o->batch < 1 || !(o->lr > 0)) throw Error(GENEO_EINVAL, "bad training options");
  const int S = (int)m->holdout.size();
  std::vector<int32_t> tr, ho;
  for (int i = 0; i < S; ++i) (m->holdout[i] ? ho : tr).push_back(i);
  *info = geneo_train_info{};
  if (tr.empty()) throw Error(GENEO_EINVAL, "no training samples collected");
  HIP_CHECK(hipEventRecord(ctx->ev[0], st));
  // the whole sample set on the device (features in BF16)
  Batcher all;
  std::vector<uint16_t> xb(m->feat.size());
  for (size_t i = 0; i < xb.size(); ++i) xb[i] = f2bf(m->feat[i]);
  all.X.upload(xb, st);
  all.V.upload(m->targ, st);
  all.M.upload(m->mask, st);
  const int B = std::min<int>(o->batch, (int)tr.size());
  Net n;
  n.alloc(m, B, true);
  DevBuf<int32_t> d_idx;
  d_idx.alloc(B);
  std::mt19937_64 rng(o->seed);
  auto run_batch = [&](const int32_t* idx, int bsz, bool update) {
    HIP_CHECK(hipMemcpyAsync(d_idx.p, idx, sizeof(int32_t) * bsz, hipMemcpyHostToDevice, st));
    n.B = bsz;
    k_gather_samples<<<dim3(1024, bsz), 256, 0, st>>>(bsz, d_idx.p, m->in_dim, all.X.p, m->R, all.V.p, m->rows,
                                                      all.M.p, n.X.p, n.V.p, n.mask.p);
    forward(m, n, st);
    const double l = backward(m, n, st);
    if (update) step_adam(m, n, o->lr, st);
    return l;
  };
  for (int ep = 0; ep < o->epochs; ++ep) {
    std::shuffle(tr.begin(), tr.end(), rng);
    double sum = 0.0;
    int cnt = 0;
    for (size_t b0 = 0; b0 + B <= tr.size(); b0 += B) {
      sum += run_batch(tr.data() + b0, B, true);
      ++cnt;
    }
    const double mean = cnt ? sum / cnt : 0.0;
    if (ep == 0) info->loss_first = mean;
    info->loss_last = mean;
  }
  if (!ho.empty()) {
    double sum = 0.0;
    int cnt = 0;
    for (size_t b0 = 0; b0 < ho.size(); b0 += B) {
      const int bsz = (int)std::min<size_t>(B, ho.size() - b0);
      sum += run_batch(ho.data() + b0, bsz, false) * bsz;
      cnt += bsz;
    }
    info->holdout_loss = sum / cnt;
  }
  HIP_CHECK(hipEventRecord(ctx->ev[1], st));
  HIP_CHECK(hipEventSynchronize(ctx->ev[1]));
  float ms = 0.f;
  HIP_CHECK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
  info->train_ms = ms;
}

// ------------------------------------------------------------- kernel-level entries
void model_predict(geneo_ctx* ctx, const geneo_model* m, int B, const float* X, float* Y) {
  hipStream_t st = ctx->stream;
  if (B < 1) throw Error(GENEO_EINVAL, "batch must be >= 1");
  Net n;
  n.alloc(m, B, false);
  std::vector<uint16_t> xb((size_t)B * m->in_dim);
  for (size_t i = 0; i < xb.size(); ++i) xb[i] = f2bf(X[i]);
  HIP_CHECK(hipMemcpyAsync(n.X.p, xb.data(), sizeof(uint16_t) * xb.size(), hipMemcpyHostToDevice, st));
  forward(m, n, st);
  HIP_CHECK(hipMemcpyAsync(Y, n.Y.p, sizeof(float) * B * m->R, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
}

double model_loss_grad(geneo_ctx* ctx, const geneo_model* m, int B, const float* X, const float* V,
                       const uint8_t* mask, float* grad) {
  hipStream_t st = ctx->stream;
  if (B < 1) throw Error(GENEO_EINVAL, "batch must be >= 1");
  Net n;
  n.alloc(m, B, true);
  std::vector<uint16_t> xb((size_t)B * m->in_dim);
  for (size_t i = 0; i < xb.size(); ++i) xb[i] = f2bf(X[i]);
  HIP_CHECK(hipMemcpyAsync(n.X.p, xb.data(), sizeof(uint16_t) * xb.size(), hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemcpyAsync(n.V.p, V, sizeof(float) * B * m->R, hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemcpyAsync(n.mask.p, mask, (size_t)B * m->rows, hipMemcpyHostToDevice, st));
  forward(m, n, st);
  const double l = backward(m, n, st);
  if (grad) {
    int64_t off = 0;
    for (int i = 0; i < 6; ++i) {
      HIP_CHECK(hipMemcpyAsync(grad + off, n.grad[i].p, sizeof(float) * m->psize[i], hipMemcpyDeviceToHost, st));
      off += m->psize[i];
    }
    HIP_CHECK(hipStreamSynchronize(st));
  }
  return l;
}

int64_t model_n_params(const geneo_model* m) {
  int64_t s = 0;
  for (int i = 0; i < 6; ++i) s += m->psize[i];
  return s;
}

// weights as their BF16 values, biases in FP32
void model_get_params(const geneo_model* m, float* out) {
  HIP_CHECK(hipDeviceSynchronize());   // pending updates on any stream
  int64_t off = 0;
  for (int i = 0; i < 6; ++i) {
    HIP_CHECK(hipMemcpy(out + off, m->p32[i].p, sizeof(float) * m->psize[i], hipMemcpyDeviceToHost));
    if (i % 2 == 0)
      for (int64_t t = 0; t < m->psize[i]; ++t) out[off + t] = bf2f(f2bf(out[off + t]));
    off += m->psize[i];
  }
}

void model_set_params(geneo_ctx* ctx, geneo_model* m, const float* in, bool round_masters) {
  hipStream_t st = ctx->stream;
  int64_t off = 0;
  for (int i = 0; i < 6; ++i) {
    std::vector<float> v(in + off, in + off + m->psize[i]);
    if (i % 2 == 0 && round_masters)
      for (auto& x : v) x = bf2f(f2bf(x));
    HIP_CHECK(hipMemcpyAsync(m->p32[i].p, v.data(), sizeof(float) * v.size(), hipMemcpyHostToDevice, st));
    HIP_CHECK(hipMemsetAsync(m->m1[i].p, 0, sizeof(float) * m->psize[i], st));
    HIP_CHECK(hipMemsetAsync(m->m2[i].p, 0, sizeof(float) * m->psize[i], st));
    if (i % 2 == 0) k_to_bf16<<<nb(m->psize[i]), 256, 0, st>>>(m->psize[i], m->p32[i].p, m->pbf[i].p);
    HIP_CHECK(hipStreamSynchronize(st));
    off += m->psize[i];
  }
  m->adam_t = 0;
}

// file: magic, version, canvas, hidden, k, then the parameters (FP32 master values)
static const char kMagic[8] = {'G', 'E', 'N', 'E', 'O', 'W', 'S', '1'};

void model_save(const geneo_model* m, const char* path) {
  std::ofstream f(path, std::ios::binary);
  if (!f) throw Error(GENEO_EINVAL, std::string("cannot write ") + path);
  f.write(kMagic, 8);
  const int32_t hdr[3] = {m->C, m->hidden, m->k};
  f.write(reinterpret_cast<const char*>(hdr), sizeof(hdr));
  f.write(reinterpret_cast<const char*>(&m->seed), sizeof(m->seed));
  HIP_CHECK(hipDeviceSynchronize());
  for (int i = 0; i < 6; ++i) {
    std::vector<float> v(m->psize[i]);
    HIP_CHECK(hipMemcpy(v.data(), m->p32[i].p, sizeof(float) * v.size(), hipMemcpyDeviceToHost));
    f.write(reinterpret_cast<const char*>(v.data()), sizeof(float) * v.size());
  }
  if (!f) throw Error(GENEO_EINVAL, std::string("write failed: ") + path);
}

void model_load(geneo_ctx* ctx, geneo_model* m, const char* path) {
  std::ifstream f(path, std::ios::binary);
  if (!f) throw Error(GENEO_EINVAL, std::string("cannot read ") + path);
  char mg[8];
  int32_t hdr[3];
  uint64_t seed = 0;
  f.read(mg, 8);
  f.read(reinterpret_cast<char*>(hdr), sizeof(hdr));
  f.read(reinterpret_cast<char*>(&seed), sizeof(seed));
  if (!f || std::memcmp(mg, kMagic, 8) != 0) throw Error(GENEO_EINVAL, std::string("not a model file: ") + path);
  geneo_model_opts o{hdr[0], hdr[1], hdr[2], seed};
  model_init(m, &o, ctx->stream);
  std::vector<float> all((size_t)model_n_params(m));
  f.read(reinterpret_cast<char*>(all.data()), sizeof(float) * all.size());
  if (!f) throw Error(GENEO_EINVAL, std::string("truncated model file: ") + path);
  model_set_params(ctx, m, all.data(), false);
}

}  // namespace geneo
