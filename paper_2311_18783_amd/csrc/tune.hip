// Autotuner of the batched dense factorisation's schedule (tile mode,
// panel group, diagonal-block kernel) and its process-wide table.
//
// The tuner factors synthetic symmetric positive definite matrices of the
// caller's sizes (diagonally dominant, generated on the device) once per
// candidate schedule, keeps the fastest (minimum over repetitions of the
// HIP-event time), and records it under the batch's key: precision,
// largest block count and batch-size class floor(log2(batch)).  Every plan
// built afterwards (setup's local, Neumann and fallback factors, the
// kernel-level entries) looks its schedule up in that table.
#include <cmath>
#include <map>
#include <mutex>
#include <sstream>
#include <tuple>

#include "precond.h"

namespace geneo {

namespace {
struct TuneKey {
  int precision, max_blk, cls;
  bool operator<(const TuneKey& o) const {
    return std::tie(precision, max_blk, cls) < std::tie(o.precision, o.max_blk, o.cls);
  }
};
struct TuneVal {
  FactorConfig cfg;
  double ms;
};
std::mutex g_tune_mutex;
std::map<TuneKey, TuneVal>& table() {
  static auto* t = new std::map<TuneKey, TuneVal>();   // lives until the process ends
  return *t;
}
int size_class(int nmat) {
  int c = 0;
  while ((2 << c) <= nmat) ++c;
  return c;
}
}  // namespace

FactorConfig tuned_factor_config(int precision, int max_blk, int nmat) {
  std::lock_guard<std::mutex> g(g_tune_mutex);
  const auto& t = table();
  const int cls = size_class(std::max(1, nmat));
  auto it = t.find({precision, max_blk, cls});
  if (it != t.end()) return it->second.cfg;
  // nearest tuned block count of the same precision and class
  const TuneVal* best = nullptr;
  int dist = 1 << 30;
  for (const auto& kv : t)
    if (kv.first.precision == precision && kv.first.cls == cls && std::abs(kv.first.max_blk - max_blk) < dist) {
      dist = std::abs(kv.first.max_blk - max_blk);
      best = &kv.second;
    }
  return best ? best->cfg : FactorConfig{};
}

void set_tuned_factor_config(int precision, int max_blk, int nmat, const FactorConfig& c, double ms) {
  std::lock_guard<std::mutex> g(g_tune_mutex);
  table()[{precision, max_blk, size_class(std::max(1, nmat))}] = TuneVal{c, ms};
}

// one line per entry: precision max_blk class mode group rec_potrf ms
std::string tune_db_text() {
  std::lock_guard<std::mutex> g(g_tune_mutex);
  std::ostringstream os;
  os << "# libgeneo factorisation schedules: precision max_blk class mode group rec_potrf ms\n";
  for (const auto& kv : table())
    os << kv.first.precision << ' ' << kv.first.max_blk << ' ' << kv.first.cls << ' ' << kv.second.cfg.mode << ' '
       << kv.second.cfg.group << ' ' << kv.second.cfg.rec_potrf << ' ' << kv.second.ms << '\n';
  return os.str();
}

void tune_db_parse(const std::string& text) {
  std::istringstream is(text);
  std::string line;
  std::map<TuneKey, TuneVal> parsed;
  int ln = 0;
  while (std::getline(is, line)) {
    ++ln;
    if (line.empty() || line[0] == '#') continue;
    std::istringstream ls(line);
    TuneKey k{};
    TuneVal v{};
    if (!(ls >> k.precision >> k.max_blk >> k.cls >> v.cfg.mode >> v.cfg.group >> v.cfg.rec_potrf >> v.ms) ||
        (k.precision != GENEO_FP64 && k.precision != GENEO_FP32_REFINE1) || k.max_blk < 1 || k.cls < 0 ||
        v.cfg.mode < 0 || v.cfg.mode > 2 || v.cfg.group < 1 || v.cfg.group > 64 || (v.cfg.rec_potrf & ~1))
      throw Error(GENEO_EINVAL, "tuning table: bad line " + std::to_string(ln));
    parsed[k] = v;
  }
  std::lock_guard<std::mutex> g(g_tune_mutex);
  for (const auto& kv : parsed) table()[kv.first] = kv.second;
}

// Diagonally dominant symmetric test matrix: a_ii = n + 1, a_ij = h(i, j) in
// [-0.5, 0.5] (a symmetric hash), identity on the pad rows and columns.
template <typename T>
__global__ void k_gen_spd(const MatDesc* __restrict__ desc, uint64_t seed, T* __restrict__ A) {
  const MatDesc d = desc[blockIdx.y];
  const int64_t len = (int64_t)d.ld * d.ld;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < len; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / d.ld, r = e % d.ld;
    double v;
    if (r >= d.n || c >= d.n) {
      v = r == c ? 1.0 : 0.0;
    } else if (r == c) {
      v = d.n + 1.0;
    } else {
      const uint64_t lo = (uint64_t)(r < c ? r : c), hi = (uint64_t)(r < c ? c : r);
      uint64_t z = seed ^ (lo * 0x9E3779B97F4A7C15ull) ^ (hi << 32);
      z ^= z >> 33;
      z *= 0xff51afd7ed558ccdull;
      z ^= z >> 33;
      z *= 0xc4ceb9fe1a85ec53ull;
      z ^= z >> 33;
      v = (double)(z >> 11) * 0x1p-53 - 0.5;
    }
    A[d.off + e] = (T)v;
  }
}

template <typename T>
static double time_schedule(geneo_ctx* ctx, FactorPlan& P, const std::vector<MatDesc>& descs,
                            const FactorConfig& cfg, T* A, T* inv, int reps) {
  hipStream_t st = ctx->stream;
  P.plan_host(descs, GENEO_FP64, &cfg);   // launches for this panel group
  P.d_syrk_prefix.upload(P.h_syrk_prefix, st);
  double best = 1e300;
  for (int r = 0; r < reps; ++r) {
    k_gen_spd<T><<<dim3(256, (unsigned)descs.size()), 256, 0, st>>>(P.d_desc.p, 2311 + r, A);
    HIP_CHECK(hipEventRecord(ctx->ev[2], st));
    factor(P, A, inv, nullptr, 0.0, nullptr, ctx->d_err, st, nullptr, false);
    HIP_CHECK(hipEventRecord(ctx->ev[3], st));
    HIP_CHECK(hipEventSynchronize(ctx->ev[3]));
    float ms = 0;
    HIP_CHECK(hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]));
    best = std::min(best, (double)ms);
  }
  check_device_error(ctx);
  return best;
}

template <typename T>
static FactorConfig tune(geneo_ctx* ctx, const std::vector<MatDesc>& descs, int64_t total, int64_t inv_total,
                         int precision, int reps, double* best_ms, int* tried) {
  DevBuf<T> A, inv;
  A.alloc(total);
  inv.alloc(inv_total);
  FactorPlan P;
  P.build(descs, ctx->stream, precision);
  std::vector<FactorConfig> cands;
  for (int mode : {0, 1, 2})
    for (int group : {4, 8, 16})
      for (int rec : {1, 0}) cands.push_back(FactorConfig{mode, group, rec});
  FactorConfig best{};
  *best_ms = 1e300;
  for (const auto& c : cands) {
    const double ms = time_schedule<T>(ctx, P, descs, c, A.p, inv.p, reps);
    if (ms < *best_ms) {
      *best_ms = ms;
      best = c;
    }
  }
  *tried = (int)cands.size();
  return best;
}

FactorConfig autotune_factor(geneo_ctx* ctx, int32_t batch, const int32_t* n_host, int precision, int reps,
                             double* best_ms, int* tried) {
  std::vector<MatDesc> descs(batch);
  int64_t off = 0, inv_off = 0;
  int32_t flag_off = 0, max_blk = 0;
  for (int32_t i = 0; i < batch; ++i) {
    if (n_host[i] < 1) throw Error(GENEO_EINVAL, "matrix sizes must be positive");
    const int64_t np = round_up(n_host[i], NB);
    descs[i] = MatDesc{off, inv_off, -1, 0, (int32_t)np, (int32_t)(np / NB), flag_off, n_host[i]};
    off += np * np;
    inv_off += 2 * np * NB;
    flag_off += (int32_t)(np / NB);
    max_blk = std::max(max_blk, (int32_t)(np / NB));
  }
  FactorConfig c;
  if (precision == GENEO_FP64)
    c = tune<double>(ctx, descs, off, inv_off, precision, reps, best_ms, tried);
  else if (precision == GENEO_FP32_REFINE1)
    c = tune<float>(ctx, descs, off, inv_off, precision, reps, best_ms, tried);
  else
    throw Error(GENEO_EINVAL, "unknown precision");
  set_tuned_factor_config(precision, max_blk, batch, c, *best_ms);
  return c;
}

}  // namespace geneo
