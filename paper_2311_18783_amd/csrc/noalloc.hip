// Batched dense Cholesky for callers that cannot allocate device memory
// (code under stream capture, serving loops, harnesses that forbid
// hipMalloc): the factorisation plan and the diagonal-block inverses live in
// one file-scope device array instead of buffers allocated per call.
//
// The array is resolved to a device address once per device, by
// geneo_create with that device current; host code passes that address to
// the kernels and never the array's name (which on the host is only a
// stand-in for the symbol).  Every call on a device shares its array, so
// calls that overlap on one device race; each call rewrites every part it
// reads (plan arrays uploaded, every diagonal-block inverse written by the
// factorisation before use), so nothing has to start at zero.
#include <mutex>

#include "dense.h"

namespace geneo {

// 64 MiB per device, held until the process ends.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[kMaxDevices] = {};

// Called by geneo_create with `device` current: resolve this device's copy of
// the scratch array (once per device).
void noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) throw Error(GENEO_EUNSUPPORTED, "device id beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_mutex);
  if (g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) throw Error(GENEO_EHIP, "scratch array has no device address");
  g_scratch_ptr[device] = ptr;
}

static void* scratch_of(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mutex);
  void* p = (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
  if (!p) throw Error(GENEO_EHIP, "scratch array not resolved on this device");
  return p;
}

// Scratch layout of a call: the diagonal-block inverses (2 n_pad x 128
// elements of the factor's type per matrix) from offset 0, then the plan
// arrays, each at a multiple of 256 bytes.
void potrf_noalloc(geneo_ctx* ctx, int32_t batch, const int32_t* n_host, const int64_t* off_host, void* A,
                   int32_t precision, double* elapsed_ms) {
  if (precision != GENEO_FP64 && precision != GENEO_FP32_REFINE1) throw Error(GENEO_EINVAL, "unknown precision");
  const size_t elem = precision == GENEO_FP64 ? sizeof(double) : sizeof(float);
  std::vector<MatDesc> descs(batch);
  int64_t inv_off = 0;
  int32_t flag_off = 0;
  for (int32_t i = 0; i < batch; ++i) {
    if (n_host[i] < 1 || off_host[i] < 0 || off_host[i] % 32) throw Error(GENEO_EINVAL, "bad matrix size/offset");
    const int64_t np = round_up(n_host[i], NB);
    descs[i] = MatDesc{off_host[i], inv_off, -1, 0, (int32_t)np, (int32_t)(np / NB), flag_off, n_host[i]};
    inv_off += 2 * np * NB;
    flag_off += (int32_t)(np / NB);
  }
  const size_t inv_bytes = (size_t)round_up((int64_t)(inv_off * elem), 256);
  if (inv_bytes > kNoAllocScratchBytes)
    throw Error(GENEO_EINVAL, "batch too large for the allocation-free factorisation: needs " +
                                  std::to_string(inv_bytes) + " bytes of diagonal-block inverses, scratch holds " +
                                  std::to_string(kNoAllocScratchBytes));
  char* base = static_cast<char*>(scratch_of(ctx->device));
  FactorPlan P;
  // plan arrays after the inverses; build_in throws GENEO_EINVAL when they do not fit
  P.build_in(descs, base + inv_bytes, kNoAllocScratchBytes - inv_bytes, ctx->stream, precision);
  HIP_CHECK(hipEventRecord(ctx->ev[0], ctx->stream));
  if (precision == GENEO_FP64)
    factor(P, static_cast<double*>(A), reinterpret_cast<double*>(base), nullptr, 0.0, nullptr, ctx->d_err,
           ctx->stream, nullptr, false);
  else
    factor(P, static_cast<float*>(A), reinterpret_cast<float*>(base), nullptr, 0.0, nullptr, ctx->d_err,
           ctx->stream, nullptr, false);
  HIP_CHECK(hipEventRecord(ctx->ev[1], ctx->stream));
  HIP_CHECK(hipEventSynchronize(ctx->ev[1]));
  float ms = 0;
  HIP_CHECK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
  if (elapsed_ms) *elapsed_ms = ms;
}

}  // namespace geneo
