// Internal declarations shared by the libgeneo translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/geneo.h"

namespace geneo {

// Panel / tile width of the dense factorisations and triangular solves.
constexpr int NB = 128;

// Host loop f(i), i in [0, n), on up to 16 threads (indices handed out
// dynamically); f may only write data owned by its index and must not throw.
template <class F>
void parallel_for(int n, F&& f) {
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int nt = std::max(1, std::min({n, 16, hw}));
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next{0};
  auto worker = [&] {
    for (int i; (i = next.fetch_add(1)) < n;) f(i);
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(worker);
  worker();
  for (auto& t : th) t.join();
}

// std::vector storage whose elements are not value-initialised (a sized
// construction or resize leaves them indeterminate): for large host arrays
// that a parallel pass fills right after, without a serial zero-fill first
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U>&) {}
  template <class U, class... Args>
  void construct(U* p, Args&&... args) {
    if constexpr (sizeof...(Args) == 0)
      ::new ((void*)p) U;
    else
      ::new ((void*)p) U(std::forward<Args>(args)...);
  }
};
template <class T>
using HostVec = std::vector<T, NoInitAlloc<T>>;

// Host wall clock between marks, printed to stderr with GENEO_VERBOSE set
struct HostClock {
  const char* tag = "setup";
  bool on = std::getenv("GENEO_VERBOSE") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void mark(const char* what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[%s] %-28s %8.2f ms\n", tag, what,
                 std::chrono::duration<double, std::milli>(now - t).count());
    t = now;
  }
};

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIP_CHECK(x)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      throw ::geneo::Error(GENEO_EHIP, std::string(#x " failed: ") + hipGetErrorString(e_)); \
  } while (0)

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Large device blocks (64 MiB and up: dense local, Neumann and coarse
// matrices, the eigensolver's block vectors, coarse temporaries) are kept
// after release and handed to a later allocation on the same device that
// fits (the smallest cached block of 1x to 2x the request), so repeated
// setups do not map and unmap them again.  Release synchronises the device
// first, as hipFree would have done: work queued on any stream before the
// release has finished before the block is handed out again.  When
// hipMalloc fails the cached blocks are freed and the call is retried.
constexpr size_t kPoolMinBytes = size_t(64) << 20;

struct BlockPool {
  struct Block {
    int dev;
    size_t bytes;
    void* p;
  };
  std::mutex m;
  std::vector<Block> free_blocks;
  static BlockPool& get() {
    static BlockPool* pool = new BlockPool;   // lives until the process ends
    return *pool;
  }
  // a cached block for `bytes` on the current device, or nullptr
  void* take(size_t bytes, size_t* got) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> g(m);
    int best = -1;
    for (int i = 0; i < (int)free_blocks.size(); ++i) {
      const Block& b = free_blocks[i];
      if (b.dev == dev && b.bytes >= bytes && b.bytes <= 2 * bytes &&
          (best < 0 || b.bytes < free_blocks[best].bytes))
        best = i;
    }
    if (best < 0) return nullptr;
    void* p = free_blocks[best].p;
    *got = free_blocks[best].bytes;
    free_blocks.erase(free_blocks.begin() + best);
    return p;
  }
  void give(void* p, size_t bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
      (void)hipFree(p);
      return;
    }
    std::lock_guard<std::mutex> g(m);
    free_blocks.push_back({dev, bytes, p});
  }
  // free every cached block of the current device (before retrying a failed hipMalloc)
  void trim() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> g(m);
    for (auto it = free_blocks.begin(); it != free_blocks.end();) {
      if (it->dev == dev) {
        (void)hipFree(it->p);
        it = free_blocks.erase(it);
      } else {
        ++it;
      }
    }
  }
};

// Device buffer owned by a handle.
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  size_t cap = 0;   // bytes of the underlying block
  bool owned = true;  // false: a view of memory owned elsewhere (never freed here)
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  // exchange buffers (pointer, count and block size together: a pooled
  // block may be larger than its request)
  void swap(DevBuf& o) {
    std::swap(p, o.p);
    std::swap(n, o.n);
    std::swap(cap, o.cap);
    std::swap(owned, o.owned);
  }
  // view of `count` elements at `q` (memory owned by the caller)
  void view(T* q, size_t count) {
    release();
    p = q;
    n = count;
    cap = count * sizeof(T);
    owned = false;
  }
  void release() {
    if (p && !owned) {
      p = nullptr;
      n = 0;
      cap = 0;
      owned = true;
      return;
    }
    if (p) {
      if (cap >= kPoolMinBytes)
        BlockPool::get().give(p, cap);
      else
        (void)hipFree(p);
    }
    p = nullptr;
    n = 0;
    cap = 0;
  }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    const size_t bytes = count * sizeof(T);
    if (bytes >= kPoolMinBytes) {
      size_t got = 0;
      if (void* q = BlockPool::get().take(bytes, &got)) {
        p = static_cast<T*>(q);
        n = count;
        cap = got;
        return;
      }
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess && bytes >= kPoolMinBytes) {
      (void)hipGetLastError();
      BlockPool::get().trim();
      e = hipMalloc(&p, bytes);
    }
    if (e != hipSuccess) {
      p = nullptr;
      throw Error(GENEO_EOOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    n = count;
    cap = bytes;
  }
  template <class Alloc>
  void upload(const std::vector<T, Alloc>& h, hipStream_t s) {
    alloc(h.size());
    if (!h.empty()) HIP_CHECK(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
};

// Device error record written by kernels: [0] status, [1] matrix, [2] index.
struct DevErr {
  int code, mat, idx, pad;
};

}  // namespace geneo

struct geneo_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  geneo::DevErr* d_err = nullptr;     // device error record
  geneo::DevErr* h_err = nullptr;     // pinned host mirror
  unsigned* d_sync = nullptr;         // [0] ticket counter, [1] epoch (sync-free solves)
  // 0-3: phase timers; 4-7: the first two coarse solves of a PCG run
  hipEvent_t ev[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  int cs_timing = -1;   // >= 0: the next coarse solves record ev[4 + 2 cs_timing], ev[5 + 2 cs_timing]
};

struct geneo_system {
  int64_t n = 0, nnz = 0, n_edges = 0, n_nodes = 0, n_free_nodes = 0, n_tets = 0, n_cells = 0;
  double gamma = 0;
  double assemble_ms = 0;
  std::vector<double> xyz;
  std::vector<int32_t> tets, cell_of_tet;
  std::vector<int32_t> edges;          // [2*n_edges] (low, high)
  std::vector<int32_t> tet_edges;      // [6*T] global edge ids, local edge order (0,1)(0,2)(0,3)(1,2)(1,3)(2,3)
  std::vector<int32_t> edge_to_free, node_to_free, free_edges, free_nodes;
  std::vector<int32_t> rowptr, colind; // CSR structure of A over free edges
  std::vector<int32_t> contrib_ptr, contrib;  // slot -> element entries t*36+p*6+q
  // device
  geneo::DevBuf<double> d_val, d_elem, d_xyz, d_mu, d_eps;
  geneo::DevBuf<int32_t> d_rowptr, d_colind, d_contrib_ptr, d_contrib, d_tets, d_tet_cell;
};

struct geneo_decomp {
  int32_t N = 0;
  int overlap = 0;
  std::vector<int32_t> part_of_cell;
  std::vector<int64_t> dofs_ptr;       // [N+1] into dofs / pou
  std::vector<int32_t> dofs;           // concatenated sorted free-edge ids
  std::vector<double> pou;             // D_i values
  std::vector<int64_t> gn_ptr;         // [N+1] into gnodes
  std::vector<int32_t> gnodes;         // kept local free-node columns (free-node ids)
  std::vector<int32_t> n_dropped;      // floating components per subdomain
  std::vector<int64_t> p_all;          // all local free nodes (paper count) per subdomain
  std::vector<int64_t> cells_ptr;      // [N+1]
  std::vector<int32_t> cells;          // concatenated cells of Omega_i (sorted)
};
