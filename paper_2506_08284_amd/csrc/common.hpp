// Shared host/device plumbing of the H(curl) AMG library: error type, device
// buffers on the handle's stream, CSR containers and launch helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hcurl_amg.h"

namespace hc {

struct Error {
  int code;
  std::string msg;
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error{code, msg}; }

#define HC_HIP(x)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess)                                                                           \
      ::hc::fail(e_ == hipErrorOutOfMemory ? HCURL_ENOMEM : HCURL_EHIP,                             \
                 std::string(#x) + " -> " + hipGetErrorString(e_) + " at " + __FILE__ + ":" +       \
                     std::to_string(__LINE__));                                                     \
  } while (0)

#define HC_LAUNCH_CHECK() HC_HIP(hipGetLastError())

// Device memory source of a handle: the caller's allocator, or (no
// functions) hipMallocAsync / hipFreeAsync on the buffer's stream.
struct Allocator {
  void* (*alloc)(size_t, void*, void*) = nullptr;
  void (*free)(void*, size_t, void*, void*) = nullptr;
  void* ctx = nullptr;
  const char* refuse = nullptr;  // set: every request fails with HCURL_EUNSUPPORTED
};

// The allocator of the handle the calling thread works for (null: the
// default), set for the duration of each entry point that takes a handle.
inline thread_local const Allocator* tl_allocator = nullptr;
struct AllocatorScope {
  const Allocator* prev;
  explicit AllocatorScope(const Allocator* a) : prev(tl_allocator) { tl_allocator = a; }
  ~AllocatorScope() { tl_allocator = prev; }
  AllocatorScope(const AllocatorScope&) = delete;
  AllocatorScope& operator=(const AllocatorScope&) = delete;
};

// Device buffer allocated in stream order on the owning handle's stream,
// from the allocator current when it was allocated (kept for its release).
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;
  const Allocator* a = nullptr;
  DBuf() = default;
  DBuf(size_t count, hipStream_t st) { alloc(count, st); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), s(o.s), a(o.a) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; n = o.n; s = o.s; a = o.a;
      o.p = nullptr; o.n = 0;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(size_t count, hipStream_t st) {
    release();
    s = st;
    n = count;
    a = tl_allocator;
    if (!count) return;
    if (a && a->refuse) {
      const std::string why = a->refuse;
      a = nullptr;
      n = 0;
      fail(HCURL_EUNSUPPORTED, why + " (a request for " + std::to_string(count * sizeof(T)) + " bytes)");
    }
    if (a) {
      p = (T*)a->alloc(count * sizeof(T), (void*)st, a->ctx);
      if (!p) {
        n = 0;
        fail(HCURL_ENOMEM, "the caller's allocator returned NULL for " + std::to_string(count * sizeof(T)) + " bytes");
      }
    } else {
      HC_HIP(hipMallocAsync((void**)&p, count * sizeof(T), st));
    }
  }
  void release() noexcept {
    if (p) {
      if (a) a->free((void*)p, n * sizeof(T), (void*)s, a->ctx);
      else (void)hipFreeAsync(p, s);
    }
    p = nullptr;
    n = 0;
  }
  T* get() const { return p; }
  size_t bytes() const { return n * sizeof(T); }
};

// CSR matrix on the device, int32 indices (nnz < 2^31 checked at creation).
struct Csr {
  int nrows = 0, ncols = 0;
  int64_t nnz = 0;
  DBuf<int> rowptr;
  DBuf<int> col;
  DBuf<double> val;   // may be empty for pattern-only matrices
  DBuf<float> val32;  // FP32 copy for the single-precision V-cycle
};

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// XCD-aware block index: consecutive logical blocks land on the same XCD so
// that neighbouring row ranges share that XCD's L2.  The hardware dispatches
// workgroup b to XCD b % 8.
__device__ __forceinline__ int xcd_block(int nblocks) {
  const int b = blockIdx.x;
  const int per = nblocks / 8;
  const int xcd = b % 8;
  const int idx = b / 8;
  if (b >= per * 8) return b;  // tail blocks keep their index
  return xcd * per + idx;
}

}  // namespace hc

namespace hc {

// Per-handle execution context: the stream, a small scratch area for
// reductions and scalars, and optional kernel timing with HIP events.
struct KernelStat {
  std::string name;
  int64_t launches = 0;
  double ms = 0.0;
  double bytes = 0.0;
};

struct Ctx {
  hipStream_t s = nullptr;
  bool profile = false;
  DBuf<double> red;      // reduction partials (kRedBlocks doubles per slot)
  DBuf<double> scal;     // device scalars
  DBuf<long long> iscal; // device integer scalars / flags
  std::vector<KernelStat> stats;
  struct Pending { int idx; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;

  static constexpr int kRedBlocks = 1024;
  static constexpr int kRedSlots = 8;
  static constexpr int kScalars = 64;

  void init(hipStream_t st, bool prof) {
    s = st;
    profile = prof;
    red.alloc((size_t)kRedBlocks * kRedSlots, s);
    scal.alloc(kScalars, s);
    iscal.alloc(kScalars, s);
    HC_HIP(hipMemsetAsync(scal.p, 0, sizeof(double) * kScalars, s));
    HC_HIP(hipMemsetAsync(iscal.p, 0, sizeof(long long) * kScalars, s));
  }
  hipEvent_t ev() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    HC_HIP(hipEventCreate(&e));
    return e;
  }
  int stat_index(const char* name) {
    for (size_t i = 0; i < stats.size(); ++i)
      if (stats[i].name == name) return (int)i;
    stats.push_back(KernelStat{name});
    return (int)stats.size() - 1;
  }
  // Runs `launch` (which enqueues one kernel on s); with profiling on, brackets
  // it by events and books `bytes` algorithmic bytes under `name`.
  template <class F>
  void run(const char* name, double bytes, F&& launch) {
    if (!profile) { launch(); HC_LAUNCH_CHECK(); return; }
    int idx = stat_index(name);
    hipEvent_t a = ev(), b = ev();
    HC_HIP(hipEventRecord(a, s));
    launch();
    HC_LAUNCH_CHECK();
    HC_HIP(hipEventRecord(b, s));
    stats[idx].launches += 1;
    stats[idx].bytes += bytes;
    pending.push_back({idx, a, b});
    if (pending.size() > 4096) drain();
  }
  void drain() {
    if (pending.empty()) return;
    HC_HIP(hipStreamSynchronize(s));
    for (auto& p : pending) {
      float ms = 0.f;
      HC_HIP(hipEventElapsedTime(&ms, p.a, p.b));
      stats[p.idx].ms += ms;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  void sync() { HC_HIP(hipStreamSynchronize(s)); }
  ~Ctx() {
    for (auto& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

template <class T>
inline void d2h(T* dst, const T* src, size_t n, Ctx& c) {
  if (!n) return;
  HC_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, c.s));
  HC_HIP(hipStreamSynchronize(c.s));
}
template <class T>
inline void h2d(T* dst, const T* src, size_t n, Ctx& c) {
  if (!n) return;
  HC_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, c.s));
  HC_HIP(hipStreamSynchronize(c.s));
}
template <class T>
inline void d2d(T* dst, const T* src, size_t n, Ctx& c) {
  if (!n) return;
  HC_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToDevice, c.s));
}

}  // namespace hc
