// common.hpp -- internal plumbing of liblcc: status/exception handling, device
// buffers, the context (scratch arena, kernel timing) and the small device
// helpers shared by the kernels.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/lcc.h"

namespace lcc {

typedef __int128 i128;
typedef unsigned __int128 u128;

// ------------------------------------------------------------------ errors

struct Error : std::runtime_error {
  lcc_status code;
  Error(lcc_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(lcc_status c, const std::string &m) { throw Error(c, m); }

inline void hip_check(hipError_t e, const char *what, const char *file, int line) {
  if (e != hipSuccess) {
    lcc_status c = (e == hipErrorOutOfMemory) ? LCC_ERR_OUT_OF_MEMORY : LCC_ERR_DEVICE;
    fail(c, std::string(what) + ": " + hipGetErrorString(e) + " at " + file + ":" + std::to_string(line));
  }
}
#define HIPCHECK(x) ::lcc::hip_check((x), #x, __FILE__, __LINE__)
#define LAUNCHCHECK() ::lcc::hip_check(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

// ----------------------------------------------------------------- buffers

// Owning device allocation (hipMalloc), movable, grows on demand.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // Ensures capacity >= b bytes (contents are not preserved on growth).
  void ensure(size_t b) {
    if (b <= bytes && p) return;
    release();
    size_t want = b < 256 ? 256 : b;
    HIPCHECK(hipMalloc(&p, want));
    bytes = want;
  }
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// A graph whose arrays the library owns (compress output, coarse levels).
struct OwnedGraph {
  int64_t n = 0, arcs = 0;
  int32_t wt_kind = LCC_WT_UNIT;
  DevBuf off, col, wt, k, s, kk;
  lcc_graph view() const {
    lcc_graph g;
    std::memset(&g, 0, sizeof(g));
    g.n = n;
    g.arcs = arcs;
    g.off = off.as<int64_t>();
    g.col = col.as<int32_t>();
    g.wt = wt_kind == LCC_WT_UNIT ? nullptr : wt.p;
    g.wt_kind = wt_kind;
    g.k = k.as<int64_t>();
    g.s = s.as<int64_t>();
    g.kk = kk.as<int64_t>();
    return g;
  }
};

// ------------------------------------------------------------------ timing

struct KernelClass {
  int64_t launches = 0;
  double ms = 0, bytes = 0, items = 0;
};

struct PendingEvent {
  std::string name;
  hipEvent_t a, b;
  double bytes, items;
};

// ------------------------------------------------------------------- context

struct Ctx {
  int device = 0;
  int num_cu = 256;
  size_t lds_per_block = 65536;
  // kernels whose dynamic-LDS limit has been raised on this device
  std::vector<const void *> lds_raised;
  // rows beyond the LDS tables go through LDS hash partitions in the current
  // Best-Moves call (else through global tables)
  bool hub_partition = false;
  bool hub_scatter = false;  // ... scattered by partition first (levels with very wide rows)
  hipStream_t stream = nullptr;
  bool timing = false;
  std::map<std::string, KernelClass> kstats;
  std::vector<PendingEvent> pending;
  std::vector<hipEvent_t> event_pool;
  // named scratch buffers, grown on demand and reused across calls
  std::map<std::string, DevBuf> scratch;
  // pinned host mailbox for small device->host reads
  void *host_mail = nullptr;
  // iterations the last small-level Best-Moves call of each phase ran: the
  // next such call queues that many before its first read-back (a timing
  // choice only; iterations past the end change nothing)
  int32_t small_iter_hint[2] = {1, 1};
  // contracted graphs of the hierarchy levels, reused across calls
  std::vector<std::unique_ptr<OwnedGraph>> level_graphs;

  OwnedGraph &level_graph(size_t l) {
    while (level_graphs.size() <= l) level_graphs.emplace_back(new OwnedGraph());
    return *level_graphs[l];
  }

  template <class T> T *buf(const std::string &name, size_t count) {
    DevBuf &b = scratch[name];
    b.ensure(count * sizeof(T));
    return b.as<T>();
  }

  hipEvent_t get_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    return e;
  }

  // Brackets launches with events when timing is on.  With `on_dispatch`
  // the scope holds exactly one kernel launch, issued through launch():
  // the events then mark that dispatch's own start and end (as a kernel
  // trace does) instead of being separate commands around it.
  struct Timer {
    Ctx *c;
    std::string name;
    double bytes, items;
    bool on_dispatch = false, used = false;
    hipEvent_t a = nullptr, b = nullptr;
    Timer(Ctx *ctx, const char *n, double by, double it, bool dispatch = false)
        : c(ctx), name(n), bytes(by), items(it), on_dispatch(dispatch) {
      if (c->timing) {
        a = c->get_event();
        b = c->get_event();
        if (on_dispatch) c->dispatch_timer = this;
        else HIPCHECK(hipEventRecord(a, c->stream));
      }
    }
    ~Timer() {
      if (!c->timing || !a) return;
      if (on_dispatch) {
        c->dispatch_timer = nullptr;
        if (!used) {  // nothing was launched: return the events
          c->event_pool.push_back(a);
          c->event_pool.push_back(b);
          return;
        }
      } else {
        (void)hipEventRecord(b, c->stream);
      }
      c->pending.push_back({name, a, b, bytes, items});
    }
  };
  Timer *dispatch_timer = nullptr;

  // Launches a kernel on the context stream; inside an on-dispatch Timer the
  // launch carries the timer's events.
  template <class F, class... Args>
  void launch(F kernel, dim3 grid, dim3 block, size_t shmem, Args... args) {
    Timer *t = dispatch_timer;
    if (t && !t->used) {
      t->used = true;
      hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)shmem, stream, t->a, t->b, 0u, args...);
    } else {
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, args...);
    }
  }

  // Resolves recorded events (the stream must have been synchronized).
  void collect_timing() {
    for (auto &p : pending) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        KernelClass &k = kstats[p.name];
        k.launches++;
        k.ms += ms;
        k.bytes += p.bytes;
        k.items += p.items;
      }
      event_pool.push_back(p.a);
      event_pool.push_back(p.b);
    }
    pending.clear();
  }

  void sync() { HIPCHECK(hipStreamSynchronize(stream)); }

  ~Ctx() {
    for (auto &p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : event_pool) (void)hipEventDestroy(e);
    if (host_mail) (void)hipHostFree(host_mail);
  }
};

// Copies `bytes` from device memory to host memory on the context stream and
// waits for it.
inline void d2h(Ctx &c, void *dst, const void *src, size_t bytes) {
  if (!bytes) return;
  HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c.stream));
  c.sync();
}
inline void h2d(Ctx &c, void *dst, const void *src, size_t bytes) {
  if (!bytes) return;
  HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c.stream));
}

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ----------------------------------------------------------- device helpers

// SplitMix64 output function (Steele, Lea, Flood 2014).
__host__ __device__ inline uint64_t mix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Per-iteration hash of the sub-round assignment.
inline uint64_t round_hash(uint64_t seed, int32_t level, int32_t phase, int32_t it) {
  uint64_t ctr = ((uint64_t)(uint32_t)level << 33) | ((uint64_t)(uint32_t)(phase & 1) << 32) |
                 (uint64_t)(uint32_t)it;
  return mix64(seed ^ mix64(ctr));
}

template <int WK> __device__ __forceinline__ int64_t load_w(const void *wt, int64_t e) {
  if constexpr (WK == LCC_WT_UNIT) return 1;
  else if constexpr (WK == LCC_WT_I16) return (int64_t)static_cast<const int16_t *>(wt)[e];
  else if constexpr (WK == LCC_WT_I32) return (int64_t)static_cast<const int32_t *>(wt)[e];
  else return static_cast<const int64_t *>(wt)[e];
}

inline int wt_bytes(int wk) {
  switch (wk) {
    case LCC_WT_I16: return 2;
    case LCC_WT_I32: return 4;
    case LCC_WT_I64: return 8;
    default: return 0;
  }
}

__device__ __forceinline__ void atomic_add_i64(int64_t *p, int64_t v) {
  atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}

}  // namespace lcc
