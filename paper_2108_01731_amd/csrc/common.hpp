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

// Owning device allocation, movable, grows on demand.  Memory comes from
// the caller's allocator when the context has one (lcc_ctx_create), else from
// hipMalloc; a buffer keeps the callbacks and the stream it was allocated on
// and returns its memory the same way.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  lcc_allocator al{};          // al.alloc == nullptr: hipMalloc / hipFree
  hipStream_t stream = nullptr;  // the stream of the call that allocated it
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), al(o.al), stream(o.stream) { o.p = nullptr; o.bytes = 0; }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; al = o.al; stream = o.stream;
      o.p = nullptr; o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      if (al.alloc) al.free(al.user, p, bytes, (void *)stream);
      else (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
  }
  // Ensures capacity >= b bytes (contents are not preserved on growth), from
  // allocator a (a.alloc == nullptr: hipMalloc) for work on stream s.  Work
  // already queued on s may still read the old block, so with the caller's
  // allocator s is drained before the block goes back (a wait on one stream,
  // where hipFree waits for the whole device).
  void ensure(size_t b, const lcc_allocator &a, hipStream_t s) {
    if (b <= bytes && p) return;
    if (p && al.alloc) HIPCHECK(hipStreamSynchronize(s));
    release();
    size_t want = b < 256 ? 256 : (b + 255) & ~(size_t)255;
    al = a;
    stream = s;
    if (al.alloc) {
      p = al.alloc(al.user, want, (void *)s);
      if (!p) fail(LCC_ERR_OUT_OF_MEMORY, "the caller's allocator returned NULL for " + std::to_string(want) + " bytes");
    } else {
      HIPCHECK(hipMalloc(&p, want));
    }
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

// One recorded kernel launch: its function, shape and argument bytes (each
// argument at its own aligned offset), enough to add it to a HIP graph.
struct LaunchRec {
  const void *func;
  dim3 grid, block;
  uint32_t shmem;
  std::vector<char> args;
  std::vector<size_t> off;
};

// Replays of recorded launch sequences as HIP graphs.  A sequence is keyed
// by its exact bytes (functions, shapes, argument values); the first time a
// sequence is seen its launches go out one by one, from its second
// occurrence on it runs as one instantiated graph (a repeated clustering
// issues the same sequences: same buffers, same arguments).
struct GraphCache {
  struct Entry {
    std::string blob;
    int seen = 0;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
  };
  std::map<uint64_t, Entry> entries;
  uint64_t clock = 0;
  static constexpr size_t MAX_ENTRIES = 512;
  ~GraphCache() {
    for (auto &kv : entries)
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  }
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
  // launches recorded for replay as a graph (see begin_record / end_record)
  bool recording = false;
  std::vector<LaunchRec> recs;
  GraphCache graphs;
  // the caller's allocator (alloc == nullptr: hipMalloc / hipFree)
  lcc_allocator alloc{};

  OwnedGraph &level_graph(size_t l) {
    while (level_graphs.size() <= l) level_graphs.emplace_back(new OwnedGraph());
    return *level_graphs[l];
  }

  template <class T> T *buf(const std::string &name, size_t count) {
    DevBuf &b = scratch[name];
    b.ensure(count * sizeof(T), alloc, stream);
    return b.as<T>();
  }
  // A library-owned array (graph arrays) from the context's allocator.
  void ensure(DevBuf &b, size_t bytes) { b.ensure(bytes, alloc, stream); }

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
  // launch carries the timer's events; while recording it is only recorded.
  template <class... KArgs, class... Args>
  void launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t shmem, Args... args) {
    static_assert(sizeof...(KArgs) == sizeof...(Args), "argument count of the kernel");
    if (recording) {
      LaunchRec r;
      r.func = reinterpret_cast<const void *>(kernel);
      r.grid = grid;
      r.block = block;
      r.shmem = (uint32_t)shmem;
      // each argument as the kernel's own parameter type
      (record_arg<typename std::decay<KArgs>::type>(r, static_cast<typename std::decay<KArgs>::type>(args)), ...);
      recs.push_back(std::move(r));
      return;
    }
    Timer *t = dispatch_timer;
    if (t && !t->used) {
      t->used = true;
      hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)shmem, stream, t->a, t->b, 0u, args...);
    } else {
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, args...);
    }
  }

  template <class T> static void record_arg(LaunchRec &r, const T &x) {
    size_t o = (r.args.size() + alignof(T) - 1) / alignof(T) * alignof(T);
    r.args.resize(o + sizeof(T));
    std::memcpy(r.args.data() + o, &x, sizeof(T));
    r.off.push_back(o);
  }

  // Starts recording the launches made through launch().
  void begin_record() {
    recs.clear();
    recording = true;
  }

  // Ends recording and runs the recorded launches on the stream: one by one
  // the first time this exact sequence is seen, as a cached graph after.
  void end_record() {
    recording = false;
    if (recs.empty()) return;
    std::string blob;
    for (const LaunchRec &r : recs) {
      blob.append(reinterpret_cast<const char *>(&r.func), sizeof(r.func));
      blob.append(reinterpret_cast<const char *>(&r.grid), sizeof(r.grid));
      blob.append(reinterpret_cast<const char *>(&r.block), sizeof(r.block));
      blob.append(reinterpret_cast<const char *>(&r.shmem), sizeof(r.shmem));
      blob.append(r.args.data(), r.args.size());
    }
    uint64_t h = 1469598103934665603ull;  // FNV-1a
    for (unsigned char ch : blob) h = (h ^ ch) * 1099511628211ull;
    GraphCache::Entry &e = graphs.entries[h];
    e.used = ++graphs.clock;
    if (e.seen && e.blob != blob) {  // a hash collision: start over
      if (e.exec) (void)hipGraphExecDestroy(e.exec);
      e = GraphCache::Entry{};
      e.used = graphs.clock;
    }
    if (!e.seen) e.blob = blob;
    e.seen++;
    if (e.seen >= 2 && !e.exec) e.exec = instantiate();
    if (e.exec) {
      HIPCHECK(hipGraphLaunch(e.exec, stream));
    } else {
      for (const LaunchRec &r : recs) {
        std::vector<void *> params(r.off.size());
        for (size_t i = 0; i < r.off.size(); i++) params[i] = const_cast<char *>(r.args.data() + r.off[i]);
        HIPCHECK(hipLaunchKernel(r.func, r.grid, r.block, params.data(), r.shmem, stream));
      }
    }
    recs.clear();
    if (graphs.entries.size() > GraphCache::MAX_ENTRIES) {  // drop the least recently used
      auto lru = graphs.entries.begin();
      for (auto it = graphs.entries.begin(); it != graphs.entries.end(); ++it)
        if (it->second.used < lru->second.used) lru = it;
      if (lru->second.exec) (void)hipGraphExecDestroy(lru->second.exec);
      graphs.entries.erase(lru);
    }
  }

  // A graph of the recorded launches as one dependency chain.
  hipGraphExec_t instantiate() {
    hipGraph_t g = nullptr;
    HIPCHECK(hipGraphCreate(&g, 0));
    hipGraphNode_t prev = nullptr;
    for (const LaunchRec &r : recs) {
      std::vector<void *> params(r.off.size());
      for (size_t i = 0; i < r.off.size(); i++) params[i] = const_cast<char *>(r.args.data() + r.off[i]);
      hipKernelNodeParams kp;
      std::memset(&kp, 0, sizeof(kp));
      kp.func = const_cast<void *>(r.func);
      kp.gridDim = r.grid;
      kp.blockDim = r.block;
      kp.sharedMemBytes = r.shmem;
      kp.kernelParams = params.data();
      hipGraphNode_t node = nullptr;
      const hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        hip_check(e, "hipGraphAddKernelNode", __FILE__, __LINE__);
      }
      prev = node;
    }
    hipGraphExec_t x = nullptr;
    const hipError_t e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHECK(e);
    return x;
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
