// api.hip -- the exported C ABI of liblcc (declared in include/lcc.h):
// argument checks, the read-only device validation pass, the exact int64
// overflow bounds, and the Parallel-CC driver (paper Algorithm 1, bottom,
// with the multi-level refinement of Sec. 3.2.3).
#include <chrono>
#include <memory>

#include "ops.hpp"
#include "prims.hpp"

struct lcc_ctx {
  lcc::Ctx c;
};

struct lcc_graph_owned {
  lcc::OwnedGraph g;
};

namespace lcc {

static thread_local std::string g_last_error;

template <class F> static lcc_status guarded(F &&f) {
  try {
    f();
    g_last_error.clear();
    return LCC_OK;
  } catch (const Error &e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return LCC_ERR_OUT_OF_MEMORY;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return LCC_ERR_DEVICE;
  } catch (...) {
    g_last_error = "unknown error";
    return LCC_ERR_DEVICE;
  }
}

// ------------------------------------------------------------- host checks

// The pointer must lie in device memory of the context's device with at
// least `bytes` bytes left in its allocation.
static void check_dev(const Ctx &c, const void *p, size_t bytes, const char *what) {
  if (bytes == 0) return;
  if (!p) fail(LCC_ERR_INVALID_ARG, std::string(what) + " is NULL");
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    fail(LCC_ERR_INVALID_ARG, std::string(what) + " is not a device pointer");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    fail(LCC_ERR_INVALID_ARG, std::string(what) + " is not device memory");
  if (attr.device != c.device) fail(LCC_ERR_INVALID_ARG, std::string(what) + " lives on another device");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
    (void)hipGetLastError();
    fail(LCC_ERR_INVALID_ARG, std::string(what) + ": allocation range unknown");
  }
  const char *b = static_cast<const char *>(base);
  const char *q = static_cast<const char *>(p);
  if (q < b || (size_t)(q - b) + bytes > size)
    fail(LCC_ERR_INVALID_ARG, std::string(what) + " is smaller than the graph requires");
}

static void check_graph_args(const Ctx &c, const lcc_graph *g) {
  if (!g) fail(LCC_ERR_INVALID_ARG, "graph is NULL");
  // cluster ids, the fresh ids [n, 2n) of isolating vertices included, stay below 2^31
  if (g->n < 0 || g->n >= ((int64_t)1 << 30)) fail(LCC_ERR_INVALID_ARG, "n must be in [0, 2^30)");
  if (g->arcs < 0) fail(LCC_ERR_INVALID_ARG, "arcs must be >= 0");
  if (g->wt_kind < LCC_WT_UNIT || g->wt_kind > LCC_WT_I64) fail(LCC_ERR_INVALID_ARG, "unknown wt_kind");
  if (g->wt_kind == LCC_WT_UNIT && g->wt != nullptr) fail(LCC_ERR_INVALID_ARG, "wt must be NULL for LCC_WT_UNIT");
  if (g->wt_kind != LCC_WT_UNIT && g->wt == nullptr && g->arcs > 0)
    fail(LCC_ERR_INVALID_ARG, "wt is NULL but wt_kind is not LCC_WT_UNIT");
  if (g->n == 0 && g->arcs != 0) fail(LCC_ERR_INVALID_ARG, "an empty graph has no arcs");
  const size_t n = (size_t)g->n, m = (size_t)g->arcs;
  if (g->n > 0) check_dev(c, g->off, (n + 1) * sizeof(int64_t), "off");
  check_dev(c, g->col, m * sizeof(int32_t), "col");
  if (g->wt) check_dev(c, g->wt, m * (size_t)wt_bytes(g->wt_kind), "wt");
  check_dev(c, g->k, n * sizeof(int64_t), "k");
  if (g->s) check_dev(c, g->s, n * sizeof(int64_t), "s");
  if (g->kk) check_dev(c, g->kk, n * sizeof(int64_t), "kk");
}

static void check_lambda(lcc_lambda lam) {
  if (lam.p < 0) fail(LCC_ERR_INVALID_ARG, "lambda numerator p must be >= 0");
  if (lam.q < 1) fail(LCC_ERR_INVALID_ARG, "lambda denominator q must be >= 1");
}

static void check_params(const lcc_params *prm) {
  if (!prm) fail(LCC_ERR_INVALID_ARG, "params is NULL");
  if (prm->S < 1 || prm->S > 64) fail(LCC_ERR_INVALID_ARG, "S must be in [1, 64]");
  if (prm->num_iter < 0) fail(LCC_ERR_INVALID_ARG, "num_iter must be >= 0");
  if (prm->frontier != LCC_FRONTIER_ALL && prm->frontier != LCC_FRONTIER_NBR &&
      prm->frontier != LCC_FRONTIER_CLUSTERS)
    fail(LCC_ERR_INVALID_ARG, "unknown frontier rule");
  if (prm->allow_isolate != 0 && prm->allow_isolate != 1) fail(LCC_ERR_INVALID_ARG, "allow_isolate must be 0 or 1");
  if (prm->refine != 0 && prm->refine != 1) fail(LCC_ERR_INVALID_ARG, "refine must be 0 or 1");
  if (prm->stop_after_subrounds < 0) fail(LCC_ERR_INVALID_ARG, "stop_after_subrounds must be >= 0");
  if (prm->hub_limit < 0 || prm->hub_limit > LCC_HUB_LIMIT_MAX)
    fail(LCC_ERR_INVALID_ARG, "hub_limit must be in [0, " + std::to_string(LCC_HUB_LIMIT_MAX) + "]");
  if (prm->queue_ahead < 0) fail(LCC_ERR_INVALID_ARG, "queue_ahead must be >= 0");
  if (prm->small_level < 0 || prm->small_level > LCC_SMALL_LEVEL_MAX)
    fail(LCC_ERR_INVALID_ARG, "small_level must be in [0, " + std::to_string(LCC_SMALL_LEVEL_MAX) + "]");
  if (prm->low_merge < 0) fail(LCC_ERR_INVALID_ARG, "low_merge must be >= 0");
  if (prm->hub_row_limit < -1) fail(LCC_ERR_INVALID_ARG, "hub_row_limit must be >= -1");
  if (prm->score_pruning < -1 || prm->score_pruning > 1)
    fail(LCC_ERR_INVALID_ARG, "score_pruning must be -1, 0 or 1");
  if (prm->async_moves != 0 && prm->async_moves != 1) fail(LCC_ERR_INVALID_ARG, "async_moves must be 0 or 1");
}

// --------------------------------------------------------- device validation

__device__ __forceinline__ uint64_t wave_sat_sum(uint64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = sat_add(x, __shfl_xor(x, o, WAVE));
  return x;
}
__device__ __forceinline__ uint64_t wave_or(uint64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, WAVE);
  return x;
}
__device__ __forceinline__ uint64_t wave_max(uint64_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t y = __shfl_xor(x, o, WAVE);
    x = y > x ? y : x;
  }
  return x;
}

enum : uint64_t {
  E_OFF = 1, E_COL = 2, E_SELF = 4, E_K = 8, E_KK = 16, E_C = 32, E_ENDS = 64,
  F_UNSORTED = 128  // not an error: some row is not strictly ascending
};

constexpr int VA_NT = 256;
constexpr int VA_U = 4;  // arcs per thread and step of the arc pass

// Per-vertex checks and sums: one row of VAL_VROW values per block.
__global__ __launch_bounds__(VA_NT) void k_validate_vertices(const int64_t *__restrict__ off, int64_t n, int64_t arcs,
                                                             const int64_t *__restrict__ k,
                                                             const int64_t *__restrict__ kk,
                                                             const int64_t *__restrict__ s,
                                                             const int32_t *__restrict__ C,
                                                             uint64_t *__restrict__ part) {
  __shared__ uint64_t red[VAL_VROW][VA_NT / WAVE];
  uint64_t err = 0, ktot = 0, kks = 0, sabs = 0, neg = 0, maxdeg = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && (off[0] != 0 || off[n] != arcs)) err |= E_ENDS;
  for (int64_t v = (int64_t)blockIdx.x * VA_NT + threadIdx.x; v < n; v += (int64_t)gridDim.x * VA_NT) {
    const int64_t a = off[v], b = off[v + 1];
    if (b < a || a < 0 || b > arcs) err |= E_OFF;
    else maxdeg = (uint64_t)(b - a) > maxdeg ? (uint64_t)(b - a) : maxdeg;
    const int64_t kv = k[v];
    if (kv < 0) err |= E_K;
    else {
      ktot = sat_add(ktot, (uint64_t)kv);
      if (!kk) kks = sat_add(kks, (uint64_t)kv > 0xFFFFFFFFull ? ~0ull : (uint64_t)kv * (uint64_t)kv);
    }
    if (kk) {
      if (kk[v] < 0) err |= E_KK;
      else kks = sat_add(kks, (uint64_t)kk[v]);
    }
    if (s) {
      const int64_t sv = s[v];
      if (sv < 0) {
        neg = 1;
        sabs = sat_add(sabs, sv == INT64_MIN ? (1ull << 63) : (uint64_t)(-sv));
      } else {
        sabs = sat_add(sabs, (uint64_t)sv);
      }
    }
    if (C && (C[v] < 0 || (int64_t)C[v] >= n)) err |= E_C;
  }
  uint64_t vals[VAL_VROW] = {wave_or(err), wave_sat_sum(ktot), wave_sat_sum(kks), wave_sat_sum(sabs), wave_or(neg),
                          wave_max(maxdeg), 0, 0};
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0)
    for (int i = 0; i < VAL_VROW; i++) red[i][w] = vals[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t r[VAL_VROW] = {0};
    for (int j = 0; j < VA_NT / WAVE; j++) {
      r[0] |= red[0][j];
      r[1] = sat_add(r[1], red[1][j]);
      r[2] = sat_add(r[2], red[2][j]);
      r[3] = sat_add(r[3], red[3][j]);
      r[4] |= red[4][j];
      r[5] = red[5][j] > r[5] ? red[5][j] : r[5];
    }
    for (int i = 0; i < VAL_VROW; i++) part[(int64_t)blockIdx.x * VAL_VROW + i] = r[i];
  }
}

// Per-arc checks: column range, self-loops, ascending rows, sum |w|.  A
// block takes VA_NT consecutive vertices at a time (offsets already checked
// by the vertex pass), stages their offsets in LDS and walks their arcs
// coalesced, finding each arc's row by binary search in LDS.
template <int WK>
__global__ __launch_bounds__(VA_NT) void k_validate_arcs(const int64_t *__restrict__ off,
                                                         const int32_t *__restrict__ col, const void *__restrict__ wt,
                                                         int64_t n, int check, uint64_t *__restrict__ part) {
  __shared__ uint64_t red[3][VA_NT / WAVE];
  __shared__ int64_t so[VA_NT + 1];
  uint64_t err = 0, wabs = 0, neg = 0;
  const int lane = lane_id();
  for (int64_t vb = (int64_t)blockIdx.x * VA_NT; vb < n; vb += (int64_t)gridDim.x * VA_NT) {
    const int nv = (int)(vb + VA_NT < n ? VA_NT : n - vb);
    __syncthreads();  // so is reused
    for (int i = threadIdx.x; i <= nv; i += VA_NT) so[i] = off[vb + i];
    __syncthreads();
    const int64_t eb = so[0], ee = so[nv];
    // VA_U strided arcs per thread at a time: their loads are in flight together
    for (int64_t e0 = eb + threadIdx.x; e0 < ee; e0 += VA_U * VA_NT) {
      int32_t u[VA_U], prev[VA_U];
      int64_t w[VA_U];
#pragma unroll
      for (int j = 0; j < VA_U; j++) {
        const int64_t e = e0 + (int64_t)j * VA_NT;
        const bool in = e < ee;
        u[j] = in && check ? col[e] : 0;
        prev[j] = in && check && e > eb ? col[e - 1] : 0;
        w[j] = in ? load_w<WK>(wt, e) : 0;
      }
#pragma unroll
      for (int j = 0; j < VA_U; j++) {
        const int64_t e = e0 + (int64_t)j * VA_NT;
        if (e >= ee) break;
        if (check) {
          int lo = 0, hi = nv - 1;  // the row: last r with so[r] <= e
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (so[mid] <= e) lo = mid;
            else hi = mid - 1;
          }
          if (u[j] < 0 || (int64_t)u[j] >= n) err |= E_COL;
          if ((int64_t)u[j] == vb + lo) err |= E_SELF;
          if (e > so[lo] && u[j] <= prev[j]) err |= F_UNSORTED;
        }
        if (w[j] < 0) {
          neg = 1;
          wabs = sat_add(wabs, w[j] == INT64_MIN ? (1ull << 63) : (uint64_t)(-w[j]));
        } else {
          wabs = sat_add(wabs, (uint64_t)w[j]);
        }
      }
    }
  }
  err = wave_or(err);
  wabs = wave_sat_sum(wabs);
  neg = wave_or(neg);
  const int w = threadIdx.x / WAVE;
  if (lane == 0) {
    red[0][w] = err;
    red[1][w] = wabs;
    red[2][w] = neg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t r0 = 0, r1 = 0, r2 = 0;
    for (int j = 0; j < VA_NT / WAVE; j++) {
      r0 |= red[0][j];
      r1 = sat_add(r1, red[1][j]);
      r2 |= red[2][j];
    }
    part[(int64_t)blockIdx.x * 3 + 0] = r0;
    part[(int64_t)blockIdx.x * 3 + 1] = r1;
    part[(int64_t)blockIdx.x * 3 + 2] = r2;
  }
}

static std::string err_text(uint64_t e) {
  std::string s;
  if (e & E_ENDS) s += "off[0] must be 0 and off[n] must equal arcs; ";
  if (e & E_OFF) s += "offsets must be non-decreasing and within [0, arcs]; ";
  if (e & E_COL) s += "a column id is outside [0, n); ";
  if (e & E_SELF) s += "the adjacency holds a self-loop; ";
  if (e & E_K) s += "a vertex weight k is negative; ";
  if (e & E_KK) s += "a kk entry is negative; ";
  if (e & E_C) s += "a cluster id is outside [0, n); ";
  return s;
}

void launch_validate_vertices(hipStream_t stream, const lcc_graph &g, const int32_t *C, int64_t nb, uint64_t *part) {
  hipLaunchKernelGGL(k_validate_vertices, dim3((unsigned)nb), dim3(VA_NT), 0, stream, g.off, g.n, g.arcs, g.k, g.kk,
                     g.s, C, part);
  LAUNCHCHECK();
}

void launch_validate_arcs(hipStream_t stream, const lcc_graph &g, bool check, int64_t nb, uint64_t *part) {
  switch (g.wt_kind) {
    case LCC_WT_UNIT:
      hipLaunchKernelGGL((k_validate_arcs<LCC_WT_UNIT>), dim3((unsigned)nb), dim3(VA_NT), 0, stream, g.off, g.col,
                         g.wt, g.n, (int)check, part);
      break;
    case LCC_WT_I16:
      hipLaunchKernelGGL((k_validate_arcs<LCC_WT_I16>), dim3((unsigned)nb), dim3(VA_NT), 0, stream, g.off, g.col,
                         g.wt, g.n, (int)check, part);
      break;
    case LCC_WT_I32:
      hipLaunchKernelGGL((k_validate_arcs<LCC_WT_I32>), dim3((unsigned)nb), dim3(VA_NT), 0, stream, g.off, g.col,
                         g.wt, g.n, (int)check, part);
      break;
    default:
      hipLaunchKernelGGL((k_validate_arcs<LCC_WT_I64>), dim3((unsigned)nb), dim3(VA_NT), 0, stream, g.off, g.col,
                         g.wt, g.n, (int)check, part);
  }
  LAUNCHCHECK();
}

bool summary_from_vertex_row(const uint64_t r[VAL_VROW], GraphSummary &s) {
  s.ktot = r[1];
  s.kksum = r[2];
  s.sabs = r[3];
  s.negative = r[4] != 0;
  s.maxdeg = (int64_t)r[5];
  if (r[0]) {
    s.ok = false;
    s.why = err_text(r[0]);
  }
  return s.ok;
}

void summary_from_arc_row(const uint64_t r[VAL_AROW], bool check, GraphSummary &s) {
  s.wabs2 = r[1];
  s.negative = s.negative || r[2] != 0;
  s.sorted_rows = check && !(r[0] & F_UNSORTED);
  const uint64_t e2 = r[0] & ~(uint64_t)F_UNSORTED;
  if (e2) {
    s.ok = false;
    s.why = err_text(e2);
  }
}

int64_t validation_blocks(const Ctx &c, int64_t n) { return std::min<int64_t>(cdiv(n, VA_NT), (int64_t)c.num_cu * 8); }

GraphSummary summarize_graph(Ctx &c, const lcc_graph &g, const int32_t *C, bool check_structure) {
  GraphSummary s;
  const int64_t n = g.n;
  if (n == 0) return s;
  Ctx::Timer tm(&c, "validate", (double)n * 40.0 + (double)g.arcs * (4.0 + wt_bytes(g.wt_kind)), (double)g.arcs);
  const int64_t nb = validation_blocks(c, n);
  uint64_t *part = c.buf<uint64_t>("va.part", (size_t)(nb * VAL_VROW));
  launch_validate_vertices(c.stream, g, C, nb, part);
  std::vector<uint64_t> h((size_t)(nb * VAL_VROW));
  d2h(c, h.data(), part, h.size() * sizeof(uint64_t));
  uint64_t r[VAL_VROW] = {0};
  for (int64_t b = 0; b < nb; b++) combine_vertex_row(r, &h[(size_t)(b * VAL_VROW)]);
  // offsets or ids unusable: stop before touching arcs
  if (!summary_from_vertex_row(r, s)) return s;
  if (g.arcs > 0 && (check_structure || g.wt_kind != LCC_WT_UNIT)) {
    uint64_t *pa = c.buf<uint64_t>("va.parta", (size_t)(nb * VAL_AROW));
    launch_validate_arcs(c.stream, g, check_structure, nb, pa);
    std::vector<uint64_t> ha((size_t)(nb * VAL_AROW));
    d2h(c, ha.data(), pa, ha.size() * sizeof(uint64_t));
    uint64_t ra[VAL_AROW] = {0};
    for (int64_t b = 0; b < nb; b++) combine_arc_row(ra, &ha[(size_t)(b * VAL_AROW)]);
    summary_from_arc_row(ra, check_structure, s);
  } else {
    s.wabs2 = (uint64_t)g.arcs;  // unit weights
    s.sorted_rows = g.arcs == 0;
  }
  return s;
}

lcc_status overflow_bounds(const GraphSummary &s, int64_t p, int64_t q, std::string *why) {
  const u128 LIM = (u128)INT64_MAX;
  const u128 SAT = (u128)~0ull;
  auto bad = [&](const char *m) {
    if (why) *why = m;
    return LCC_ERR_OVERFLOW;
  };
  if ((u128)s.wabs2 == SAT || (u128)s.sabs == SAT || (u128)s.ktot == SAT || (u128)s.kksum == SAT)
    return bad("a weight sum exceeds 2^64");
  const u128 wabs = (u128)(s.wabs2 / 2) + (u128)s.sabs;
  const u128 kt = s.ktot;
  if (kt > LIM) return bad("sum of k exceeds 2^63-1");
  if (wabs > LIM) return bad("sum of |w| exceeds 2^63-1");
  if ((u128)s.kksum > LIM) return bad("sum of kk exceeds 2^63-1");
  const u128 kq = (kt * kt) / 4;
  if ((u128)q * wabs > LIM) return bad("q * sum|w| exceeds 2^63-1");
  if ((u128)p * kt > LIM) return bad("p * sum k exceeds 2^63-1");
  if ((u128)p * kq > LIM) return bad("p * (sum k)^2 / 4 exceeds 2^63-1");
  if (s.negative && (u128)q * wabs + (u128)p * kq > LIM)
    return bad("with negative weights, q * sum|w| + p * (sum k)^2 / 4 exceeds 2^63-1");
  return LCC_OK;
}

static GraphSummary checked_summary(Ctx &c, const lcc_graph &g, const int32_t *C, bool structure, int64_t p,
                                    int64_t q) {
  GraphSummary s = summarize_graph(c, g, C, structure);
  if (!s.ok) fail(LCC_ERR_INVALID_ARG, s.why);
  std::string why;
  if (overflow_bounds(s, p, q, &why) != LCC_OK) fail(LCC_ERR_OVERFLOW, why);
  return s;
}

static bool wide_weights(const GraphSummary &s) {
  const u128 wabs = (u128)(s.wabs2 / 2) + (u128)s.sabs;
  return wabs >= ((u128)1 << 31);
}

static void begin(Ctx &c, void *stream, const lcc_params *prm) {
  HIPCHECK(hipSetDevice(c.device));
  c.stream = (hipStream_t)stream;
  c.timing = prm ? prm->timing != 0 : false;
}

static void fill_objective(i128 N, int64_t q, lcc_objective_out *o) {
  o->num_hi = (int64_t)(N >> 64);
  o->num_lo = (uint64_t)N;
  o->den = q;
  o->value = (double)N / (double)q;
}

}  // namespace lcc

using namespace lcc;

extern "C" {

void lcc_params_default(lcc_params *prm) {
  if (!prm) return;
  std::memset(prm, 0, sizeof(*prm));
  prm->S = 4;
  prm->num_iter = 10;
  prm->seed = 1;
  prm->frontier = LCC_FRONTIER_NBR;
  prm->refine = 1;
  prm->allow_isolate = 1;
  prm->max_levels = 64;
  prm->stop_after_subrounds = 0;
  prm->validate = 1;
  prm->timing = 0;
}

const char *lcc_last_error(void) { return g_last_error.c_str(); }

lcc_status lcc_ctx_create(int32_t device, const lcc_allocator *alloc, lcc_ctx **out) {
  return guarded([&] {
    if (!out) fail(LCC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (alloc && (!alloc->alloc || !alloc->free)) fail(LCC_ERR_INVALID_ARG, "allocator with a NULL callback");
    int count = 0;
    HIPCHECK(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) fail(LCC_ERR_INVALID_ARG, "no such device");
    HIPCHECK(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIPCHECK(hipGetDeviceProperties(&prop, device));
    std::unique_ptr<lcc_ctx> ctx(new lcc_ctx());
    ctx->c.device = device;
    ctx->c.num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    ctx->c.lds_per_block = prop.sharedMemPerBlock > 0 ? prop.sharedMemPerBlock : 65536;
    if (alloc) ctx->c.alloc = *alloc;
    noalloc_setup(device);
    *out = ctx.release();
  });
}

lcc_status lcc_ctx_destroy(lcc_ctx *ctx) {
  return guarded([&] {
    if (!ctx) return;
    (void)hipSetDevice(ctx->c.device);
    (void)hipDeviceSynchronize();
    delete ctx;
  });
}

lcc_status lcc_best_move(lcc_ctx *ctx, const lcc_graph *g, lcc_lambda lam, const lcc_params *prm, int32_t level,
                         int32_t phase, int32_t *C_inout, lcc_bm_stats *stats, void *stream) {
  return guarded([&] {
    if (!ctx) fail(LCC_ERR_INVALID_ARG, "ctx is NULL");
    Ctx &c = ctx->c;
    check_params(prm);
    check_lambda(lam);
    if (level < 0) fail(LCC_ERR_INVALID_ARG, "level must be >= 0");
    if (phase != 0 && phase != 1) fail(LCC_ERR_INVALID_ARG, "phase must be 0 or 1");
    begin(c, stream, prm);
    check_graph_args(c, g);
    check_dev(c, C_inout, (size_t)g->n * sizeof(int32_t), "C_inout");
    GraphSummary s = checked_summary(c, *g, C_inout, prm->validate != 0, lam.p, lam.q);
    lcc_bm_stats st;
    best_moves(c, *g, lam.p, lam.q, *prm, level, phase, C_inout, BMShape{s.maxdeg, !wide_weights(s), false, false},
               st);
    c.sync();
    if (c.timing) c.collect_timing();
    if (stats) *stats = st;
  });
}

lcc_status lcc_compress(lcc_ctx *ctx, const lcc_graph *g, const int32_t *C, lcc_graph_owned **out, int32_t *map_out,
                        void *stream) {
  return guarded([&] {
    if (!ctx) fail(LCC_ERR_INVALID_ARG, "ctx is NULL");
    if (!out) fail(LCC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    Ctx &c = ctx->c;
    begin(c, stream, nullptr);
    check_graph_args(c, g);
    check_dev(c, C, (size_t)g->n * sizeof(int32_t), "C");
    check_dev(c, map_out, (size_t)g->n * sizeof(int32_t), "map_out");
    GraphSummary s = checked_summary(c, *g, C, true, 0, 1);
    std::unique_ptr<lcc_graph_owned> h(new lcc_graph_owned());
    int64_t md = 0;
    compress_graph(c, *g, C, h->g, map_out, wide_weights(s), &md);
    c.sync();
    *out = h.release();
  });
}

lcc_status lcc_graph_owned_view(const lcc_graph_owned *h, lcc_graph *view) {
  return guarded([&] {
    if (!h || !view) fail(LCC_ERR_INVALID_ARG, "NULL argument");
    *view = h->g.view();
  });
}

lcc_status lcc_graph_owned_free(lcc_ctx *ctx, lcc_graph_owned *h) {
  return guarded([&] {
    if (ctx) (void)hipSetDevice(ctx->c.device);
    delete h;
  });
}

lcc_status lcc_objective(lcc_ctx *ctx, const lcc_graph *g, lcc_lambda lam, const int32_t *C, lcc_objective_out *out,
                         void *stream) {
  return guarded([&] {
    if (!ctx) fail(LCC_ERR_INVALID_ARG, "ctx is NULL");
    if (!out) fail(LCC_ERR_INVALID_ARG, "out is NULL");
    Ctx &c = ctx->c;
    check_lambda(lam);
    begin(c, stream, nullptr);
    check_graph_args(c, g);
    check_dev(c, C, (size_t)g->n * sizeof(int32_t), "C");
    (void)checked_summary(c, *g, C, true, lam.p, lam.q);
    i128 N = objective_num(c, *g, lam.p, lam.q, C);
    c.sync();
    fill_objective(N, lam.q, out);
  });
}

lcc_status lcc_objective_noalloc(lcc_ctx *ctx, const lcc_graph *g, lcc_lambda lam, const int32_t *C,
                                 lcc_objective_out *out, void *stream) {
  return guarded([&] {
    if (!ctx) fail(LCC_ERR_INVALID_ARG, "ctx is NULL");
    if (!out) fail(LCC_ERR_INVALID_ARG, "out is NULL");
    Ctx &c = ctx->c;
    check_lambda(lam);
    begin(c, stream, nullptr);
    check_graph_args(c, g);
    if (g->n > LCC_NOALLOC_MAX_N)
      fail(LCC_ERR_INVALID_ARG, "n = " + std::to_string(g->n) + " exceeds LCC_NOALLOC_MAX_N = " +
                                    std::to_string((int64_t)LCC_NOALLOC_MAX_N));
    check_dev(c, C, (size_t)g->n * sizeof(int32_t), "C");
    i128 N = objective_num_noalloc(c, *g, lam.p, lam.q, C);
    c.sync();
    fill_objective(N, lam.q, out);
  });
}

lcc_status lcc_cluster(lcc_ctx *ctx, const lcc_graph *g, lcc_lambda lam, const lcc_params *prm, int32_t *labels_out,
                       lcc_objective_out *obj, lcc_cluster_stats *stats, void *stream) {
  return guarded([&] {
    if (!ctx) fail(LCC_ERR_INVALID_ARG, "ctx is NULL");
    Ctx &c = ctx->c;
    check_params(prm);
    check_lambda(lam);
    if (prm->max_levels < 1 || prm->max_levels > LCC_MAX_LEVELS)
      fail(LCC_ERR_INVALID_ARG, "max_levels must be in [1, 64]");
    begin(c, stream, prm);
    check_graph_args(c, g);
    check_dev(c, labels_out, (size_t)g->n * sizeof(int32_t), "labels_out");
    using clk = std::chrono::steady_clock;
    auto t0 = clk::now();
    lcc_cluster_stats cs;
    std::memset(&cs, 0, sizeof(cs));
    GraphSummary s = checked_summary(c, *g, nullptr, prm->validate != 0, lam.p, lam.q);
    const bool wide = wide_weights(s);
    // per-level arrays live in the context and are reused by later calls
    std::vector<lcc_graph> G;
    std::vector<int32_t *> Cl, maps;
    std::vector<int64_t> maxdeg, mindeg;
    G.push_back(*g);
    maxdeg.push_back(s.maxdeg);
    mindeg.push_back(0);
    int top = 0;
    double ms_bm = 0, ms_cp = 0;
    for (int l = 0;; l++) {
      const int64_t n = G[l].n;
      cs.n_level[l] = n;
      cs.arcs_level[l] = G[l].arcs;
      cs.levels = l + 1;
      Cl.push_back(c.buf<int32_t>("lv.C" + std::to_string(l), (size_t)(n > 0 ? n : 1)));
      int32_t *C = Cl.back();
      iota_i32(c, C, n);
      lcc_bm_stats st;
      auto a = clk::now();
      // compressed levels have strictly ascending rows by construction
      const bool simple = l > 0 || s.sorted_rows;
      best_moves(c, G[l], lam.p, lam.q, *prm, l, 0, C, BMShape{maxdeg[l], !wide, true, simple, mindeg[l]}, st);
      ms_bm += std::chrono::duration<double, std::milli>(clk::now() - a).count();
      cs.iters_coarsen[l] = st.iterations;
      cs.moves_total += st.moves;
      cs.arcs_scanned_total += st.arcs_scanned;
      // the recursion goes on only if the call changed the partition: moves
      // that merely exchanged the ids of singletons (every vertex still
      // alone) count as no move
      const bool changed = st.moved_any && job_cluster_counts(c, n, C, 1, nullptr)[0] < n;
      if (!changed || l + 1 == prm->max_levels) {
        top = l;
        cs.top_moved = changed;
        break;
      }
      maps.push_back(c.buf<int32_t>("lv.map" + std::to_string(l), (size_t)(n > 0 ? n : 1)));
      OwnedGraph &next = c.level_graph((size_t)l + 1);
      int64_t md = 0, mnd = 0;
      a = clk::now();
      compress_graph(c, G[l], C, next, maps.back(), wide, &md, nullptr, &mnd);
      ms_cp += std::chrono::duration<double, std::milli>(clk::now() - a).count();
      G.push_back(next.view());
      maxdeg.push_back(md);
      mindeg.push_back(mnd);
    }
    // The objective: contraction keeps it, so the clustering flattened onto
    // level 0 scores what the level-1 clustering scores on the level-1 graph
    // (summed over 850M instead of 3.6G arcs on the benchmark graph); only
    // the arcs of the vertices that level 0's refinement moves are read again.
    ObjectiveParts parts1;
    int32_t *P0 = nullptr;
    for (int l = top - 1; l >= 0; l--) {
      int32_t *C = Cl[l];
      if (l == 0 && obj) parts1 = objective_parts(c, G[1], Cl[1]);
      flatten(c, G[l].n, maps[l], Cl[l + 1], C);
      if (l == 0 && obj && prm->refine) {
        P0 = c.buf<int32_t>("ob.P", (size_t)G[0].n);
        HIPCHECK(hipMemcpyAsync(P0, C, (size_t)G[0].n * sizeof(int32_t), hipMemcpyDeviceToDevice, c.stream));
      }
      if (prm->refine) {
        lcc_bm_stats st;
        auto a = clk::now();
        best_moves(c, G[l], lam.p, lam.q, *prm, l, 1, C, BMShape{maxdeg[l], !wide, false, false, mindeg[l]}, st);
        ms_bm += std::chrono::duration<double, std::milli>(clk::now() - a).count();
        cs.iters_refine[l] = st.iterations;
        cs.moves_total += st.moves;
        cs.arcs_scanned_total += st.arcs_scanned;
      }
    }
    cs.clusters = canonical_labels(c, g->n, Cl[0], labels_out);
    if (obj) {
      i128 N;
      if (top == 0)
        N = objective_num(c, *g, lam.p, lam.q, Cl[0]);
      else if (P0)
        N = objective_after_refine(c, *g, lam.p, lam.q, P0, Cl[0], parts1);
      else  // no refinement: level 0 is the flattened level-1 clustering
        N = objective_from_sums(lam.p, lam.q, parts1.pairs2, parts1.win2, parts1.ssum);
      fill_objective(N, lam.q, obj);
    }
    c.sync();
    if (c.timing) c.collect_timing();
    cs.ms_best_move = ms_bm;
    cs.ms_compress = ms_cp;
    cs.ms_total = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    if (stats) *stats = cs;
  });
}

// The level loop of a batched run, after validation: coarsening with per-job
// Best-Moves and compression, then the unwinding with flatten and refinement,
// canonical per-job labels and (want_obj) per-job objectives.  shared_n1 > 0
// marks the jobs as identical copies of one graph of shared_n1 vertices.
static void batch_levels(Ctx &c, const lcc_graph *g, int64_t J, const std::vector<int64_t> &hstart,
                         const std::vector<int64_t> &vch, int64_t *d_start, const int64_t *d_jp, const int64_t *d_jq,
                         uint8_t *d_cont, const lcc_lambda *lambdas, const lcc_params *prm, const GraphSummary &s,
                         bool wide, int32_t *labels_out, bool want_obj, std::vector<lcc_job_out> &jo,
                         lcc_batch_stats &bs, int64_t shared_n1) {
  using clk = std::chrono::steady_clock;
  // level 0 job layout; per-level arrays live in the context
  std::vector<int32_t *> jidl, Cl, maps;
  std::vector<int64_t *> jbasel;
  std::vector<lcc_graph> G;
  std::vector<int64_t> maxdeg, mindeg;
  jidl.push_back(c.buf<int32_t>("lv.jid0", (size_t)g->n));
  batch_fill_jid(c, d_start, J, g->n, jidl.back());
  jbasel.push_back(d_start);
  G.push_back(*g);
  maxdeg.push_back(s.maxdeg);
  mindeg.push_back(0);
  std::vector<uint8_t> run((size_t)J), cont((size_t)J), moved((size_t)J);
  std::vector<int32_t> top((size_t)J, 0), iters((size_t)J);
  for (int64_t j = 0; j < J; j++) run[(size_t)j] = hstart[(size_t)j + 1] > hstart[(size_t)j];
  int maxtop = 0;
  double ms_bm = 0, ms_cp = 0;
  for (int l = 0;; l++) {
    const int64_t n = G[l].n;
    bs.n_level[l] = n;
    bs.arcs_level[l] = G[l].arcs;
    bs.levels = l + 1;
    Cl.push_back(c.buf<int32_t>("lv.C" + std::to_string(l), (size_t)(n > 0 ? n : 1)));
    int32_t *C = Cl.back();
    iota_i32(c, C, n);
    BatchLevel bl;
    bl.jobs = J;
    bl.jid = jidl[l];
    bl.jbase = jbasel[l];
    bl.jp = d_jp;
    bl.jq = d_jq;
    bl.active = run.data();
    bl.iters = iters.data();
    bl.moved_any = moved.data();
    bl.shared_n = l == 0 ? shared_n1 : 0;
    lcc_bm_stats st;
    auto a = clk::now();
    const bool simple = l > 0 || s.sorted_rows;
    best_moves(c, G[l], 0, 1, *prm, l, 0, C, BMShape{maxdeg[l], !wide, true, simple, mindeg[l]}, st, &bl);
    ms_bm += std::chrono::duration<double, std::milli>(clk::now() - a).count();
    bs.moves_total += st.moves;
    bs.arcs_scanned_total += st.arcs_scanned;
    // a job goes on only if its call changed its partition (fewer clusters
    // than vertices; ids exchanged between singletons count as no move)
    bool any_moved = false;
    for (int64_t j = 0; j < J; j++) any_moved = any_moved || (run[(size_t)j] && moved[(size_t)j]);
    if (any_moved) {
      const std::vector<int64_t> ncl = job_cluster_counts(c, n, C, J, jbasel[l]);
      std::vector<int64_t> jb((size_t)(J + 1));
      d2h(c, jb.data(), jbasel[l], jb.size() * sizeof(int64_t));
      for (int64_t j = 0; j < J; j++)
        if (moved[(size_t)j] && ncl[(size_t)j] >= jb[(size_t)(j + 1)] - jb[(size_t)j]) moved[(size_t)j] = 0;
    }
    bool any = false;
    for (int64_t j = 0; j < J; j++) {
      cont[(size_t)j] = 0;
      if (!run[(size_t)j]) continue;
      if (moved[(size_t)j] && l + 1 < prm->max_levels) {
        cont[(size_t)j] = 1;
        any = true;
      } else {
        top[(size_t)j] = l;
        jo[(size_t)j].top_moved = moved[(size_t)j];
      }
    }
    if (!any) {
      maxtop = l;
      break;
    }
    h2d(c, d_cont, cont.data(), (size_t)J);
    maps.push_back(c.buf<int32_t>("lv.map" + std::to_string(l), (size_t)(n > 0 ? n : 1)));
    OwnedGraph &next = c.level_graph((size_t)l + 1);
    // the next level's job of every vertex and job bases
    jidl.push_back(c.buf<int32_t>("lv.jid" + std::to_string(l + 1), (size_t)(n > 0 ? n : 1)));
    jbasel.push_back(c.buf<int64_t>("lv.jbase" + std::to_string(l + 1), (size_t)(J + 1)));
    CompressJobs cj;
    cj.jobs = J;
    cj.jid = jidl[l];
    cj.jcont = d_cont;
    cj.jid_next = jidl[l + 1];
    cj.jbase_next = jbasel[l + 1];
    int64_t md = 0;
    a = clk::now();
    int64_t mnd = 0;
    compress_graph(c, G[l], C, next, maps.back(), wide, &md, &cj, &mnd);
    ms_cp += std::chrono::duration<double, std::milli>(clk::now() - a).count();
    G.push_back(next.view());
    maxdeg.push_back(md);
    mindeg.push_back(mnd);
    run = cont;
  }
  for (int l = maxtop - 1; l >= 0; l--) {
    int32_t *C = Cl[l];
    // jobs that stopped coarsening at this level keep their clustering (map < 0)
    batch_flatten(c, G[l].n, maps[l], Cl[l + 1], jidl[l], jbasel[l], jbasel[l + 1], C);
    if (prm->refine) {
      bool any = false;
      for (int64_t j = 0; j < J; j++) {
        run[(size_t)j] = top[(size_t)j] > l;
        any = any || run[(size_t)j];
      }
      if (!any) continue;
      BatchLevel bl;
      bl.jobs = J;
      bl.jid = jidl[l];
      bl.jbase = jbasel[l];
      bl.jp = d_jp;
      bl.jq = d_jq;
      bl.active = run.data();
      bl.iters = iters.data();
      bl.moved_any = moved.data();
      bl.shared_n = l == 0 ? shared_n1 : 0;
      lcc_bm_stats st;
      auto a = clk::now();
      best_moves(c, G[l], 0, 1, *prm, l, 1, C, BMShape{maxdeg[l], !wide, false, false, mindeg[l]}, st, &bl);
      ms_bm += std::chrono::duration<double, std::milli>(clk::now() - a).count();
      bs.moves_total += st.moves;
      bs.arcs_scanned_total += st.arcs_scanned;
    }
  }
  // canonical labels over the packed graph, then made job-local
  const int64_t n0 = g->n;
  int32_t *glab = c.buf<int32_t>("bt.glab", (size_t)n0);
  const int64_t total = canonical_labels(c, n0, Cl[0], glab);
  batch_local_labels(c, glab, jidl[0], d_start, n0, labels_out);
  std::vector<int32_t> first = batch_first_labels(c, glab, d_start, J);
  // clusters of job j are the global labels [first_j, first of the next non-empty job)
  int64_t nxt = total;
  for (int64_t j = J - 1; j >= 0; j--) {
    if (first[(size_t)j] < 0) continue;
    jo[(size_t)j].clusters = nxt - first[(size_t)j];
    nxt = first[(size_t)j];
  }
  for (int64_t j = 0; j < J; j++) jo[(size_t)j].levels = top[(size_t)j] + 1;
  if (want_obj) {
    int64_t *K = c.buf<int64_t>("bt.K", (size_t)n0);
    int64_t *KK = c.buf<int64_t>("bt.KK", (size_t)n0);
    cluster_sums_k_kk(c, *g, glab, K, KK);
    std::vector<int64_t> cch;
    for (int64_t j = 0; j < J; j++) {
      if (first[(size_t)j] < 0) continue;
      const int64_t xb = first[(size_t)j], xe = xb + jo[(size_t)j].clusters;
      for (int64_t x = xb; x < xe; x += BATCH_CHUNK) {
        cch.push_back(j);
        cch.push_back(x);
        cch.push_back(std::min<int64_t>(x + BATCH_CHUNK, xe));
      }
    }
    std::vector<i128> intra, self, pairs;
    batch_objective_parts(c, *g, glab, vch, K, KK, cch, intra, self, pairs);
    std::vector<i128> w2((size_t)J, 0), ss((size_t)J, 0), pp((size_t)J, 0);
    for (size_t i = 0; i < vch.size() / 3; i++) {
      w2[(size_t)vch[3 * i]] += intra[i];
      ss[(size_t)vch[3 * i]] += self[i];
    }
    for (size_t i = 0; i < cch.size() / 3; i++) pp[(size_t)cch[3 * i]] += pairs[i];
    for (int64_t j = 0; j < J; j++) {
      const size_t u = (size_t)j;
      const i128 N = (i128)lambdas[j].q * (ss[u] + w2[u] / 2) - (i128)lambdas[j].p * (pp[u] / 2);
      fill_objective(N, lambdas[j].q, &jo[u].obj);
    }
  }
  c.sync();
  if (c.timing) c.collect_timing();
  bs.ms_best_move = ms_bm;
  bs.ms_compress = ms_cp;
}

// Automatic score pruning (score_pruning = 0) turns on where a level has at
// least 2^23 vertices, because there the cluster totals miss the caches.  A
// batch or a sweep packs many jobs into one level whose size says nothing
// about that: each job reads only its own totals.  So unless one job has that
// many vertices, automatic means off here (the 16-resolution sweep of a
// 1M-vertex graph: 501 -> 424 ms, results identical, as they are either way).
constexpr int64_t PRUNE_JOB_MIN_N = (int64_t)1 << 23;

static lcc_params batch_params(const lcc_params &prm, int64_t largest_job) {
  lcc_params p = prm;
  if (p.score_pruning == 0 && largest_job < PRUNE_JOB_MIN_N) p.score_pruning = -1;
  return p;
}

lcc_status lcc_cluster_batch(lcc_ctx *ctx, const lcc_graph *g, int64_t jobs, const int64_t *job_start,
                             const lcc_lambda *lambdas, const lcc_params *prm, int32_t *labels_out,
                             lcc_job_out *jobs_out, lcc_batch_stats *stats, void *stream) {
  return guarded([&] {
    if (!ctx) fail(LCC_ERR_INVALID_ARG, "ctx is NULL");
    Ctx &c = ctx->c;
    check_params(prm);
    if (prm->max_levels < 1 || prm->max_levels > LCC_MAX_LEVELS)
      fail(LCC_ERR_INVALID_ARG, "max_levels must be in [1, 64]");
    if (prm->stop_after_subrounds != 0) fail(LCC_ERR_INVALID_ARG, "stop_after_subrounds must be 0 in a batch");
    if (jobs < 0 || jobs > INT32_MAX) fail(LCC_ERR_INVALID_ARG, "jobs must be in [0, 2^31)");
    if (jobs > 0 && (!job_start || !lambdas)) fail(LCC_ERR_INVALID_ARG, "job_start or lambdas is NULL");
    begin(c, stream, prm);
    check_graph_args(c, g);
    if (jobs == 0 && g->n != 0) fail(LCC_ERR_INVALID_ARG, "a batch without jobs must have n = 0");
    if (jobs > 0) {
      if (job_start[0] != 0 || job_start[jobs] != g->n)
        fail(LCC_ERR_INVALID_ARG, "job_start must run from 0 to n");
      for (int64_t j = 0; j < jobs; j++) {
        if (job_start[j + 1] < job_start[j]) fail(LCC_ERR_INVALID_ARG, "job_start must be non-decreasing");
        check_lambda(lambdas[j]);
      }
    }
    check_dev(c, labels_out, (size_t)g->n * sizeof(int32_t), "labels_out");
    using clk = std::chrono::steady_clock;
    auto t0 = clk::now();
    lcc_batch_stats bs;
    std::memset(&bs, 0, sizeof(bs));
    std::vector<lcc_job_out> jo((size_t)jobs);
    for (auto &o : jo) {
      std::memset(&o, 0, sizeof(o));
      o.levels = 1;
      o.obj.den = 1;
    }
    if (g->n == 0) {
      for (int64_t j = 0; j < jobs; j++) fill_objective(0, lambdas[j].q, &jo[(size_t)j].obj);
      if (jobs_out) std::copy(jo.begin(), jo.end(), jobs_out);
      bs.levels = 1;
      if (stats) *stats = bs;
      return;
    }
    const int64_t J = jobs;
    const std::vector<int64_t> hstart(job_start, job_start + J + 1);
    int64_t largest = 0;
    for (int64_t j = 0; j < J; j++) largest = std::max(largest, hstart[(size_t)j + 1] - hstart[(size_t)j]);
    const lcc_params prb = batch_params(*prm, largest);
    prm = &prb;
    // vertex chunks of level 0: (job, first, end), never spanning two jobs
    std::vector<int64_t> vch;
    for (int64_t j = 0; j < J; j++)
      for (int64_t b = hstart[(size_t)j]; b < hstart[(size_t)j + 1]; b += BATCH_CHUNK) {
        vch.push_back(j);
        vch.push_back(b);
        vch.push_back(std::min<int64_t>(b + BATCH_CHUNK, hstart[(size_t)j + 1]));
      }
    int64_t *d_start = c.buf<int64_t>("bt.start", (size_t)(J + 1));
    int64_t *d_jp = c.buf<int64_t>("bt.jp", (size_t)J);
    int64_t *d_jq = c.buf<int64_t>("bt.jq", (size_t)J);
    uint8_t *d_cont = c.buf<uint8_t>("bt.cont", (size_t)J);
    {
      std::vector<int64_t> hp((size_t)J), hq((size_t)J);
      for (int64_t j = 0; j < J; j++) {
        hp[(size_t)j] = lambdas[j].p;
        hq[(size_t)j] = lambdas[j].q;
      }
      h2d(c, d_start, hstart.data(), (size_t)(J + 1) * sizeof(int64_t));
      h2d(c, d_jp, hp.data(), (size_t)J * sizeof(int64_t));
      h2d(c, d_jq, hq.data(), (size_t)J * sizeof(int64_t));
      c.sync();
    }
    // validation: structure of the packed graph, then per-job sums (arcs that
    // leave their job, and each job's overflow bounds under its own lambda)
    GraphSummary s = summarize_graph(c, *g, nullptr, prm->validate != 0);
    if (!s.ok) fail(LCC_ERR_INVALID_ARG, s.why);
    bool wide = false;
    {
      std::vector<uint64_t> part = batch_vertex_sums(c, *g, d_start, vch, true);
      std::vector<GraphSummary> sj((size_t)J);
      auto sat = [](uint64_t a, uint64_t b) {
        uint64_t r = a + b;
        return r < a ? ~0ull : r;
      };
      for (size_t i = 0; i < vch.size() / 3; i++) {
        GraphSummary &t = sj[(size_t)vch[3 * i]];
        const uint64_t *r = &part[6 * i];
        t.wabs2 = sat(t.wabs2, r[0]);
        t.ktot = sat(t.ktot, r[1]);
        t.kksum = sat(t.kksum, r[2]);
        t.sabs = sat(t.sabs, r[3]);
        t.negative = t.negative || r[4];
        if (r[5]) fail(LCC_ERR_INVALID_ARG, "an arc of job " + std::to_string(vch[3 * i]) + " leaves the job");
      }
      for (int64_t j = 0; j < J; j++) {
        std::string why;
        if (overflow_bounds(sj[(size_t)j], lambdas[j].p, lambdas[j].q, &why) != LCC_OK)
          fail(LCC_ERR_OVERFLOW, "job " + std::to_string(j) + ": " + why);
        wide = wide || wide_weights(sj[(size_t)j]);
      }
    }
    batch_levels(c, g, J, hstart, vch, d_start, d_jp, d_jq, d_cont, lambdas, prm, s, wide, labels_out,
                 jobs_out != nullptr, jo, bs, 0);
    bs.ms_total = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    if (jobs_out) std::copy(jo.begin(), jo.end(), jobs_out);
    if (stats) *stats = bs;
  });
}

lcc_status lcc_sweep(lcc_ctx *ctx, const lcc_graph *g, int64_t count, const lcc_lambda *lambdas,
                     const lcc_params *prm, int32_t *labels_out, lcc_job_out *jobs_out, lcc_batch_stats *stats,
                     void *stream) {
  return guarded([&] {
    if (!ctx) fail(LCC_ERR_INVALID_ARG, "ctx is NULL");
    Ctx &c = ctx->c;
    check_params(prm);
    if (prm->max_levels < 1 || prm->max_levels > LCC_MAX_LEVELS)
      fail(LCC_ERR_INVALID_ARG, "max_levels must be in [1, 64]");
    if (prm->stop_after_subrounds != 0) fail(LCC_ERR_INVALID_ARG, "stop_after_subrounds must be 0 in a sweep");
    if (count < 0 || count > LCC_SWEEP_MAX) fail(LCC_ERR_INVALID_ARG, "count must be in [0, 16]");
    if (count > 0 && !lambdas) fail(LCC_ERR_INVALID_ARG, "lambdas is NULL");
    begin(c, stream, prm);
    check_graph_args(c, g);
    for (int64_t j = 0; j < count; j++) check_lambda(lambdas[j]);
    const int64_t J = count, n1 = g->n;
    if (J * n1 >= ((int64_t)1 << 30)) fail(LCC_ERR_INVALID_ARG, "count * n must be below 2^30");
    check_dev(c, labels_out, (size_t)(J * n1) * sizeof(int32_t), "labels_out");
    using clk = std::chrono::steady_clock;
    auto t0 = clk::now();
    lcc_batch_stats bs;
    std::memset(&bs, 0, sizeof(bs));
    std::vector<lcc_job_out> jo((size_t)J);
    for (auto &o : jo) {
      std::memset(&o, 0, sizeof(o));
      o.levels = 1;
      o.obj.den = 1;
    }
    if (J == 0 || n1 == 0) {
      for (int64_t j = 0; j < J; j++) fill_objective(0, lambdas[j].q, &jo[(size_t)j].obj);
      if (jobs_out) std::copy(jo.begin(), jo.end(), jobs_out);
      bs.levels = 1;
      if (stats) *stats = bs;
      return;
    }
    // the graph is validated once; every resolution checks its own bounds
    GraphSummary s = summarize_graph(c, *g, nullptr, prm->validate != 0);
    if (!s.ok) fail(LCC_ERR_INVALID_ARG, s.why);
    for (int64_t j = 0; j < J; j++) {
      std::string why;
      if (overflow_bounds(s, lambdas[j].p, lambdas[j].q, &why) != LCC_OK)
        fail(LCC_ERR_OVERFLOW, "lambda " + std::to_string(j) + ": " + why);
    }
    const bool wide = wide_weights(s);
    const lcc_params prb = batch_params(*prm, n1);
    prm = &prb;
    // J copies packed block-diagonally (level 0 of the batch)
    const lcc_graph gp = batch_replicate(c, *g, J, c.level_graph(0));
    std::vector<int64_t> hstart((size_t)J + 1), vch;
    for (int64_t j = 0; j <= J; j++) hstart[(size_t)j] = j * n1;
    for (int64_t j = 0; j < J; j++)
      for (int64_t b = j * n1; b < (j + 1) * n1; b += BATCH_CHUNK) {
        vch.push_back(j);
        vch.push_back(b);
        vch.push_back(std::min<int64_t>(b + BATCH_CHUNK, (j + 1) * n1));
      }
    int64_t *d_start = c.buf<int64_t>("bt.start", (size_t)(J + 1));
    int64_t *d_jp = c.buf<int64_t>("bt.jp", (size_t)J);
    int64_t *d_jq = c.buf<int64_t>("bt.jq", (size_t)J);
    uint8_t *d_cont = c.buf<uint8_t>("bt.cont", (size_t)J);
    {
      std::vector<int64_t> hp((size_t)J), hq((size_t)J);
      for (int64_t j = 0; j < J; j++) {
        hp[(size_t)j] = lambdas[j].p;
        hq[(size_t)j] = lambdas[j].q;
      }
      h2d(c, d_start, hstart.data(), (size_t)(J + 1) * sizeof(int64_t));
      h2d(c, d_jp, hp.data(), (size_t)J * sizeof(int64_t));
      h2d(c, d_jq, hq.data(), (size_t)J * sizeof(int64_t));
      c.sync();
    }
    batch_levels(c, &gp, J, hstart, vch, d_start, d_jp, d_jq, d_cont, lambdas, prm, s, wide, labels_out,
                 jobs_out != nullptr, jo, bs, n1);
    bs.ms_total = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    if (jobs_out) std::copy(jo.begin(), jo.end(), jobs_out);
    if (stats) *stats = bs;
  });
}

lcc_status lcc_ctx_kernel_stats(lcc_ctx *ctx, lcc_kernel_stat *out, int32_t max, int32_t *count) {
  return guarded([&] {
    if (!ctx || !count || (max > 0 && !out)) fail(LCC_ERR_INVALID_ARG, "NULL argument");
    int32_t i = 0;
    for (auto &kv : ctx->c.kstats) {
      if (i < max) {
        lcc_kernel_stat &o = out[i];
        std::memset(&o, 0, sizeof(o));
        std::strncpy(o.name, kv.first.c_str(), sizeof(o.name) - 1);
        o.launches = kv.second.launches;
        o.total_ms = kv.second.ms;
        o.bytes = kv.second.bytes;
        o.items = kv.second.items;
      }
      i++;
    }
    *count = i;
  });
}

lcc_status lcc_ctx_reset_kernel_stats(lcc_ctx *ctx) {
  return guarded([&] {
    if (!ctx) fail(LCC_ERR_INVALID_ARG, "ctx is NULL");
    ctx->c.kstats.clear();
  });
}

}  // extern "C"
