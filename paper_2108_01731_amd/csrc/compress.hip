// compress.hip -- graph compression (paper Sec. 3.1 / Appendix B), flatten,
// canonical labels and per-cluster totals on gfx950.
//
// Compress: clusters are renumbered by the rank of their id among non-empty
// ids (a prefix sum over presence flags).  The input graph is symmetric with
// equal weights both ways, so the coarse weight of a cluster pair X < Y is
// the sum over the arcs from X into Y alone: only those "upper" arcs become
// keys (X << b | Y, 64-bit, or 32-bit when 2b <= 32) carrying their weight.
// A stable LSD radix sort over the 2b significant bits groups equal pairs;
// heads of equal-key runs give the unique upper pairs, and run sums come from
// an inclusive prefix sum (differences at run boundaries, exact in int64) or,
// for unit weights, from run lengths.  The unique pairs, in (X, Y) order, are
// the upper part of each coarse row.  Re-keyed as Y << b | X and sorted
// stably on the high b bits they come out in (Y, X) order: the lower part of
// each row, already in column order.  Row r of the coarse graph is its lower
// part followed by its upper part, so its offset is the number of upper pairs
// with X < r plus the number of lower entries with Y < r (two lower bounds).
// Per-cluster sums of k, kk and the self weight come from a radix sort of the
// vertices by cluster followed by prefix-sum differences: no atomics, so huge
// clusters cost nothing extra.
#include "ops.hpp"
#include "prims.hpp"

namespace lcc {

constexpr int CP_NT = 256;

__global__ void k_iota(int32_t *__restrict__ a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = (int32_t)i;
}

__global__ void k_copy_u32(const int32_t *__restrict__ a, uint32_t *__restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (uint32_t)a[i];
}

inline unsigned grid_for(int64_t n, int nt = 256) {
  int64_t g = cdiv(n > 0 ? n : 1, nt);
  return (unsigned)(g < 65536 ? g : 65536);
}

void iota_i32(Ctx &c, int32_t *C, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(256), 0, c.stream, C, n);
  LAUNCHCHECK();
}

// ------------------------------------------------------ sort vertices by key

struct ByKey {
  const uint32_t *key;  // sorted keys
  const int32_t *perm;  // vertex at each sorted position (ascending inside a key)
};

// Stable sort of the vertices 0..n-1 by key[v] in [0, nkeys).
static ByKey sort_by_key(Ctx &c, const int32_t *key, int64_t n, int64_t nkeys, const char *tag) {
  std::string t(tag);
  uint32_t *k0 = c.buf<uint32_t>(t + ".k0", (size_t)n);
  uint32_t *k1 = c.buf<uint32_t>(t + ".k1", (size_t)n);
  int32_t *p0 = c.buf<int32_t>(t + ".p0", (size_t)n);
  int32_t *p1 = c.buf<int32_t>(t + ".p1", (size_t)n);
  hipLaunchKernelGGL(k_copy_u32, dim3(grid_for(n)), dim3(256), 0, c.stream, key, k0, n);
  LAUNCHCHECK();
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(256), 0, c.stream, p0, n);
  LAUNCHCHECK();
  bool flip = radix_sort<uint32_t, int32_t, true>(c, k0, p0, k1, p1, n, bits_for(nkeys - 1), (t + ".rs").c_str());
  return flip ? ByKey{k1, p1} : ByKey{k0, p0};
}

// start[key] = first sorted position of the key (only keys that occur).
__global__ void k_seg_heads(const uint32_t *__restrict__ sk, int64_t n, int64_t *__restrict__ start) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (i == 0 || sk[i] != sk[i - 1]) start[sk[i]] = i;
}

enum GatherKind { G_K = 0, G_KK = 1, G_SELF2 = 2 };

// val[i] for the vertex at sorted position i: k, kk (or k^2), or 2*s + intra.
__global__ void k_seg_gather(const int32_t *__restrict__ perm, int64_t n, int kind, const int64_t *__restrict__ k,
                             const int64_t *__restrict__ kk, const int64_t *__restrict__ s,
                             const int64_t *__restrict__ intra, int64_t *__restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = perm[i];
    int64_t x;
    if (kind == G_K) x = k[v];
    else if (kind == G_KK) x = kk ? kk[v] : k[v] * k[v];
    else x = 2 * (s ? s[v] : 0) + (intra ? intra[v] : 0);
    out[i] = x;
  }
}

// At the last position of each key's run: out[key] = run sum (from the
// inclusive prefix P), cnt[key] = run length (if cnt), halve if requested.
__global__ void k_seg_tails(const uint32_t *__restrict__ sk, int64_t n, const int64_t *__restrict__ start,
                            const int64_t *__restrict__ P, int64_t *__restrict__ out, int32_t *__restrict__ cnt,
                            int halve) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (i == n - 1 || sk[i] != sk[i + 1]) {
      const uint32_t x = sk[i];
      const int64_t st = start[x];
      if (out) {
        int64_t sum = P[i] - (st > 0 ? P[st - 1] : 0);
        out[x] = halve ? sum / 2 : sum;
      }
      if (cnt) cnt[x] = (int32_t)(i - st + 1);
    }
  }
}

// Sums of one per-vertex quantity per key (keys that do not occur get 0).
static void seg_sum(Ctx &c, const ByKey &bk, int64_t n, int64_t nkeys, const int64_t *start, int kind,
                    const lcc_graph &g, const int64_t *intra, int64_t *out, int32_t *cnt, bool halve) {
  int64_t *vals = c.buf<int64_t>("seg.vals", (size_t)n);
  if (out) HIPCHECK(hipMemsetAsync(out, 0, (size_t)nkeys * sizeof(int64_t), c.stream));
  if (cnt) HIPCHECK(hipMemsetAsync(cnt, 0, (size_t)nkeys * sizeof(int32_t), c.stream));
  if (out) {
    hipLaunchKernelGGL(k_seg_gather, dim3(grid_for(n)), dim3(256), 0, c.stream, bk.perm, n, kind, g.k, g.kk, g.s,
                       intra, vals);
    LAUNCHCHECK();
    scan<int64_t, int64_t>(c, vals, vals, n, true, (int64_t *)nullptr);
  }
  hipLaunchKernelGGL(k_seg_tails, dim3(grid_for(n)), dim3(256), 0, c.stream, bk.key, n, start, vals, out, cnt,
                     (int)halve);
  LAUNCHCHECK();
}

void cluster_totals(Ctx &c, int64_t n, const int32_t *C, const int64_t *k, int64_t *K, int32_t *cnt) {
  if (n <= 0) return;
  ByKey bk = sort_by_key(c, C, n, n, "ct");
  int64_t *start = c.buf<int64_t>("ct.start", (size_t)n);
  hipLaunchKernelGGL(k_seg_heads, dim3(grid_for(n)), dim3(256), 0, c.stream, bk.key, n, start);
  LAUNCHCHECK();
  lcc_graph g;
  std::memset(&g, 0, sizeof(g));
  g.k = k;
  seg_sum(c, bk, n, n, start, G_K, g, nullptr, K, cnt, false);
}

// Per-cluster sums of k and kk (kk = k^2 when absent) for ids in [0, n).
void cluster_sums_k_kk(Ctx &c, const lcc_graph &g, const int32_t *C, int64_t *K, int64_t *KK) {
  const int64_t n = g.n;
  if (n <= 0) return;
  ByKey bk = sort_by_key(c, C, n, n, "ct");
  int64_t *start = c.buf<int64_t>("ct.start", (size_t)n);
  hipLaunchKernelGGL(k_seg_heads, dim3(grid_for(n)), dim3(256), 0, c.stream, bk.key, n, start);
  LAUNCHCHECK();
  seg_sum(c, bk, n, n, start, G_K, g, nullptr, K, nullptr, false);
  seg_sum(c, bk, n, n, start, G_KK, g, nullptr, KK, nullptr, false);
}

// ------------------------------------------------------------------ flatten

__global__ void k_flatten(const int32_t *__restrict__ map, const int32_t *__restrict__ Cn, int32_t *__restrict__ C,
                          int64_t n) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t m = map[v];
    if (m >= 0) C[v] = Cn[m];  // map < 0: the vertex's job stopped coarsening at this level
  }
}

void flatten(Ctx &c, int64_t n, const int32_t *map, const int32_t *Cnext, int32_t *C) {
  if (n <= 0) return;
  Ctx::Timer tm(&c, "flatten", 12.0 * (double)n, (double)n);
  hipLaunchKernelGGL(k_flatten, dim3(grid_for(n)), dim3(256), 0, c.stream, map, Cnext, C, n);
  LAUNCHCHECK();
}

// ---------------------------------------------------------- canonical labels

__global__ void k_first_members(const uint32_t *__restrict__ sk, const int32_t *__restrict__ perm, int64_t n,
                                uint8_t *__restrict__ first) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (i == 0 || sk[i] != sk[i - 1]) first[perm[i]] = 1;
}

__global__ void k_cluster_label(const uint32_t *__restrict__ sk, const int32_t *__restrict__ perm, int64_t n,
                                const int32_t *__restrict__ rank, int32_t *__restrict__ lab) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (i == 0 || sk[i] != sk[i - 1]) lab[sk[i]] = rank[perm[i]];
}

__global__ void k_apply_label(const int32_t *__restrict__ C, const int32_t *__restrict__ lab, int32_t *__restrict__ out,
                              int64_t n) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    out[v] = lab[C[v]];
}

int64_t canonical_labels(Ctx &c, int64_t n, const int32_t *C, int32_t *labels) {
  if (n <= 0) return 0;
  Ctx::Timer tm(&c, "labels", 0.0, (double)n);
  ByKey bk = sort_by_key(c, C, n, n, "lab");
  uint8_t *first = c.buf<uint8_t>("lab.first", (size_t)n);
  int32_t *rank = c.buf<int32_t>("lab.rank", (size_t)n);
  int32_t *lab = c.buf<int32_t>("lab.lab", (size_t)n);
  int64_t *tot = c.buf<int64_t>("lab.tot", 1);
  HIPCHECK(hipMemsetAsync(first, 0, (size_t)n, c.stream));
  hipLaunchKernelGGL(k_first_members, dim3(grid_for(n)), dim3(256), 0, c.stream, bk.key, bk.perm, n, first);
  LAUNCHCHECK();
  int32_t *tot32 = reinterpret_cast<int32_t *>(tot);
  scan<uint8_t, int32_t>(c, first, rank, n, false, tot32);
  hipLaunchKernelGGL(k_cluster_label, dim3(grid_for(n)), dim3(256), 0, c.stream, bk.key, bk.perm, n, rank, lab);
  LAUNCHCHECK();
  hipLaunchKernelGGL(k_apply_label, dim3(grid_for(n)), dim3(256), 0, c.stream, C, lab, labels, n);
  LAUNCHCHECK();
  int32_t h = 0;
  d2h(c, &h, tot32, sizeof(int32_t));
  return h;
}

// ------------------------------------------------------------------ compress

// In batched runs only the vertices of continuing jobs are kept; the others
// get map = -1 and take no part in the contracted graph.
__device__ __forceinline__ bool kept(const int32_t *jid, const uint8_t *jcont, int64_t v) {
  return !jid || jcont[jid[v]];
}

__global__ void k_mark_present(const int32_t *__restrict__ C, int64_t n, const int32_t *__restrict__ jid,
                               const uint8_t *__restrict__ jcont, uint8_t *__restrict__ present) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (kept(jid, jcont, v)) present[C[v]] = 1;
}

__global__ void k_map(const int32_t *__restrict__ C, const int32_t *__restrict__ rank, int64_t n,
                      const int32_t *__restrict__ jid, const uint8_t *__restrict__ jcont, int32_t *__restrict__ map) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    map[v] = kept(jid, jcont, v) ? rank[C[v]] : -1;
}

// Distinct cluster ids of a clustering (the recursion of Parallel-CC goes on
// only if a coarsening call changed the partition, i.e. left fewer clusters
// than vertices).
__global__ void k_flag_ids(const int32_t *__restrict__ C, int64_t n, uint8_t *__restrict__ present) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    present[C[v]] = 1;
}

// out[j] = rank[jbase[j]], out[J + 1 + j] = jbase[j] for j <= J.
__global__ void k_rank_at(const int32_t *__restrict__ rank, const int64_t *__restrict__ jbase, int64_t J,
                          int64_t *__restrict__ out) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= J; j += (int64_t)gridDim.x * blockDim.x) {
    out[j] = rank[jbase[j]];
    out[J + 1 + j] = jbase[j];
  }
}

std::vector<int64_t> job_cluster_counts(Ctx &c, int64_t n, const int32_t *C, int64_t J, const int64_t *jbase) {
  std::vector<int64_t> counts((size_t)J, 0);
  if (n <= 0 || J <= 0) return counts;
  uint8_t *present = c.buf<uint8_t>("cc.present", (size_t)n);
  int32_t *rank = c.buf<int32_t>("cc.rank", (size_t)n + 1);
  int64_t *out = c.buf<int64_t>("cc.out", (size_t)(2 * (J + 1)));
  HIPCHECK(hipMemsetAsync(present, 0, (size_t)n, c.stream));
  hipLaunchKernelGGL(k_flag_ids, dim3(grid_for(n)), dim3(256), 0, c.stream, C, n, present);
  LAUNCHCHECK();
  scan<uint8_t, int32_t>(c, present, rank, n, false, rank + n);
  if (jbase) {
    hipLaunchKernelGGL(k_rank_at, dim3(grid_for(J + 1)), dim3(256), 0, c.stream, (const int32_t *)rank, jbase, J, out);
    LAUNCHCHECK();
    std::vector<int64_t> h((size_t)(2 * (J + 1)));
    d2h(c, h.data(), out, h.size() * sizeof(int64_t));
    for (int64_t j = 0; j < J; j++) counts[(size_t)j] = h[(size_t)(j + 1)] - h[(size_t)j];
  } else {
    int32_t t = 0;
    d2h(c, &t, rank + n, sizeof(t));
    counts[0] = t;
  }
  return counts;
}

// Sort keys for the per-cluster sums: dropped vertices go to the extra key n2.
__global__ void k_keys_with_sentinel(const int32_t *__restrict__ map, int64_t n, int32_t n2, int32_t *__restrict__ key) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    key[v] = map[v] < 0 ? n2 : map[v];
}

// Job of every contracted vertex, and the job bases of the next level.
__global__ void k_next_jid(const int32_t *__restrict__ map, const int32_t *__restrict__ jid, int64_t n,
                           int32_t *__restrict__ jid_next) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (map[v] >= 0) jid_next[map[v]] = jid[v];
}

__global__ void k_next_jbase(const int32_t *__restrict__ jid_next, int64_t n2, int64_t jobs,
                             int64_t *__restrict__ jbase_next) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= jobs; j += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = n2;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (jid_next[mid] < j) lo = mid + 1;
      else hi = mid;
    }
    jbase_next[j] = lo;
  }
}

// G lanes per vertex: number of upper arcs (into a cluster of higher rank)
// and weight of intra arcs; mu[e] = map[col[e]] is kept for the emit pass,
// which then streams it instead of gathering map a second time.  U rounds of
// G arcs are loaded, and their map entries gathered, together.
template <int G, int U, int WK>
__global__ __launch_bounds__(CP_NT) void k_cp_count(const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                    const void *__restrict__ wt, const int32_t *__restrict__ map,
                                                    int64_t n, int64_t *__restrict__ inter,
                                                    int64_t *__restrict__ intra, int32_t *__restrict__ mu) {
  const int gl = threadIdx.x % G;
  const int64_t v = (int64_t)blockIdx.x * (CP_NT / G) + threadIdx.x / G;
  int64_t ni = 0, wi = 0;
  if (v < n && map[v] >= 0) {
    const int32_t mv = map[v];
    const int64_t end = off[v + 1];
    for (int64_t e0 = off[v] + gl; e0 < end; e0 += U * G) {
      int32_t u[U], m[U];
#pragma unroll
      for (int j = 0; j < U; j++) {
        const int64_t e = e0 + j * G;
        u[j] = e < end ? col[e] : -1;
      }
#pragma unroll
      for (int j = 0; j < U; j++) m[j] = u[j] >= 0 ? map[u[j]] : 0;
#pragma unroll
      for (int j = 0; j < U; j++) {
        const int64_t e = e0 + j * G;
        if (e < end) {
          mu[e] = m[j];
          if (m[j] > mv) ni++;
          else if (m[j] == mv) wi += load_w<WK>(wt, e);
        }
      }
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    ni += __shfl_xor(ni, o, WAVE);
    wi += __shfl_xor(wi, o, WAVE);
  }
  if (v < n && gl == 0) {
    inter[v] = ni;
    intra[v] = wi;
  }
}

// G lanes per vertex: writes the vertex's upper arcs (map[u] > map[v]), in
// row order, as (map[v] << b | map[u], w) starting at eoff[v].  U rounds of
// G arcs are loaded before any is written, so a wave keeps U loads per lane
// in flight for each of its 64 / G vertices.  K / V: 64-bit keys and
// weights, or 32-bit ones where 2b <= 32 and the weights are at most 32-bit
// (the sort then moves half the bytes).
template <int G, int U, int WK, bool WEIGHTED, class K, class V>
__global__ __launch_bounds__(CP_NT) void k_cp_emit(const int64_t *__restrict__ off, const int32_t *__restrict__ mu,
                                                   const void *__restrict__ wt, const int32_t *__restrict__ map,
                                                   int64_t n, const int64_t *__restrict__ eoff, int b,
                                                   K *__restrict__ keys, V *__restrict__ vals) {
  const int gl = threadIdx.x % G;
  const int lane = lane_id();
  const int g0 = lane - gl;
  const int64_t v = (int64_t)blockIdx.x * (CP_NT / G) + threadIdx.x / G;
  const uint64_t gmask = G >= 64 ? ~0ull : ((1ull << (G & 63)) - 1);
  int64_t beg = 0, end = 0, pos = 0;
  int32_t mv = 0;
  if (v < n && map[v] >= 0) {
    beg = off[v];
    end = off[v + 1];
    pos = eoff[v];
    mv = map[v];
  }
  // every lane of the wave runs the same number of rounds (ballots need it)
  int64_t maxr = cdiv(end - beg, G);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    int64_t y = __shfl_xor(maxr, o, WAVE);
    maxr = y > maxr ? y : maxr;
  }
  for (int64_t r = 0; r < maxr; r += U) {
    int32_t m[U];
    int64_t w[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t e = beg + (r + u) * G + gl;
      m[u] = e < end ? mu[e] : mv;  // mv: not an upper arc
      w[u] = WEIGHTED && e < end ? load_w<WK>(wt, e) : 0;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const bool is_up = m[u] > mv;
      const uint64_t bal = (__ballot(is_up) >> g0) & gmask;
      if (is_up) {
        const int64_t at = pos + __popcll(bal & ((1ull << gl) - 1));
        keys[at] = ((K)(uint32_t)mv << b) | (K)(uint32_t)m[u];
        if constexpr (WEIGHTED) vals[at] = (V)w[u];
      }
      pos += __popcll(bal);
    }
  }
}

template <class K>
__global__ void k_cp_heads(const K *__restrict__ keys, int64_t T, uint8_t *__restrict__ head) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < T; i += (int64_t)gridDim.x * blockDim.x)
    head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

__global__ void k_cp_ustart(const uint8_t *__restrict__ head, const int64_t *__restrict__ uidx, int64_t T,
                            int64_t *__restrict__ ustart) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < T; i += (int64_t)gridDim.x * blockDim.x)
    if (head[i]) ustart[uidx[i]] = i;
}

// Unique upper pair j = (X, Y), X < Y, from the sorted run starting at
// ustart[j]: re-keyed as Y << b | X with its summed weight, into two copies
// (one kept for placing the upper parts, one sorted into the lower parts).
template <class K, class WOut>
__global__ void k_cp_pairs(const K *__restrict__ keys, const int64_t *__restrict__ ustart, int64_t U, int64_t T,
                           const int64_t *__restrict__ P, int b, K *__restrict__ tkeep, K *__restrict__ tsort,
                           WOut *__restrict__ wkeep, WOut *__restrict__ wsort) {
  const uint64_t mask = (1ull << b) - 1;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < U; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = ustart[j];
    const int64_t e = j + 1 < U ? ustart[j + 1] : T;
    const uint64_t key = (uint64_t)keys[s];
    const K t = (K)(((key & mask) << b) | (key >> b));
    const WOut w = (WOut)(P ? (P[e - 1] - (s > 0 ? P[s - 1] : 0)) : (e - s));
    tkeep[j] = t;
    tsort[j] = t;
    wkeep[j] = w;
    wsort[j] = w;
  }
}

// start[r] = first i with ((keys[i] >> shift) & mask) >= r, for r in
// [0, n2]; the field is non-decreasing over the U keys.
template <class K>
__global__ void k_cp_bounds(const K *__restrict__ keys, int64_t U, int shift, int b, int64_t n2,
                            int64_t *__restrict__ start) {
  const uint64_t mask = (1ull << b) - 1;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n2; r += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = U;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)(((uint64_t)keys[mid] >> shift) & mask) < r) lo = mid + 1;
      else hi = mid;
    }
    start[r] = lo;
  }
}

// off[r] = upper pairs of rows < r plus lower entries of rows < r.
__global__ void k_cp_offsets(const int64_t *__restrict__ urow, const int64_t *__restrict__ lrow, int64_t n2,
                             int64_t *__restrict__ off) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n2; r += (int64_t)gridDim.x * blockDim.x)
    off[r] = urow[r] + lrow[r];
}

// Places the coarse arcs.  Upper pair j (key Y << b | X, in (X, Y) order)
// goes to row X after the row's lower part: off[X] + (lrow[X + 1] - lrow[X])
// + (j - urow[X]) = j + lrow[X + 1].  Lower entry t of the (Y, X)-sorted
// copy goes to row Y at off[Y] + (t - lrow[Y]) = t + urow[Y].
template <class K, class WOut, bool UPPER>
__global__ void k_cp_place(const K *__restrict__ tk, const WOut *__restrict__ tw, int64_t U, int b,
                           const int64_t *__restrict__ other, int32_t *__restrict__ col, WOut *__restrict__ wt) {
  const uint64_t mask = (1ull << b) - 1;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < U; j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = (uint64_t)tk[j];
    const int64_t hi = (int64_t)(key >> b), lo = (int64_t)(key & mask);
    const int64_t at = UPPER ? j + other[lo + 1] : j + other[hi];
    col[at] = (int32_t)(UPPER ? hi : lo);
    wt[at] = tw[j];
  }
}

// out[0] = largest row length (atomicMax), out[1] = smallest (atomicMin).
__global__ void k_deg_range(const int64_t *__restrict__ off, int64_t n, unsigned long long *__restrict__ out) {
  unsigned long long m = 0, lo = ~0ull;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    unsigned long long d = (unsigned long long)(off[v + 1] - off[v]);
    m = d > m ? d : m;
    lo = d < lo ? d : lo;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long y = __shfl_xor(m, o, WAVE);
    m = y > m ? y : m;
    y = __shfl_xor(lo, o, WAVE);
    lo = y < lo ? y : lo;
  }
  if (lane_id() == 0) {
    if (m) atomicMax(&out[0], m);
    atomicMin(&out[1], lo);
  }
}

int64_t max_degree(Ctx &c, const int64_t *off, int64_t n, int64_t *min_out) {
  if (n <= 0) {
    if (min_out) *min_out = 0;
    return 0;
  }
  unsigned long long *d = c.buf<unsigned long long>("maxdeg", 2);
  const unsigned long long init[2] = {0ull, ~0ull};
  h2d(c, d, init, sizeof(init));
  hipLaunchKernelGGL(k_deg_range, dim3(grid_for(n)), dim3(256), 0, c.stream, off, n, d);
  LAUNCHCHECK();
  unsigned long long h[2] = {0, 0};
  d2h(c, h, d, sizeof(h));
  if (min_out) *min_out = (int64_t)h[1];
  return (int64_t)h[0];
}

namespace {

int lanes_for(const lcc_graph &g) {
  const double avg = g.n > 0 ? (double)g.arcs / (double)g.n : 0.0;
  if (avg <= 8) return 8;
  if (avg <= 16) return 16;
  if (avg <= 32) return 32;
  return 64;
}

// One round at a time: the pass is bound by its map gathers, and narrower
// lane groups with more rounds in flight measured slower.
template <int G, int WK>
void launch_count(Ctx &c, const lcc_graph &g, const int32_t *map, int64_t *inter, int64_t *intra, int32_t *mu) {
  hipLaunchKernelGGL((k_cp_count<G, 1, WK>), dim3((unsigned)cdiv(g.n, CP_NT / G)), dim3(CP_NT), 0, c.stream, g.off,
                     g.col, g.wt, map, g.n, inter, intra, mu);
  LAUNCHCHECK();
}

// The emit covers the count pass's G arcs per vertex and round with at most
// 16 lanes and G / 16 rounds loaded together.
template <int GC, int WK>
void launch_emit(Ctx &c, const lcc_graph &g, const int32_t *map, const int32_t *mu, const int64_t *eoff, int b,
                 uint64_t *keys, int64_t *vals, bool narrow) {
  constexpr int G = GC > 16 ? 16 : GC, U = GC / G;
  const dim3 gr((unsigned)cdiv(g.n, CP_NT / G));
  if (narrow) {
    uint32_t *k32 = reinterpret_cast<uint32_t *>(keys);
    int32_t *v32 = reinterpret_cast<int32_t *>(vals);
    if (WK == LCC_WT_UNIT)
      hipLaunchKernelGGL((k_cp_emit<G, U, WK, false, uint32_t, int32_t>), gr, dim3(CP_NT), 0, c.stream, g.off, mu, g.wt,
                         map, g.n, eoff, b, k32, v32);
    else if (WK != LCC_WT_I64)
      hipLaunchKernelGGL((k_cp_emit<G, U, WK, true, uint32_t, int32_t>), gr, dim3(CP_NT), 0, c.stream, g.off, mu, g.wt,
                         map, g.n, eoff, b, k32, v32);
    else
      fail(LCC_ERR_DEVICE, "internal: 64-bit weights take 64-bit sort values");
  } else if (WK == LCC_WT_UNIT) {
    hipLaunchKernelGGL((k_cp_emit<G, U, WK, false, uint64_t, int64_t>), gr, dim3(CP_NT), 0, c.stream, g.off, mu, g.wt,
                       map, g.n, eoff, b, keys, vals);
  } else {
    hipLaunchKernelGGL((k_cp_emit<G, U, WK, true, uint64_t, int64_t>), gr, dim3(CP_NT), 0, c.stream, g.off, mu, g.wt,
                       map, g.n, eoff, b, keys, vals);
  }
  LAUNCHCHECK();
}

template <int WK>
void count_and_emit(Ctx &c, const lcc_graph &g, const int32_t *map, int32_t *mu, int64_t *inter, int64_t *intra,
                    const int64_t *eoff, int b, uint64_t *keys, int64_t *vals, bool emit, bool narrow) {
  switch (lanes_for(g)) {
    case 8: emit ? launch_emit<8, WK>(c, g, map, mu, eoff, b, keys, vals, narrow) : launch_count<8, WK>(c, g, map, inter, intra, mu); break;
    case 16: emit ? launch_emit<16, WK>(c, g, map, mu, eoff, b, keys, vals, narrow) : launch_count<16, WK>(c, g, map, inter, intra, mu); break;
    case 32: emit ? launch_emit<32, WK>(c, g, map, mu, eoff, b, keys, vals, narrow) : launch_count<32, WK>(c, g, map, inter, intra, mu); break;
    default: emit ? launch_emit<64, WK>(c, g, map, mu, eoff, b, keys, vals, narrow) : launch_count<64, WK>(c, g, map, inter, intra, mu); break;
  }
}

void dispatch_ce(Ctx &c, const lcc_graph &g, const int32_t *map, int32_t *mu, int64_t *inter, int64_t *intra,
                 const int64_t *eoff, int b, uint64_t *keys, int64_t *vals, bool emit, bool narrow = false) {
  switch (g.wt_kind) {
    case LCC_WT_UNIT: count_and_emit<LCC_WT_UNIT>(c, g, map, mu, inter, intra, eoff, b, keys, vals, emit, narrow); break;
    case LCC_WT_I16: count_and_emit<LCC_WT_I16>(c, g, map, mu, inter, intra, eoff, b, keys, vals, emit, narrow); break;
    case LCC_WT_I32: count_and_emit<LCC_WT_I32>(c, g, map, mu, inter, intra, eoff, b, keys, vals, emit, narrow); break;
    default: count_and_emit<LCC_WT_I64>(c, g, map, mu, inter, intra, eoff, b, keys, vals, emit, narrow); break;
  }
}

}  // namespace

// ---------------------------------------------- dense compress, small graphs

// A graph of at most DN_MAX vertices (one clustering, no batch) contracts
// through an n' x n' matrix: arc counts F (an entry with F > 0 is a coarse
// arc, also when its weights sum to zero) and weight sums W (absent for unit
// weights, where the count is the weight).  Rows come out in column order, as
// the sorting path gives them.  Six launches and one read-back replace the
// relabel scan, the key sort and the run sums, which cost far more than the
// work on the coarse levels of a hierarchy.  info: n', coarse arcs, largest
// coarse degree.
constexpr int64_t DN_MAX = 2048;
constexpr int DN_NT = 1024;

// One block: present ids and their ranks (in LDS), n', map, and the
// per-cluster sums of k, kk (k^2 when absent) and 2s (halved with the intra
// weight later), each cleared first (n' + 1 entries: the sorting path's
// extra slot stays zero).
__global__ __launch_bounds__(DN_NT) void k_dn_relabel(const int32_t *__restrict__ C, int64_t n,
                                                      const int64_t *__restrict__ k, const int64_t *__restrict__ kk,
                                                      const int64_t *__restrict__ s, int32_t *__restrict__ map,
                                                      int64_t *__restrict__ ok, int64_t *__restrict__ okk,
                                                      int64_t *__restrict__ os2, int64_t *__restrict__ info) {
  __shared__ int32_t pres[DN_MAX];
  __shared__ int32_t rank[DN_MAX];
  for (int64_t i = threadIdx.x; i < n; i += DN_NT) pres[i] = 0;
  __syncthreads();
  for (int64_t v = threadIdx.x; v < n; v += DN_NT) pres[C[v]] = 1;
  __syncthreads();
  int32_t carry = 0;
  for (int64_t x0 = 0; x0 < n; x0 += DN_NT) {
    const int64_t x = x0 + threadIdx.x;
    int32_t tot;
    const int32_t r = carry + block_excl_scan<int32_t, DN_NT>(x < n ? pres[x] : 0, &tot);
    if (x < n) rank[x] = r;
    carry += tot;
  }
  const int64_t n2 = carry;
  for (int64_t x = threadIdx.x; x <= n2; x += DN_NT) {
    ok[x] = 0;
    okk[x] = 0;
    os2[x] = 0;
  }
  __syncthreads();
  for (int64_t v = threadIdx.x; v < n; v += DN_NT) {
    const int32_t m = rank[C[v]];
    map[v] = m;
    const int64_t kv = k[v];
    atomic_add_i64(&ok[m], kv);
    atomic_add_i64(&okk[m], kk ? kk[v] : kv * kv);
    if (s && s[v]) atomic_add_i64(&os2[m], 2 * s[v]);
  }
  if (threadIdx.x == 0) info[0] = n2;
}

__global__ void k_dn_clear(uint32_t *__restrict__ F, int64_t *__restrict__ W, const int64_t *__restrict__ info) {
  const int64_t n2 = info[0], total = n2 * n2;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    F[i] = 0;
    if (W) W[i] = 0;
  }
}

// G lanes per vertex: inter arcs counted (and weighed) into row map[v] of the
// matrix, intra weight added to the cluster's 2s'.
template <int G, int WK>
__global__ __launch_bounds__(CP_NT) void k_dn_scatter(const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                      const void *__restrict__ wt, const int32_t *__restrict__ map,
                                                      int64_t n, const int64_t *__restrict__ info,
                                                      uint32_t *__restrict__ F, int64_t *__restrict__ W,
                                                      int64_t *__restrict__ os2) {
  const int gl = threadIdx.x % G;
  const int64_t v = (int64_t)blockIdx.x * (CP_NT / G) + threadIdx.x / G;
  const int64_t n2 = info[0];
  int64_t wi = 0;
  int32_t mv = 0;
  if (v < n) {
    mv = map[v];
    for (int64_t e = off[v] + gl; e < off[v + 1]; e += G) {
      const int32_t mu = map[col[e]];
      const int64_t w = load_w<WK>(wt, e);
      if (mu != mv) {
        const int64_t idx = (int64_t)mv * n2 + mu;
        atomicAdd(&F[idx], 1u);
        if constexpr (WK != LCC_WT_UNIT) atomic_add_i64(&W[idx], w);
      } else {
        wi += w;
      }
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) wi += __shfl_xor(wi, o, WAVE);
  if (v < n && gl == 0 && wi) atomic_add_i64(&os2[mv], wi);
}

// One block per coarse row: its number of coarse arcs.
__global__ __launch_bounds__(CP_NT) void k_dn_rowcount(const uint32_t *__restrict__ F, const int64_t *__restrict__ info,
                                                       int64_t *__restrict__ rowcnt) {
  const int64_t n2 = info[0], r = blockIdx.x;
  if (r >= n2) return;
  int64_t c = 0;
  for (int64_t j = threadIdx.x; j < n2; j += CP_NT) c += F[r * n2 + j] != 0;
  int64_t tot;
  block_excl_scan<int64_t, CP_NT>(c, &tot);
  if (threadIdx.x == 0) rowcnt[r] = tot;
}

// One block: row offsets (off[n'] = coarse arcs), the largest row, and s' =
// (sum of 2s + intra weight) / 2.
__global__ __launch_bounds__(DN_NT) void k_dn_finish(const int64_t *__restrict__ rowcnt, int64_t *__restrict__ off,
                                                     int64_t *__restrict__ os2, int64_t *__restrict__ info) {
  const int64_t n2 = info[0];
  int64_t carry = 0, mx = 0;
  for (int64_t r0 = 0; r0 < n2; r0 += DN_NT) {
    const int64_t r = r0 + threadIdx.x;
    const int64_t c = r < n2 ? rowcnt[r] : 0;
    mx = c > mx ? c : mx;
    int64_t tot;
    const int64_t pre = carry + block_excl_scan<int64_t, DN_NT>(c, &tot);
    if (r < n2) off[r] = pre;
    carry += tot;
  }
  for (int64_t x = threadIdx.x; x < n2; x += DN_NT) os2[x] /= 2;
  __shared__ int64_t red[DN_NT / WAVE];
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const int64_t y = __shfl_xor(mx, o, WAVE);
    mx = y > mx ? y : mx;
  }
  if (lane_id() == 0) red[threadIdx.x / WAVE] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < DN_NT / WAVE; i++) mx = red[i] > mx ? red[i] : mx;
    off[n2] = carry;
    info[1] = carry;
    info[2] = mx;
  }
}

// One block per coarse row: its arcs in column order.
template <class WOut>
__global__ __launch_bounds__(CP_NT) void k_dn_emit(const uint32_t *__restrict__ F, const int64_t *__restrict__ W,
                                                   const int64_t *__restrict__ info, const int64_t *__restrict__ off,
                                                   int32_t *__restrict__ ocol, WOut *__restrict__ owt) {
  const int64_t n2 = info[0], r = blockIdx.x;
  if (r >= n2) return;
  int64_t pos = off[r];
  for (int64_t j0 = 0; j0 < n2; j0 += CP_NT) {
    const int64_t j = j0 + threadIdx.x;
    const uint32_t f = j < n2 ? F[r * n2 + j] : 0;
    int64_t tot;
    const int64_t at = pos + block_excl_scan<int64_t, CP_NT>(f != 0, &tot);
    if (f) {
      ocol[at] = (int32_t)j;
      owt[at] = (WOut)(W ? W[r * n2 + j] : (int64_t)f);
    }
    pos += tot;
  }
}

namespace {

template <int G>
void launch_dn_scatter(Ctx &c, const lcc_graph &g, const int32_t *map, const int64_t *info, uint32_t *F, int64_t *W,
                       int64_t *os2) {
  const dim3 gr((unsigned)cdiv(g.n, CP_NT / G));
  switch (g.wt_kind) {
    case LCC_WT_UNIT:
      hipLaunchKernelGGL((k_dn_scatter<G, LCC_WT_UNIT>), gr, dim3(CP_NT), 0, c.stream, g.off, g.col, g.wt, map, g.n,
                         info, F, W, os2);
      break;
    case LCC_WT_I16:
      hipLaunchKernelGGL((k_dn_scatter<G, LCC_WT_I16>), gr, dim3(CP_NT), 0, c.stream, g.off, g.col, g.wt, map, g.n,
                         info, F, W, os2);
      break;
    case LCC_WT_I32:
      hipLaunchKernelGGL((k_dn_scatter<G, LCC_WT_I32>), gr, dim3(CP_NT), 0, c.stream, g.off, g.col, g.wt, map, g.n,
                         info, F, W, os2);
      break;
    default:
      hipLaunchKernelGGL((k_dn_scatter<G, LCC_WT_I64>), gr, dim3(CP_NT), 0, c.stream, g.off, g.col, g.wt, map, g.n,
                         info, F, W, os2);
      break;
  }
  LAUNCHCHECK();
}

void compress_dense(Ctx &c, const lcc_graph &g, const int32_t *C, OwnedGraph &out, int32_t *map, bool wide,
                    int64_t *maxdeg_out) {
  const int64_t n = g.n;
  const size_t nn = (size_t)n;
  const bool weighted = g.wt_kind != LCC_WT_UNIT;
  Ctx::Timer tm(&c, "cp_dense", 40.0 * (double)n + (8.0 + wt_bytes(g.wt_kind)) * (double)g.arcs, (double)g.arcs);
  // capacities from host-known bounds: n' <= n, coarse arcs <= min(arcs, n^2)
  const int64_t ub = std::max<int64_t>(1, std::min<int64_t>(g.arcs, n * n));
  c.ensure(out.off, (nn + 1) * sizeof(int64_t));
  c.ensure(out.col, (size_t)ub * sizeof(int32_t));
  c.ensure(out.wt, (size_t)ub * (wide ? 8 : 4));
  c.ensure(out.k, (nn + 1) * sizeof(int64_t));
  c.ensure(out.s, (nn + 1) * sizeof(int64_t));
  c.ensure(out.kk, (nn + 1) * sizeof(int64_t));
  int64_t *info = c.buf<int64_t>("dn.info", 4);
  uint32_t *F = c.buf<uint32_t>("dn.F", nn * nn);
  int64_t *W = weighted ? c.buf<int64_t>("dn.W", nn * nn) : nullptr;
  int64_t *rowcnt = c.buf<int64_t>("dn.rowcnt", nn);
  int64_t *os2 = out.s.as<int64_t>();
  hipLaunchKernelGGL(k_dn_relabel, dim3(1), dim3(DN_NT), 0, c.stream, C, n, g.k, g.kk, g.s, map, out.k.as<int64_t>(),
                     out.kk.as<int64_t>(), os2, info);
  LAUNCHCHECK();
  hipLaunchKernelGGL(k_dn_clear, dim3(grid_for(n * n)), dim3(256), 0, c.stream, F, W, (const int64_t *)info);
  LAUNCHCHECK();
  switch (lanes_for(g)) {
    case 8: launch_dn_scatter<8>(c, g, map, info, F, W, os2); break;
    case 16: launch_dn_scatter<16>(c, g, map, info, F, W, os2); break;
    case 32: launch_dn_scatter<32>(c, g, map, info, F, W, os2); break;
    default: launch_dn_scatter<64>(c, g, map, info, F, W, os2); break;
  }
  hipLaunchKernelGGL(k_dn_rowcount, dim3((unsigned)n), dim3(CP_NT), 0, c.stream, (const uint32_t *)F,
                     (const int64_t *)info, rowcnt);
  LAUNCHCHECK();
  hipLaunchKernelGGL(k_dn_finish, dim3(1), dim3(DN_NT), 0, c.stream, (const int64_t *)rowcnt, out.off.as<int64_t>(),
                     os2, info);
  LAUNCHCHECK();
  if (wide)
    hipLaunchKernelGGL((k_dn_emit<int64_t>), dim3((unsigned)n), dim3(CP_NT), 0, c.stream, (const uint32_t *)F,
                       (const int64_t *)W, (const int64_t *)info, (const int64_t *)out.off.as<int64_t>(),
                       out.col.as<int32_t>(), out.wt.as<int64_t>());
  else
    hipLaunchKernelGGL((k_dn_emit<int32_t>), dim3((unsigned)n), dim3(CP_NT), 0, c.stream, (const uint32_t *)F,
                       (const int64_t *)W, (const int64_t *)info, (const int64_t *)out.off.as<int64_t>(),
                       out.col.as<int32_t>(), out.wt.as<int32_t>());
  LAUNCHCHECK();
  int64_t h[3] = {0, 0, 0};
  d2h(c, h, info, sizeof(h));
  out.n = h[0];
  out.arcs = h[1];
  if (maxdeg_out) *maxdeg_out = h[2];
}

// From the U unique upper pairs (sorted keys ks, runs at ustart, run sums
// from the prefix P or run lengths) to the coarse CSR: both halves of every
// row, row offsets included.
template <class K, class WOut>
void mirror_pairs(Ctx &c, const K *ks, const int64_t *ustart, int64_t U, int64_t T, const int64_t *P, int b,
                  int64_t n2, OwnedGraph &out) {
  int64_t *urow = c.buf<int64_t>("cp.urow", (size_t)(n2 + 1));
  int64_t *lrow = c.buf<int64_t>("cp.lrow", (size_t)(n2 + 1));
  int64_t *off = out.off.as<int64_t>();
  Ctx::Timer tm(&c, "cp_mirror",
                (double)U * (3.0 * (sizeof(K) + sizeof(WOut)) + 2.0 * (sizeof(K) + sizeof(WOut)) * cdiv(b, RS_BITS) +
                             2.0 * (sizeof(K) + sizeof(WOut)) + 2.0 * (4.0 + sizeof(WOut))),
                (double)U);
  const size_t u = (size_t)(U > 0 ? U : 1);
  K *tkk = c.buf<K>("cp.tkk", u), *tk0 = c.buf<K>("cp.tk0", u), *tk1 = c.buf<K>("cp.tk1", u);
  WOut *twk = c.buf<WOut>("cp.twk", u), *tw0 = c.buf<WOut>("cp.tw0", u), *tw1 = c.buf<WOut>("cp.tw1", u);
  bool flip = false;
  if (U > 0) {
    hipLaunchKernelGGL((k_cp_pairs<K, WOut>), dim3(grid_for(U)), dim3(256), 0, c.stream, ks, ustart, U, T, P, b,
                       tkk, tk0, twk, tw0);
    LAUNCHCHECK();
    // stable on the high b bits (Y): the (X, Y) order becomes (Y, X)
    flip = radix_sort<K, WOut, true>(c, tk0, tw0, tk1, tw1, U, 2 * b, "cp.ms", b);
  }
  const K *tl = flip ? tk1 : tk0;
  const WOut *wl = flip ? tw1 : tw0;
  hipLaunchKernelGGL((k_cp_bounds<K>), dim3(grid_for(n2 + 1)), dim3(256), 0, c.stream, tkk, U, 0, b, n2, urow);
  LAUNCHCHECK();
  hipLaunchKernelGGL((k_cp_bounds<K>), dim3(grid_for(n2 + 1)), dim3(256), 0, c.stream, tl, U, b, b, n2, lrow);
  LAUNCHCHECK();
  hipLaunchKernelGGL(k_cp_offsets, dim3(grid_for(n2 + 1)), dim3(256), 0, c.stream, urow, lrow, n2, off);
  LAUNCHCHECK();
  if (U <= 0) return;
  int32_t *col = out.col.as<int32_t>();
  WOut *wt = out.wt.as<WOut>();
  hipLaunchKernelGGL((k_cp_place<K, WOut, true>), dim3(grid_for(U)), dim3(256), 0, c.stream, tkk, twk, U, b, lrow,
                     col, wt);
  LAUNCHCHECK();
  hipLaunchKernelGGL((k_cp_place<K, WOut, false>), dim3(grid_for(U)), dim3(256), 0, c.stream, tl, wl, U, b, urow,
                     col, wt);
  LAUNCHCHECK();
}

}  // namespace

void compress_graph(Ctx &c, const lcc_graph &g, const int32_t *C, OwnedGraph &out, int32_t *map, bool wide,
                    int64_t *maxdeg_out, const CompressJobs *cj, int64_t *mindeg_out) {
  if (mindeg_out) *mindeg_out = 0;  // unknown: rows of every length may be present
  const int32_t *jid = cj ? cj->jid : nullptr;
  const uint8_t *jcont = cj ? cj->jcont : nullptr;
  const int64_t n = g.n;
  out.n = 0;
  out.arcs = 0;
  out.wt_kind = wide ? LCC_WT_I64 : LCC_WT_I32;
  if (n <= 0) {
    c.ensure(out.off, sizeof(int64_t));
    HIPCHECK(hipMemsetAsync(out.off.p, 0, sizeof(int64_t), c.stream));
    if (maxdeg_out) *maxdeg_out = 0;
    return;
  }
  if (!cj && n <= DN_MAX) {
    compress_dense(c, g, C, out, map, wide, maxdeg_out);
    return;
  }
  const size_t nn = (size_t)n;
  uint8_t *present = c.buf<uint8_t>("cp.present", nn);
  int32_t *rank = c.buf<int32_t>("cp.rank", nn);
  int64_t *inter = c.buf<int64_t>("cp.inter", nn + 1);
  int64_t *intra = c.buf<int64_t>("cp.intra", nn);
  int64_t *tots = c.buf<int64_t>("cp.tots", 4);
  int32_t *mu = c.buf<int32_t>("cp.mu", (size_t)(g.arcs > 0 ? g.arcs : 1));  // map[col[e]] per arc
  HIPCHECK(hipMemsetAsync(tots, 0, 4 * sizeof(int64_t), c.stream));
  {
    Ctx::Timer tm(&c, "cp_relabel", 13.0 * (double)n, (double)n);
    HIPCHECK(hipMemsetAsync(present, 0, nn, c.stream));
    hipLaunchKernelGGL(k_mark_present, dim3(grid_for(n)), dim3(256), 0, c.stream, C, n, jid, jcont, present);
    LAUNCHCHECK();
    scan<uint8_t, int32_t>(c, present, rank, n, false, reinterpret_cast<int32_t *>(tots));
    hipLaunchKernelGGL(k_map, dim3(grid_for(n)), dim3(256), 0, c.stream, C, rank, n, jid, jcont, map);
    LAUNCHCHECK();
  }
  const int wb = wt_bytes(g.wt_kind);
  {
    Ctx::Timer tm(&c, "cp_count", 28.0 * (double)n + (12.0 + wb) * (double)g.arcs, (double)g.arcs);
    dispatch_ce(c, g, map, mu, inter, intra, nullptr, 0, nullptr, nullptr, false);
  }
  scan<int64_t, int64_t>(c, inter, inter, n, false, tots + 1);
  int64_t h[2] = {0, 0};
  d2h(c, h, tots, 2 * sizeof(int64_t));
  const int64_t n2 = (int64_t)(int32_t)(h[0] & 0xffffffff);
  const int64_t T = h[1];
  out.n = n2;
  const int b = bits_for(n2 > 1 ? n2 - 1 : 1);
  const bool weighted = g.wt_kind != LCC_WT_UNIT;
  // 32-bit keys and weights when both fit: half the sort's bytes
  const bool narrow = 2 * b <= 32 && g.wt_kind != LCC_WT_I64;
  const double kb = narrow ? 4.0 : 8.0, vb = weighted ? kb : 0.0;
  uint64_t *k0 = c.buf<uint64_t>("cp.k0", (size_t)(T > 0 ? T : 1));
  uint64_t *k1 = c.buf<uint64_t>("cp.k1", (size_t)(T > 0 ? T : 1));
  int64_t *v0 = weighted ? c.buf<int64_t>("cp.v0", (size_t)(T > 0 ? T : 1)) : nullptr;
  int64_t *v1 = weighted ? c.buf<int64_t>("cp.v1", (size_t)(T > 0 ? T : 1)) : nullptr;
  if (T > 0) {
    Ctx::Timer tm(&c, "cp_emit", 28.0 * (double)n + (4.0 + wb) * (double)g.arcs + (kb + vb) * (double)T,
                  (double)g.arcs);
    dispatch_ce(c, g, map, mu, inter, intra, inter, b, k0, v0, true, narrow);
  }
  uint64_t *ks = k0;
  int64_t *vs = v0, *vfree = v1;  // vfree: the value buffer the sorted data left
  if (T > 1) {
    Ctx::Timer tm(&c, "cp_sort", 2.0 * (kb + vb) * (double)T * (double)cdiv(2 * b, RS_BITS), (double)T);
    bool flip;
    if (narrow) {
      uint32_t *a0 = reinterpret_cast<uint32_t *>(k0), *a1 = reinterpret_cast<uint32_t *>(k1);
      int32_t *w0 = reinterpret_cast<int32_t *>(v0), *w1 = reinterpret_cast<int32_t *>(v1);
      flip = weighted ? radix_sort<uint32_t, int32_t, true>(c, a0, w0, a1, w1, T, 2 * b, "cp.rs")
                      : radix_sort<uint32_t, int32_t, false>(c, a0, nullptr, a1, nullptr, T, 2 * b, "cp.rs");
    } else {
      flip = weighted ? radix_sort<uint64_t, int64_t, true>(c, k0, v0, k1, v1, T, 2 * b, "cp.rs")
                      : radix_sort<uint64_t, int64_t, false>(c, k0, nullptr, k1, nullptr, T, 2 * b, "cp.rs");
    }
    if (flip) {
      ks = k1;
      vs = v1;
      vfree = v0;
    }
  }
  // unique upper pairs
  int64_t U = 0;
  uint8_t *head = c.buf<uint8_t>("cp.head", (size_t)(T > 0 ? T : 1));
  int64_t *uidx = c.buf<int64_t>("cp.uidx", (size_t)(T > 0 ? T : 1));
  if (T > 0) {
    Ctx::Timer tm(&c, "cp_reduce", (double)T * (8.0 + 1.0 + 8.0), (double)T);
    if (narrow)
      hipLaunchKernelGGL(k_cp_heads<uint32_t>, dim3(grid_for(T)), dim3(256), 0, c.stream,
                         (const uint32_t *)reinterpret_cast<uint32_t *>(ks), T, head);
    else
      hipLaunchKernelGGL(k_cp_heads<uint64_t>, dim3(grid_for(T)), dim3(256), 0, c.stream, (const uint64_t *)ks, T,
                         head);
    LAUNCHCHECK();
    scan<uint8_t, int64_t>(c, head, uidx, T, false, tots + 2);
    d2h(c, &U, tots + 2, sizeof(int64_t));
  }
  out.arcs = 2 * U;
  c.ensure(out.off, (size_t)(n2 + 1) * sizeof(int64_t));
  c.ensure(out.col, (size_t)(U > 0 ? 2 * U : 1) * sizeof(int32_t));
  c.ensure(out.wt, (size_t)(U > 0 ? 2 * U : 1) * (wide ? 8 : 4));
  // one extra slot: the per-cluster sums park dropped vertices at key n2
  c.ensure(out.k, (size_t)(n2 + 1) * sizeof(int64_t));
  c.ensure(out.s, (size_t)(n2 + 1) * sizeof(int64_t));
  c.ensure(out.kk, (size_t)(n2 + 1) * sizeof(int64_t));
  const int64_t *P = nullptr;
  int64_t *ustart = c.buf<int64_t>("cp.ustart", (size_t)(U > 0 ? U : 1));
  if (U > 0) {
    Ctx::Timer tm(&c, "cp_unique", (double)U * 8.0 + (double)T * (weighted ? (narrow ? 12.0 : 16.0) : 0.0),
                  (double)U);
    hipLaunchKernelGGL(k_cp_ustart, dim3(grid_for(T)), dim3(256), 0, c.stream, head, uidx, T, ustart);
    LAUNCHCHECK();
    if (weighted && narrow) {  // run sums from a 64-bit prefix of the 32-bit weights
      scan<int32_t, int64_t>(c, reinterpret_cast<const int32_t *>(vs), vfree, T, true, (int64_t *)nullptr);
      P = vfree;
    } else if (weighted) {
      scan<int64_t, int64_t>(c, vs, vs, T, true, (int64_t *)nullptr);
      P = vs;
    }
  }
  if (narrow && wide)
    mirror_pairs<uint32_t, int64_t>(c, reinterpret_cast<const uint32_t *>(ks), ustart, U, T, P, b, n2, out);
  else if (narrow)
    mirror_pairs<uint32_t, int32_t>(c, reinterpret_cast<const uint32_t *>(ks), ustart, U, T, P, b, n2, out);
  else if (wide)
    mirror_pairs<uint64_t, int64_t>(c, ks, ustart, U, T, P, b, n2, out);
  else
    mirror_pairs<uint64_t, int32_t>(c, ks, ustart, U, T, P, b, n2, out);
  // per-cluster k', kk', s'
  {
    Ctx::Timer tm(&c, "cp_totals", 0.0, (double)n);
    const int32_t *keys = map;
    int64_t nkeys = n2;
    if (jid) {
      int32_t *kb = c.buf<int32_t>("cpv.keys", nn);
      hipLaunchKernelGGL(k_keys_with_sentinel, dim3(grid_for(n)), dim3(256), 0, c.stream, map, n, (int32_t)n2, kb);
      LAUNCHCHECK();
      keys = kb;
      nkeys = n2 + 1;
    }
    ByKey bk = sort_by_key(c, keys, n, nkeys, "cpv");
    int64_t *start = c.buf<int64_t>("cpv.start", (size_t)(nkeys > 0 ? nkeys : 1));
    hipLaunchKernelGGL(k_seg_heads, dim3(grid_for(n)), dim3(256), 0, c.stream, bk.key, n, start);
    LAUNCHCHECK();
    seg_sum(c, bk, n, nkeys, start, G_K, g, nullptr, out.k.as<int64_t>(), nullptr, false);
    seg_sum(c, bk, n, nkeys, start, G_KK, g, nullptr, out.kk.as<int64_t>(), nullptr, false);
    seg_sum(c, bk, n, nkeys, start, G_SELF2, g, intra, out.s.as<int64_t>(), nullptr, true);
  }
  if (jid) {
    hipLaunchKernelGGL(k_next_jid, dim3(grid_for(n)), dim3(256), 0, c.stream, map, jid, n, cj->jid_next);
    LAUNCHCHECK();
    hipLaunchKernelGGL(k_next_jbase, dim3(grid_for(cj->jobs + 1)), dim3(256), 0, c.stream, cj->jid_next, n2,
                       cj->jobs, cj->jbase_next);
    LAUNCHCHECK();
  }
  if (maxdeg_out) *maxdeg_out = max_degree(c, out.off.as<int64_t>(), n2, mindeg_out);
}

}  // namespace lcc
