// bestmove.hip -- Best-Moves (paper Algorithm 1, top) on gfx950.
//
// One iteration = S synchronous sub-rounds.  For each iteration the active
// vertices are partitioned into (sub-round, degree bin) buckets; every
// sub-round then runs one aggregation kernel per non-empty degree bin and one
// apply kernel:
//
//   aggregate  a group of G lanes per vertex streams the vertex's CSR row
//              (coalesced col / weight reads), gathers C[u], and sums the
//              weight per neighbor cluster in an LDS open-addressing hash
//              (a global-memory hash for vertices above 2047 neighbors).  It
//              then scores every distinct cluster against the snapshot
//              (int64: q*w - p*k_v*K_X), reduces (score desc, id asc) across
//              the group, decides, writes D[v], and for a mover marks its
//              neighbors in the next frontier.
//   apply      movers update C and the cluster totals K / sizes with int64 /
//              int32 atomics (integer adds commute, so the result does not
//              depend on their order); isolating vertices are collected and
//              handed the ascending empty ids by a guarded scan-and-pair pass.
//
// Nothing in a sub-round reads what the same sub-round writes: aggregation
// reads C, K, cnt and writes only D / flags / counters; apply runs after it.
#include "ops.hpp"
#include "prims.hpp"

namespace lcc {

constexpr int BM_NT = 256;
constexpr int NBINS = 7;
constexpr int32_t ISO_ID = INT32_MAX;  // ranks after every real cluster id

// Largest degree each bin accepts; bins 0-5 hash in LDS with >= 2(deg+1) slots.
__host__ __device__ constexpr int64_t bin_limit(int b) {
  return b == 0 ? 7 : b == 1 ? 15 : b == 2 ? 31 : b == 3 ? 63 : b == 4 ? 255 : b == 5 ? 2047 : INT64_MAX;
}
__host__ __device__ inline int bin_of(int64_t deg) {
  int b = 0;
  while (b < NBINS - 1 && deg > bin_limit(b)) b++;
  return b;
}

__device__ __forceinline__ int64_t cdiv_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct AggArgs {
  const int64_t *off;
  const int32_t *col;
  const void *wt;
  const int64_t *k;
  const int32_t *C;
  const int64_t *K;
  const int32_t *cnt;
  int64_t p, q;
  int32_t allow_iso;
  const int32_t *list;
  int64_t count;
  int32_t *D;
  uint8_t *next_flag;  // nullptr: frontier = all vertices, no marking
  int64_t *ctr;        // [0] movers, [1] candidates, [2] arcs of movers, [3] capacity errors
  int32_t *gkeys;      // global hash (bin 6)
  int64_t *gvals;
  int64_t gcap;
};

// (score, id) order: higher score first, then lower id.
__device__ __forceinline__ bool better(int64_t s, int32_t id, int64_t bs, int32_t bid) {
  return s > bs || (s == bs && id < bid);
}

template <int H> __device__ __forceinline__ uint32_t slot_of(int32_t X) {
  constexpr int LOG = __builtin_ctz(H);
  return ((uint32_t)X * 0x9E3779B1u) >> (32 - LOG);
}

// Adds w to key X in an LDS table of H slots (keys -1 = empty).
template <int H, class Acc>
__device__ __forceinline__ void lds_insert(int32_t *keys, Acc *vals, int32_t X, int64_t w) {
  uint32_t h = slot_of<H>(X);
  while (true) {
    int32_t cur = keys[h];
    if (cur == -1) {
      cur = atomicCAS(&keys[h], -1, X);
      if (cur == -1) cur = X;
    }
    if (cur == X) {
      if (w) {
        if constexpr (sizeof(Acc) == 8)
          atomicAdd(reinterpret_cast<unsigned long long *>(&vals[h]), (unsigned long long)w);
        else
          atomicAdd(&vals[h], (Acc)w);
      }
      return;
    }
    h = (h + 1) & (H - 1);
  }
}

// Decision from the reduced group results (identical in every lane).
__device__ __forceinline__ int32_t decide(int64_t best_s, int32_t best_id, int64_t stay, bool iso_ok,
                                          int32_t c) {
  if (iso_ok && (best_s == INT64_MIN || 0 > best_s)) {
    best_s = 0;
    best_id = ISO_ID;
  }
  if (best_s != INT64_MIN && best_s > stay) return best_id == ISO_ID ? -1 : best_id;
  return c;
}

// Block-wide aggregation of the three counters, one atomic each per block.
__device__ __forceinline__ void flush_counters(int64_t *ctr, int64_t movers, int64_t cands, int64_t marcs) {
  __shared__ int64_t red[3][BM_NT / WAVE];
  movers = wave_sum(movers);
  cands = wave_sum(cands);
  marcs = wave_sum(marcs);
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    red[0][w] = movers;
    red[1][w] = cands;
    red[2][w] = marcs;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    int64_t s = 0;
    for (int i = 0; i < BM_NT / WAVE; i++) s += red[threadIdx.x][i];
    if (s) atomic_add_i64(&ctr[threadIdx.x], s);
  }
}

// G lanes per vertex (G <= 64, inside one wavefront), H LDS slots per vertex.
template <int G, int H, int WK>
__global__ __launch_bounds__(BM_NT) void k_bm_aggregate(AggArgs a) {
  using Acc = typename std::conditional<(WK == LCC_WT_UNIT || WK == LCC_WT_I16), int32_t, int64_t>::type;
  constexpr int GPB = BM_NT / G;
  __shared__ int32_t hk[GPB * H];
  __shared__ Acc hv[GPB * H];
  const int t = threadIdx.x, grp = t / G, gl = t % G;
  const int64_t gi = (int64_t)blockIdx.x * GPB + grp;
  const bool valid = gi < a.count;
  int32_t *keys = hk + grp * H;
  Acc *vals = hv + grp * H;
#pragma unroll
  for (int j = gl; j < H; j += G) {
    keys[j] = -1;
    vals[j] = 0;
  }
  __syncthreads();
  int32_t v = 0, c = 0;
  int64_t beg = 0, end = 0;
  if (valid) {
    v = a.list[gi];
    beg = a.off[v];
    end = a.off[v + 1];
    c = a.C[v];
    if (gl == 0) lds_insert<H, Acc>(keys, vals, c, 0);
    for (int64_t e = beg + gl; e < end; e += G) {
      int32_t X = a.C[a.col[e]];
      lds_insert<H, Acc>(keys, vals, X, load_w<WK>(a.wt, e));
    }
  }
  __syncthreads();
  int64_t best_s = INT64_MIN, wc = 0, ncand = 0;
  int32_t best_id = ISO_ID;
  int64_t kv = 0, pk = 0;
  if (valid) {
    kv = a.k[v];
    pk = a.p * kv;
#pragma unroll
    for (int j = gl; j < H; j += G) {
      int32_t X = keys[j];
      if (X < 0) continue;
      ncand++;
      int64_t wx = (int64_t)vals[j];
      if (X == c) {
        wc = wx;
      } else {
        int64_t s = a.q * wx - pk * a.K[X];
        if (better(s, X, best_s, best_id)) {
          best_s = s;
          best_id = X;
        }
      }
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    int64_t os = __shfl_xor(best_s, o, WAVE);
    int32_t oid = __shfl_xor(best_id, o, WAVE);
    if (better(os, oid, best_s, best_id)) {
      best_s = os;
      best_id = oid;
    }
    wc += __shfl_xor(wc, o, WAVE);
  }
  bool moved = false;
  if (valid) {
    int64_t stay = a.q * wc - pk * (a.K[c] - kv);
    bool iso_ok = a.allow_iso && a.cnt[c] >= 2;
    int32_t d = decide(best_s, best_id, stay, iso_ok, c);
    moved = d != c;
    if (gl == 0) a.D[v] = d;
    if (moved && a.next_flag)
      for (int64_t e = beg + gl; e < end; e += G) a.next_flag[a.col[e]] = 1;
  }
  flush_counters(a.ctr, (moved && gl == 0) ? 1 : 0, ncand, (moved && gl == 0) ? end - beg : 0);
}

// Block per vertex, 4096-slot LDS hash (degrees 256..2047).
template <int WK>
__global__ __launch_bounds__(BM_NT) void k_bm_aggregate_block(AggArgs a) {
  using Acc = typename std::conditional<(WK == LCC_WT_UNIT || WK == LCC_WT_I16), int32_t, int64_t>::type;
  constexpr int H = 4096;
  __shared__ int32_t keys[H];
  __shared__ Acc vals[H];
  __shared__ int64_t rs[BM_NT / WAVE];
  __shared__ int32_t rid[BM_NT / WAVE];
  __shared__ int64_t rw[BM_NT / WAVE];
  __shared__ int32_t sh_d;
  const int t = threadIdx.x, w = t / WAVE;
  const int64_t gi = blockIdx.x;
  for (int j = t; j < H; j += BM_NT) {
    keys[j] = -1;
    vals[j] = 0;
  }
  __syncthreads();
  const int32_t v = a.list[gi];
  const int64_t beg = a.off[v], end = a.off[v + 1];
  const int32_t c = a.C[v];
  if (t == 0) lds_insert<H, Acc>(keys, vals, c, 0);
  for (int64_t e = beg + t; e < end; e += BM_NT) lds_insert<H, Acc>(keys, vals, a.C[a.col[e]], load_w<WK>(a.wt, e));
  __syncthreads();
  const int64_t kv = a.k[v], pk = a.p * kv;
  int64_t best_s = INT64_MIN, wc = 0, cands = 0;
  int32_t best_id = ISO_ID;
  for (int j = t; j < H; j += BM_NT) {
    int32_t X = keys[j];
    if (X < 0) continue;
    cands++;
    int64_t wx = (int64_t)vals[j];
    if (X == c) {
      wc = wx;
    } else {
      int64_t s = a.q * wx - pk * a.K[X];
      if (better(s, X, best_s, best_id)) {
        best_s = s;
        best_id = X;
      }
    }
  }
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    int64_t os = __shfl_xor(best_s, o, WAVE);
    int32_t oid = __shfl_xor(best_id, o, WAVE);
    if (better(os, oid, best_s, best_id)) {
      best_s = os;
      best_id = oid;
    }
    wc += __shfl_xor(wc, o, WAVE);
  }
  if (lane_id() == 0) {
    rs[w] = best_s;
    rid[w] = best_id;
    rw[w] = wc;
  }
  __syncthreads();
  int64_t movers = 0, marcs = 0;
  if (t == 0) {
    int64_t bs = rs[0], ww = rw[0];
    int32_t bi = rid[0];
    for (int i = 1; i < BM_NT / WAVE; i++) {
      if (better(rs[i], rid[i], bs, bi)) {
        bs = rs[i];
        bi = rid[i];
      }
      ww += rw[i];
    }
    int64_t stay = a.q * ww - pk * (a.K[c] - kv);
    bool iso_ok = a.allow_iso && a.cnt[c] >= 2;
    int32_t d = decide(bs, bi, stay, iso_ok, c);
    a.D[v] = d;
    sh_d = d;
    if (d != c) {
      movers = 1;
      marcs = end - beg;
    }
  }
  __syncthreads();
  if (sh_d != c && a.next_flag)
    for (int64_t e = beg + t; e < end; e += BM_NT) a.next_flag[a.col[e]] = 1;
  flush_counters(a.ctr, movers, cands, marcs);
}

// Block per vertex (grid-stride), hash table in this block's global region.
template <int WK>
__global__ __launch_bounds__(BM_NT) void k_bm_aggregate_global(AggArgs a) {
  __shared__ int64_t rs[BM_NT / WAVE];
  __shared__ int32_t rid[BM_NT / WAVE];
  __shared__ int64_t rw[BM_NT / WAVE];
  __shared__ int32_t sh_d;
  int32_t *keys = a.gkeys + (int64_t)blockIdx.x * a.gcap;
  int64_t *vals = a.gvals + (int64_t)blockIdx.x * a.gcap;
  const int t = threadIdx.x, w = t / WAVE;
  int64_t movers = 0, cands = 0, marcs = 0;
  for (int64_t gi = blockIdx.x; gi < a.count; gi += gridDim.x) {
    const int32_t v = a.list[gi];
    const int64_t beg = a.off[v], end = a.off[v + 1];
    const int32_t c = a.C[v];
    int64_t cap = 1;
    while (cap < 2 * (end - beg + 1)) cap <<= 1;
    if (cap > a.gcap) {  // the host sized the table from the maximum degree
      if (t == 0) {
        a.D[v] = c;
        atomic_add_i64(&a.ctr[3], 1);
      }
      continue;
    }
    const uint32_t mask = (uint32_t)(cap - 1);
    int lg = 0;
    while ((1ll << lg) < cap) lg++;
    for (int64_t j = t; j < cap; j += BM_NT) {
      keys[j] = -1;
      vals[j] = 0;
    }
    __threadfence();
    __syncthreads();
    auto insert = [&](int32_t X, int64_t wgt) {
      uint32_t h = lg ? (((uint32_t)X * 0x9E3779B1u) >> (32 - lg)) : 0u;
      while (true) {
        int32_t cur = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == -1) {
          cur = atomicCAS(&keys[h], -1, X);
          if (cur == -1) cur = X;
        }
        if (cur == X) {
          if (wgt) atomic_add_i64(&vals[h], wgt);
          return;
        }
        h = (h + 1) & mask;
      }
    };
    if (t == 0) insert(c, 0);
    for (int64_t e = beg + t; e < end; e += BM_NT) insert(a.C[a.col[e]], load_w<WK>(a.wt, e));
    __threadfence();
    __syncthreads();
    const int64_t kv = a.k[v], pk = a.p * kv;
    int64_t best_s = INT64_MIN, wc = 0;
    int32_t best_id = ISO_ID;
    for (int64_t j = t; j < cap; j += BM_NT) {
      int32_t X = __hip_atomic_load(&keys[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (X < 0) continue;
      cands++;
      int64_t wx = __hip_atomic_load(&vals[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (X == c) {
        wc = wx;
      } else {
        int64_t s = a.q * wx - pk * a.K[X];
        if (better(s, X, best_s, best_id)) {
          best_s = s;
          best_id = X;
        }
      }
    }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
      int64_t os = __shfl_xor(best_s, o, WAVE);
      int32_t oid = __shfl_xor(best_id, o, WAVE);
      if (better(os, oid, best_s, best_id)) {
        best_s = os;
        best_id = oid;
      }
      wc += __shfl_xor(wc, o, WAVE);
    }
    if (lane_id() == 0) {
      rs[w] = best_s;
      rid[w] = best_id;
      rw[w] = wc;
    }
    __syncthreads();
    if (t == 0) {
      int64_t bs = rs[0], ww = rw[0];
      int32_t bi = rid[0];
      for (int i = 1; i < BM_NT / WAVE; i++) {
        if (better(rs[i], rid[i], bs, bi)) {
          bs = rs[i];
          bi = rid[i];
        }
        ww += rw[i];
      }
      int64_t stay = a.q * ww - pk * (a.K[c] - kv);
      bool iso_ok = a.allow_iso && a.cnt[c] >= 2;
      int32_t d = decide(bs, bi, stay, iso_ok, c);
      a.D[v] = d;
      sh_d = d;
      if (d != c) {
        movers++;
        marcs += end - beg;
      }
    }
    __syncthreads();
    if (sh_d != c && a.next_flag)
      for (int64_t e = beg + t; e < end; e += BM_NT) a.next_flag[a.col[e]] = 1;
    __syncthreads();
  }
  flush_counters(a.ctr, movers, cands, marcs);
}

// Applies the sub-round's decisions.
__global__ __launch_bounds__(BM_NT) void k_bm_apply(const int32_t *__restrict__ list, int64_t count,
                                                    const int32_t *__restrict__ D, int32_t *__restrict__ C,
                                                    int64_t *__restrict__ K, int32_t *__restrict__ cnt,
                                                    const int64_t *__restrict__ k, uint8_t *__restrict__ iso_flag,
                                                    int64_t *__restrict__ iso_ctr) {
  const int64_t i = (int64_t)blockIdx.x * BM_NT + threadIdx.x;
  int64_t niso = 0;
  if (i < count) {
    const int32_t v = list[i];
    const int32_t d = D[v], c = C[v];
    if (d != c) {
      const int64_t kv = k[v];
      if (kv) atomic_add_i64(&K[c], -kv);
      atomicSub(&cnt[c], 1);
      if (d < 0) {
        C[v] = -1;
        iso_flag[v] = 1;
        niso = 1;
      } else {
        if (kv) atomic_add_i64(&K[d], kv);
        atomicAdd(&cnt[d], 1);
        C[v] = d;
      }
    }
  }
  niso = wave_sum(niso);
  if (lane_id() == 0 && niso) atomic_add_i64(iso_ctr, niso);
}

// --- isolation: the j-th isolated vertex (ascending) gets the j-th empty id.
constexpr int ISO_TILE = CMP_TILE;

__global__ __launch_bounds__(CMP_NT) void k_iso_count(const uint8_t *__restrict__ iso_flag,
                                                      const int32_t *__restrict__ cnt, int64_t n,
                                                      const int64_t *__restrict__ iso_ctr,
                                                      int64_t *__restrict__ part) {
  if (*iso_ctr == 0) return;
  const int64_t base = (int64_t)blockIdx.x * ISO_TILE + (int64_t)threadIdx.x * CMP_IPT;
  int64_t a = 0, b = 0;
#pragma unroll
  for (int i = 0; i < CMP_IPT; i++) {
    int64_t x = base + i;
    if (x < n) {
      a += iso_flag[x] != 0;
      b += cnt[x] == 0;
    }
  }
  int64_t ta, tb;
  (void)block_excl_scan<int64_t, CMP_NT>(a, &ta);
  (void)block_excl_scan<int64_t, CMP_NT>(b, &tb);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ta;
    part[2 * blockIdx.x + 1] = tb;
  }
}

// Single-block exclusive scan of the (isolated, empty) pairs per tile.
__global__ __launch_bounds__(1024) void k_iso_scan(int64_t *part, int64_t nb, const int64_t *iso_ctr) {
  if (*iso_ctr == 0) return;
  __shared__ int64_t carry[2];
  if (threadIdx.x == 0) carry[0] = carry[1] = 0;
  __syncthreads();
  for (int64_t s = 0; s < nb; s += 1024) {
    int64_t i = s + threadIdx.x;
    int64_t a = i < nb ? part[2 * i] : 0, b = i < nb ? part[2 * i + 1] : 0;
    int64_t ta, tb;
    int64_t pa = block_excl_scan<int64_t, 1024>(a, &ta);
    int64_t pb = block_excl_scan<int64_t, 1024>(b, &tb);
    if (i < nb) {
      part[2 * i] = carry[0] + pa;
      part[2 * i + 1] = carry[1] + pb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      carry[0] += ta;
      carry[1] += tb;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(CMP_NT) void k_iso_lists(const uint8_t *__restrict__ iso_flag,
                                                      const int32_t *__restrict__ cnt, int64_t n,
                                                      const int64_t *__restrict__ iso_ctr,
                                                      const int64_t *__restrict__ part,
                                                      int32_t *__restrict__ iso_list,
                                                      int32_t *__restrict__ empty_list) {
  const int64_t niso = *iso_ctr;
  if (niso == 0) return;
  const int64_t base = (int64_t)blockIdx.x * ISO_TILE + (int64_t)threadIdx.x * CMP_IPT;
  int64_t a = 0, b = 0;
#pragma unroll
  for (int i = 0; i < CMP_IPT; i++) {
    int64_t x = base + i;
    if (x < n) {
      a += iso_flag[x] != 0;
      b += cnt[x] == 0;
    }
  }
  int64_t ta, tb;
  int64_t pa = block_excl_scan<int64_t, CMP_NT>(a, &ta) + part[2 * blockIdx.x];
  int64_t pb = block_excl_scan<int64_t, CMP_NT>(b, &tb) + part[2 * blockIdx.x + 1];
#pragma unroll
  for (int i = 0; i < CMP_IPT; i++) {
    int64_t x = base + i;
    if (x < n) {
      if (iso_flag[x]) iso_list[pa++] = (int32_t)x;
      if (cnt[x] == 0) {
        if (pb < niso) empty_list[pb] = (int32_t)x;
        pb++;
      }
    }
  }
}

__global__ __launch_bounds__(BM_NT) void k_iso_pair(const int64_t *__restrict__ iso_ctr,
                                                    const int32_t *__restrict__ iso_list,
                                                    const int32_t *__restrict__ empty_list,
                                                    int32_t *__restrict__ C, int64_t *__restrict__ K,
                                                    int32_t *__restrict__ cnt, const int64_t *__restrict__ k,
                                                    uint8_t *__restrict__ iso_flag, int64_t n,
                                                    int64_t *__restrict__ err) {
  const int64_t niso = *iso_ctr;
  for (int64_t j = (int64_t)blockIdx.x * BM_NT + threadIdx.x; j < niso; j += (int64_t)gridDim.x * BM_NT) {
    const int32_t v = iso_list[j], x = empty_list[j];
    // by counting, at least niso ids are empty after the moves; a violation
    // is reported instead of indexing out of range
    if (v < 0 || (int64_t)v >= n || x < 0 || (int64_t)x >= n) {
      atomic_add_i64(err, 1);
      continue;
    }
    C[v] = x;
    K[x] = k[v];
    cnt[x] = 1;
    iso_flag[v] = 0;
  }
}

// --- partition of the active vertices into (sub-round, bin) buckets

__global__ __launch_bounds__(BM_NT) void k_part_count(const int32_t *__restrict__ list, int64_t na,
                                                      const int64_t *__restrict__ off, uint64_t h, int32_t S,
                                                      uint16_t *__restrict__ bucket_of,
                                                      int64_t *__restrict__ bcnt, int64_t *__restrict__ barcs) {
  extern __shared__ int64_t sm[];
  const int NB = S * NBINS;
  int64_t *lc = sm;
  int64_t *la = sm + NB;
  for (int i = threadIdx.x; i < 2 * NB; i += BM_NT) sm[i] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * BM_NT + threadIdx.x; i < na; i += (int64_t)gridDim.x * BM_NT) {
    const int32_t v = list ? list[i] : (int32_t)i;
    const int64_t deg = off[v + 1] - off[v];
    const int s = (int)(mix64(h ^ (uint64_t)(int64_t)v) % (uint64_t)S);
    const int b = s * NBINS + bin_of(deg);
    bucket_of[i] = (uint16_t)b;
    atomicAdd(reinterpret_cast<unsigned long long *>(&lc[b]), 1ull);
    if (deg) atomicAdd(reinterpret_cast<unsigned long long *>(&la[b]), (unsigned long long)deg);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NB; i += BM_NT) {
    if (lc[i]) atomic_add_i64(&bcnt[i], lc[i]);
    if (la[i]) atomic_add_i64(&barcs[i], la[i]);
  }
}

// Bucket starts (exclusive scan of the counts) into the scatter cursors.
__global__ void k_part_starts(const int64_t *__restrict__ bcnt, int64_t *__restrict__ cursor, int NB) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int64_t s = 0;
    for (int i = 0; i < NB; i++) {
      cursor[i] = s;
      s += bcnt[i];
    }
  }
}

__global__ __launch_bounds__(BM_NT) void k_part_scatter(const int32_t *__restrict__ list, int64_t na,
                                                        const uint16_t *__restrict__ bucket_of, int32_t S,
                                                        int64_t *__restrict__ cursor, int32_t *__restrict__ out) {
  extern __shared__ int64_t sm[];
  const int NB = S * NBINS;
  int64_t *lc = sm;        // items of this block per bucket
  int64_t *lbase = sm + NB;  // reserved global position per bucket
  for (int i = threadIdx.x; i < NB; i += BM_NT) lc[i] = 0;
  __syncthreads();
  // each block owns one contiguous range of the list
  const int64_t per = cdiv_dev(na, gridDim.x);
  const int64_t beg = (int64_t)blockIdx.x * per;
  const int64_t end = beg + per < na ? beg + per : na;
  for (int64_t i = beg + threadIdx.x; i < end; i += BM_NT)
    atomicAdd(reinterpret_cast<unsigned long long *>(&lc[bucket_of[i]]), 1ull);
  __syncthreads();
  for (int i = threadIdx.x; i < NB; i += BM_NT) {
    lbase[i] = lc[i] ? (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(&cursor[i]),
                                          (unsigned long long)lc[i])
                     : 0;
    lc[i] = 0;
  }
  __syncthreads();
  for (int64_t i = beg + threadIdx.x; i < end; i += BM_NT) {
    const int b = bucket_of[i];
    const int64_t r = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(&lc[b]), 1ull);
    out[lbase[b] + r] = list ? list[i] : (int32_t)i;
  }
}

__global__ void k_init_identity(const int64_t *__restrict__ k, int64_t *__restrict__ K, int32_t *__restrict__ cnt,
                                int64_t n) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    K[v] = k[v];
    cnt[v] = 1;
  }
}

// ------------------------------------------------------------------- host

namespace {

struct AggLaunch {
  int bin;
  int64_t verts, arcs;
  size_t pending_idx;  // index into ctx.pending when timed
  int slot;
};

template <int WK>
void launch_bin(Ctx &c, int bin, AggArgs a) {
  const int64_t cnt = a.count;
  switch (bin) {
    case 0:
      hipLaunchKernelGGL((k_bm_aggregate<8, 16, WK>), dim3((unsigned)cdiv(cnt, BM_NT / 8)), dim3(BM_NT), 0,
                         c.stream, a);
      break;
    case 1:
      hipLaunchKernelGGL((k_bm_aggregate<16, 32, WK>), dim3((unsigned)cdiv(cnt, BM_NT / 16)), dim3(BM_NT), 0,
                         c.stream, a);
      break;
    case 2:
      hipLaunchKernelGGL((k_bm_aggregate<32, 64, WK>), dim3((unsigned)cdiv(cnt, BM_NT / 32)), dim3(BM_NT), 0,
                         c.stream, a);
      break;
    case 3:
      hipLaunchKernelGGL((k_bm_aggregate<64, 128, WK>), dim3((unsigned)cdiv(cnt, BM_NT / 64)), dim3(BM_NT), 0,
                         c.stream, a);
      break;
    case 4:
      hipLaunchKernelGGL((k_bm_aggregate<64, 512, WK>), dim3((unsigned)cdiv(cnt, BM_NT / 64)), dim3(BM_NT), 0,
                         c.stream, a);
      break;
    case 5:
      hipLaunchKernelGGL((k_bm_aggregate_block<WK>), dim3((unsigned)cnt), dim3(BM_NT), 0, c.stream, a);
      break;
    default: {
      int64_t grid = cnt < (int64_t)c.num_cu * 2 ? cnt : (int64_t)c.num_cu * 2;
      hipLaunchKernelGGL((k_bm_aggregate_global<WK>), dim3((unsigned)grid), dim3(BM_NT), 0, c.stream, a);
    }
  }
  LAUNCHCHECK();
}

const char *bin_name(int b) {
  static const char *names[NBINS] = {"bm_aggregate_g8", "bm_aggregate_g16", "bm_aggregate_g32",
                                     "bm_aggregate_g64", "bm_aggregate_g64_h512", "bm_aggregate_block",
                                     "bm_aggregate_global"};
  return names[b];
}

}  // namespace

void best_moves(Ctx &c, const lcc_graph &g, int64_t p, int64_t q, const lcc_params &prm, int32_t level,
                int32_t phase, int32_t *C, bool identity, int64_t maxdeg, lcc_bm_stats &st) {
  std::memset(&st, 0, sizeof(st));
  const int64_t n = g.n;
  const int S = prm.S;
  const int NB = S * NBINS;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  int32_t *D = c.buf<int32_t>("bm.D", nn);
  int64_t *K = c.buf<int64_t>("bm.K", nn);
  int32_t *cnt = c.buf<int32_t>("bm.cnt", nn);
  uint8_t *next = c.buf<uint8_t>("bm.next", nn);
  uint8_t *iso = c.buf<uint8_t>("bm.iso", nn);
  int32_t *active = c.buf<int32_t>("bm.active", nn);
  int32_t *blist = c.buf<int32_t>("bm.blist", nn);
  uint16_t *bucket_of = c.buf<uint16_t>("bm.bucket", nn);
  int32_t *iso_list = c.buf<int32_t>("bm.isolist", nn);
  int32_t *empty_list = c.buf<int32_t>("bm.emptylist", nn);
  const int64_t iso_nb = cdiv(n > 0 ? n : 1, ISO_TILE);
  int64_t *iso_part = c.buf<int64_t>("bm.isopart", (size_t)(2 * iso_nb));
  // per iteration: bucket counts, bucket arcs, cursors, per-launch counters, per-sub-round isolations
  const size_t nctr = (size_t)NB * 3 + (size_t)NB * 4 + (size_t)S + 2;
  int64_t *dctr = c.buf<int64_t>("bm.ctr", nctr);
  int64_t *bcnt = dctr, *barcs = dctr + NB, *cursor = dctr + 2 * NB, *lctr = dctr + 3 * NB;
  int64_t *isoc = lctr + 4 * NB, *nact = isoc + S;
  std::vector<int64_t> hctr(nctr);

  if (n > 0) {
    HIPCHECK(hipMemsetAsync(next, 0, nn, c.stream));
    HIPCHECK(hipMemsetAsync(iso, 0, nn, c.stream));
    if (identity) {
      hipLaunchKernelGGL(k_init_identity, dim3((unsigned)std::min<int64_t>(cdiv(n, 256), 65535)), dim3(256), 0,
                         c.stream, g.k, K, cnt, n);
      LAUNCHCHECK();
    } else {
      cluster_totals(c, n, C, g.k, K, cnt);
    }
  }
  // global hash for the top bin
  int64_t gcap = 1;
  while (gcap < 2 * (maxdeg + 1)) gcap <<= 1;
  const int64_t ggrid = (int64_t)c.num_cu * 2;
  int32_t *gkeys = nullptr;
  int64_t *gvals = nullptr;
  if (maxdeg > bin_limit(NBINS - 2)) {
    gkeys = c.buf<int32_t>("bm.gkeys", (size_t)(gcap * ggrid));
    gvals = c.buf<int64_t>("bm.gvals", (size_t)(gcap * ggrid));
  }
  const int wb = wt_bytes(g.wt_kind);
  const bool nbr = prm.frontier == LCC_FRONTIER_NBR;
  const int32_t *list = nullptr;  // nullptr = every vertex
  int64_t na = n;
  st.term = LCC_TERM_NUM_ITER;
  bool stopped = false;
  for (int32_t it = 0; it < prm.num_iter && !stopped; it++) {
    const uint64_t h = round_hash(prm.seed, level, phase, it);
    st.iterations++;
    HIPCHECK(hipMemsetAsync(dctr, 0, nctr * sizeof(int64_t), c.stream));
    if (na > 0) {
      const size_t smem = (size_t)2 * NB * sizeof(int64_t);
      int64_t grid = std::min<int64_t>(cdiv(na, BM_NT * 8), (int64_t)c.num_cu * 8);
      hipLaunchKernelGGL(k_part_count, dim3((unsigned)grid), dim3(BM_NT), smem, c.stream, list, na, g.off, h, S,
                         bucket_of, bcnt, barcs);
      LAUNCHCHECK();
      hipLaunchKernelGGL(k_part_starts, dim3(1), dim3(1), 0, c.stream, bcnt, cursor, NB);
      LAUNCHCHECK();
      hipLaunchKernelGGL(k_part_scatter, dim3((unsigned)grid), dim3(BM_NT), smem, c.stream, list, na, bucket_of,
                         S, cursor, blist);
      LAUNCHCHECK();
    }
    d2h(c, hctr.data(), dctr, (size_t)2 * NB * sizeof(int64_t));
    std::vector<int64_t> start(NB + 1, 0);
    for (int i = 0; i < NB; i++) start[i + 1] = start[i] + hctr[i];
    std::vector<AggLaunch> launches;
    if (it < LCC_MAX_ITER_STATS) st.active_per_iter[it] = na;
    for (int s = 0; s < S; s++) {
      if (prm.stop_after_subrounds > 0 && st.subrounds >= prm.stop_after_subrounds) {
        st.term = LCC_TERM_STOPPED;
        stopped = true;
        break;
      }
      int64_t total_s = 0;
      for (int b = 0; b < NBINS; b++) {
        const int bi = s * NBINS + b;
        const int64_t cntb = hctr[bi];
        if (!cntb) continue;
        total_s += cntb;
        AggArgs a;
        a.off = g.off;
        a.col = g.col;
        a.wt = g.wt;
        a.k = g.k;
        a.C = C;
        a.K = K;
        a.cnt = cnt;
        a.p = p;
        a.q = q;
        a.allow_iso = prm.allow_isolate;
        a.list = blist + start[bi];
        a.count = cntb;
        a.D = D;
        a.next_flag = nbr ? next : nullptr;
        a.ctr = lctr + 4 * bi;
        a.gkeys = gkeys;
        a.gvals = gvals;
        a.gcap = gcap;
        const double arcs_b = (double)hctr[NB + bi];
        size_t pidx = c.pending.size();
        {
          Ctx::Timer tm(&c, bin_name(b), (double)cntb * 48.0 + arcs_b * (8.0 + wb), arcs_b);
          switch (g.wt_kind) {
            case LCC_WT_UNIT: launch_bin<LCC_WT_UNIT>(c, b, a); break;
            case LCC_WT_I16: launch_bin<LCC_WT_I16>(c, b, a); break;
            case LCC_WT_I32: launch_bin<LCC_WT_I32>(c, b, a); break;
            default: launch_bin<LCC_WT_I64>(c, b, a); break;
          }
        }
        launches.push_back({b, cntb, hctr[NB + bi], c.timing ? pidx : (size_t)-1, bi});
        st.vertices_processed += cntb;
        st.arcs_scanned += hctr[NB + bi];
      }
      if (total_s > 0) {
        {
          Ctx::Timer tm(&c, "bm_apply", (double)total_s * 12.0, (double)total_s);
          hipLaunchKernelGGL(k_bm_apply, dim3((unsigned)cdiv(total_s, BM_NT)), dim3(BM_NT), 0, c.stream,
                             blist + start[s * NBINS], total_s, D, C, K, cnt, g.k, iso, isoc + s);
          LAUNCHCHECK();
        }
        if (prm.allow_isolate) {
          Ctx::Timer tm(&c, "bm_isolate", 0.0, 0.0);
          hipLaunchKernelGGL(k_iso_count, dim3((unsigned)iso_nb), dim3(CMP_NT), 0, c.stream, iso, cnt, n, isoc + s,
                             iso_part);
          LAUNCHCHECK();
          hipLaunchKernelGGL(k_iso_scan, dim3(1), dim3(1024), 0, c.stream, iso_part, iso_nb, isoc + s);
          LAUNCHCHECK();
          hipLaunchKernelGGL(k_iso_lists, dim3((unsigned)iso_nb), dim3(CMP_NT), 0, c.stream, iso, cnt, n, isoc + s,
                             iso_part, iso_list, empty_list);
          LAUNCHCHECK();
          hipLaunchKernelGGL(k_iso_pair, dim3((unsigned)std::min<int64_t>(cdiv(n, BM_NT), 1024)), dim3(BM_NT), 0,
                             c.stream, isoc + s, iso_list, empty_list, C, K, cnt, g.k, iso, n, nact + 1);
          LAUNCHCHECK();
        }
      }
      st.subrounds++;
    }
    // next frontier
    bool more = false;
    if (nbr && n > 0) {
      compact_flags(c, next, n, active, nact, true, "bm.cmp");
    }
    d2h(c, hctr.data() + 3 * NB, lctr, (size_t)(4 * NB + S + 2) * sizeof(int64_t));
    const int64_t *hl = hctr.data() + 3 * NB;
    int64_t moved_it = 0;
    int64_t cap_err = 0;
    for (int i = 0; i < NB; i++) {
      moved_it += hl[4 * i];
      st.candidates += hl[4 * i + 1];
      cap_err += hl[4 * i + 3];
    }
    if (cap_err) fail(LCC_ERR_DEVICE, "internal: a vertex degree exceeded the hash capacity sized from the maximum degree");
    if (hl[4 * NB + S + 1]) fail(LCC_ERR_DEVICE, "internal: isolated vertices outnumbered the empty cluster ids");
    if (c.timing) {
      for (auto &L : launches) {
        if (L.pending_idx < c.pending.size()) {
          // candidates gather K (8 B each); movers store one flag per neighbor
          c.pending[L.pending_idx].bytes += 8.0 * (double)hl[4 * L.slot + 1] + (double)hl[4 * L.slot + 2];
        }
      }
    }
    if (it < LCC_MAX_ITER_STATS) st.moves_per_iter[it] = moved_it;
    st.moves += moved_it;
    if (moved_it) st.moved_any = 1;
    if (stopped) break;
    if (moved_it == 0) {
      st.term = LCC_TERM_NO_MOVES;
      break;
    }
    (void)more;
    if (nbr) {
      na = hl[4 * NB + S];
      list = active;
    } else {
      na = n;
      list = nullptr;
    }
  }
  if (c.timing) c.collect_timing();
}

}  // namespace lcc
