// bestmove.hip -- Best-Moves (paper Algorithm 1, top) on gfx950.
//
// One iteration = S synchronous sub-rounds.  For each iteration the active
// vertices are partitioned into (sub-round, degree bin) buckets; every
// sub-round then runs one aggregation kernel per non-empty degree bin, one
// apply kernel and one isolation kernel:
//
//   aggregate  the vertex's CSR row is streamed (coalesced col / weight
//              reads), C[u] gathered and the weight summed per neighbor
//              cluster in an open-addressing hash table; every distinct
//              cluster is then scored against the snapshot (int64:
//              q*w - p*k_v*K_X), the best (score desc, id asc) is reduced
//              across the lanes, the decision written to D[v], and a mover
//              marks its neighbors in the next frontier.  Degree bins pick the
//              shape: 8/16/32/64-lane groups with a private LDS table (degree
//              < 256), a block per vertex with a degree-sized table in up to
//              160 KB of LDS, and a 1024-thread block with a global-memory
//              table for the rare rows beyond that.
//   apply      movers update C and the cluster totals K / sizes with int64 /
//              int32 atomics (integer adds commute, so the order of the
//              atomics never matters); a vertex v that isolates moves to the
//              fresh id n + v (a vertex is in one sub-round per iteration, so
//              the id is unused within the iteration).
//
// At the end of an iteration in which someone isolated, the non-empty fresh
// clusters are renamed, ascending, to the ascending empty ids in [0, n).
//
// Nothing in a sub-round reads what the same sub-round writes: aggregation
// reads C, K, cnt and writes only D / flags / counters; apply runs after it.
#include "ops.hpp"
#include "prims.hpp"

namespace lcc {

constexpr int BM_NT = 256;
constexpr int WIDE_NT = 1024;
constexpr int NBINS = 8;
constexpr int NSPREAD = 8;   // counter copies per launch (spreads same-address atomics)
constexpr int NCTR = 7;  // movers, candidates, arcs of movers, capacity errors, shared rows, their arcs,
                         // hub partitions that overflowed
constexpr int32_t ISO_ID = INT32_MAX;  // ranks after every real cluster id

// Thrown by a Best-Moves call whose hub partitions overflowed (see k_hp_part).
struct HubOverflow {};
constexpr int MID_SLOTS = 4096;        // table of the block-per-vertex bin (degree < 2048)

// Largest degree of each bin; bin 6's limit depends on the LDS size and the
// accumulator width and is passed at run time.
__host__ __device__ constexpr int64_t bin_limit_fixed(int b) {
  return b == 0 ? 7 : b == 1 ? 15 : b == 2 ? 31 : b == 3 ? 63 : b == 4 ? 255 : 2047;
}
__host__ __device__ inline int bin_of(int64_t deg, int64_t wide_max) {
  if (deg <= 2047) {
    int b = 0;
    while (deg > bin_limit_fixed(b)) b++;
    return b;
  }
  return deg <= wide_max ? 6 : 7;
}

// Batched runs: several independent jobs packed block-diagonally in one graph.
// Each vertex belongs to one job; the job supplies lambda, the base that
// turns a vertex id into its job-local id (the sub-round hash uses local
// ids), whether the job is still iterating, and a per-job mover counter.
struct JobView {
  const int32_t *jid = nullptr;  // nullptr: one job, scalar lambda
  const int64_t *jbase = nullptr;
  const int64_t *jp = nullptr;
  const int64_t *jq = nullptr;
  const uint8_t *jrun = nullptr;
  int64_t *jmoved = nullptr;
};

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
  uint8_t *next_flag;  // neighbors-of-movers frontier: movers mark their neighbors here
  uint8_t *left_flag;  // neighbors-of-clusters frontier: movers mark the cluster they left here
  int64_t *ctr;        // NSPREAD x NCTR counters of this launch
  int32_t *gkeys;      // global tables (bin 7)
  int64_t *gvals;
  int64_t hcap;        // table capacity in slots (dynamic-LDS or global bins)
  JobView jv;
  // device-driven launches: the vertices are
  // list[dstart[bucket] .. dstart[bucket + nbuckets]) (consecutive buckets)
  const int64_t *dstart;
  int32_t bucket;
  int32_t nbuckets;
  // small levels keep two copies of (C, K, cnt): a sub-round reads one and
  // applies its own moves to the other (Cw, Kw, cntw), into which it also
  // replays the previous sub-round's moves (buckets rb0 .. rb1-1 of list;
  // none when rb1 <= rb0).  Cw == nullptr: a separate apply kernel runs.
  // Asynchronous moves: Cw, Kw, cntw are C, K, cnt themselves, so a move is
  // applied to the state the other decisions read the moment it is decided.
  int32_t *Cw;
  int64_t *Kw;
  int32_t *cntw;
  int64_t nlev;       // vertices of the level (fresh ids are nlev + v)
  int64_t *iso_ctr;   // isolations of the sub-round
  int32_t rb0, rb1;
  int32_t hub_limit;  // distinct clusters a hub partition may hold (see k_hp_part)
  int32_t hub_row_limit;  // one-pass hub rows: 0 automatic, -1 never, k > 0 at most k clusters (k_hub_row)
  int32_t prune;          // 1 = pruned scoring (see score_floor) in the kernels that use it
  int32_t *hub_seen;      // per vertex: distinct clusters its hub row met when last decided (k_hub_row)
};

// The launch's vertex list and count (host-given, or read from the bucket
// starts in device memory).
__device__ __forceinline__ void work_of(const AggArgs &a, const int32_t *&list, int64_t &count) {
  if (a.dstart) {
    const int64_t b0 = a.dstart[a.bucket];
    list = a.list + b0;
    count = a.dstart[a.bucket + a.nbuckets] - b0;
  } else {
    list = a.list;
    count = a.count;
  }
}

// lambda of the job owning v (the scalar lambda outside batched runs).
__device__ __forceinline__ void job_lambda(const AggArgs &a, int32_t v, int64_t &p, int64_t &q, int32_t &job) {
  if (a.jv.jid) {
    job = a.jv.jid[v];
    p = a.jv.jp[job];
    q = a.jv.jq[job];
  } else {
    job = 0;
    p = a.p;
    q = a.q;
  }
}

// Applies v's move c -> d (d < 0: to the fresh id nlev + v) to the copy
// (Cw, Kw, cntw); integer atomics, so the order of moves never matters.
__device__ __forceinline__ void apply_to_copy(const AggArgs &a, int32_t v, int32_t c, int32_t d, int64_t kv) {
  const int32_t t = d < 0 ? (int32_t)(a.nlev + v) : d;
  if (kv) {
    atomic_add_i64(&a.Kw[c], -kv);
    atomic_add_i64(&a.Kw[t], kv);
  }
  atomicSub(&a.cntw[c], 1);
  atomicAdd(&a.cntw[t], 1);
  a.Cw[v] = t;
}

// A vertex's own move in the copy, counted (isolations, moved jobs).
__device__ __forceinline__ void own_move(const AggArgs &a, int32_t v, int32_t c, int32_t d, int64_t kv,
                                         int64_t &niso) {
  apply_to_copy(a, v, c, d, kv);
  if (d < 0) niso++;
  if (a.jv.jid) a.jv.jmoved[a.jv.jid[v]] = 1;
}

// The previous sub-round's moves replayed into the copy (whole grid).  The
// copy still holds those vertices' old clusters, so a decision that differs
// from it is a move.
template <int NT> __device__ __forceinline__ void replay_prev(const AggArgs &a) {
  if (a.rb1 <= a.rb0) return;
  const int64_t lo = a.dstart[a.rb0], hi = a.dstart[a.rb1];
  for (int64_t i = lo + (int64_t)blockIdx.x * NT + threadIdx.x; i < hi; i += (int64_t)gridDim.x * NT) {
    const int32_t v = a.list[i];
    const int32_t d = a.D[v], c = a.Cw[v];
    if (d != c) apply_to_copy(a, v, c, d, a.k[v]);
  }
}

// (score, id) order: higher score first, then lower id.
__device__ __forceinline__ bool better(int64_t s, int32_t id, int64_t bs, int32_t bid) {
  return s > bs || (s == bs && id < bid);
}

// Pruned scoring.  With p >= 0 and every k >= 0, a candidate's score
// q*w_X - p*k_v*K_X never exceeds q*w_X.  The heaviest candidate other than
// the vertex's own cluster, X*, has a score L that the best score reaches at
// least, so a candidate with q*w_X < L scores strictly below the best and can
// neither win nor tie: its K_X is never read.  On level 0 most candidates
// share a single arc with the vertex while the few clusters it belongs with
// share many, so nearly all K gathers go away.  The decision is unchanged.
// It pays where K misses the caches (a level of at least PRUNE_MIN_N
// vertices) and rows are long enough that the extra pass over the table is
// small beside the gathers it saves (the block-per-row kernels and the
// 512-slot lane groups); elsewhere the kernels score every candidate.
constexpr int64_t PRUNE_MIN_N = (int64_t)1 << 23;
__device__ __forceinline__ void heavier(int64_t w, int32_t X, int64_t &bw, int32_t &bX) {
  if (w > bw || (w == bw && X < bX)) {
    bw = w;
    bX = X;
  }
}

// (weight, id) of the heaviest candidate over the G lanes of a group.
template <int G> __device__ __forceinline__ void group_heaviest(int64_t &bw, int32_t &bX) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) heavier(__shfl_xor(bw, o, WAVE), __shfl_xor(bX, o, WAVE), bw, bX);
}

// The same over a block of NT threads; every thread gets the result.
template <int NT> __device__ __forceinline__ void block_heaviest(int64_t &bw, int32_t &bX) {
  group_heaviest<WAVE>(bw, bX);
  __shared__ int64_t hw[NT / WAVE];
  __shared__ int32_t hx[NT / WAVE];
  if (lane_id() == 0) {
    hw[threadIdx.x / WAVE] = bw;
    hx[threadIdx.x / WAVE] = bX;
  }
  __syncthreads();
  for (int i = 0; i < NT / WAVE; i++) heavier(hw[i], hx[i], bw, bX);
}

// L from the heaviest candidate (INT64_MIN when the vertex has none).
__device__ __forceinline__ int64_t score_floor(const int64_t *__restrict__ K, int64_t lq, int64_t pk, int64_t bw,
                                               int32_t bX) {
  return bX == INT32_MAX ? INT64_MIN : lq * bw - pk * K[bX];
}


// Multiplicative hash reduced to [0, H) (H need not be a power of two).
__device__ __forceinline__ uint32_t slot_of(int32_t X, uint32_t H) {
  return (uint32_t)(((uint64_t)((uint32_t)X * 0x9E3779B1u) * (uint64_t)H) >> 32);
}

// Pruned scoring, the bound that needs no gather at all (the other one is
// score_floor's): a vertex moves only to a target scoring strictly above its
// stay score, so a candidate with q*w_X <= stay can never be the one it
// moves to; and leaving such candidates out cannot change whether the empty
// cluster (score 0) is taken instead, since that needs 0 > stay as well.
// The stay score comes from the vertex's own cluster weight, read from its
// slot of the table (the own cluster is always inserted), and K_c, loaded
// with the vertex.
template <class Acc>
__device__ __forceinline__ int64_t own_weight(const int32_t *keys, const Acc *vals, uint32_t H, int32_t c) {
  uint32_t h = slot_of(c, H);
  while (keys[h] != c) h = (h + 1 == H) ? 0 : h + 1;
  return (int64_t)vals[h];
}

__device__ __forceinline__ uint32_t pow2_at_least(int64_t x) {
  uint32_t h = 1;
  while ((int64_t)h < x) h <<= 1;
  return h;
}

// Adds w to key X in an LDS table of H slots (keys -1 = empty).  The caller
// guarantees fewer distinct keys than slots.
template <class Acc>
__device__ __forceinline__ void lds_insert(int32_t *keys, Acc *vals, uint32_t H, int32_t X, int64_t w) {
  uint32_t h = slot_of(X, H);
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
    h = (h + 1 == H) ? 0 : h + 1;
  }
}

// lds_insert that reports the slot it claimed for a new key (-1 otherwise).
template <class Acc>
__device__ __forceinline__ int32_t lds_insert_claim(int32_t *keys, Acc *vals, uint32_t H, int32_t X, int64_t w) {
  uint32_t h = slot_of(X, H);
  int32_t claimed = -1;
  while (true) {
    int32_t cur = keys[h];
    if (cur == -1) {
      cur = atomicCAS(&keys[h], -1, X);
      if (cur == -1) {
        claimed = (int32_t)h;
        cur = X;
      }
    }
    if (cur == X) {
      if (w) {
        if constexpr (sizeof(Acc) == 8)
          atomicAdd(reinterpret_cast<unsigned long long *>(&vals[h]), (unsigned long long)w);
        else
          atomicAdd(&vals[h], (Acc)w);
      }
      return claimed;
    }
    h = (h + 1 == H) ? 0 : h + 1;
  }
}

// Appends the slots the lanes of a wave claimed (claimed >= 0) to the
// occupied list: one LDS atomic per wave.  Every lane of the wave calls it.
__device__ __forceinline__ void list_claims(int32_t claimed, uint16_t *occ, int32_t *occ_n) {
  const uint64_t m = __ballot(claimed >= 0);
  if (!m) return;
  const int lead = __ffsll((unsigned long long)m) - 1;
  int32_t base = 0;
  if (lane_id() == lead) base = atomicAdd(occ_n, (int32_t)__popcll(m));
  base = __shfl(base, lead, WAVE);
  if (claimed >= 0) occ[base + __popcll(m & __lanemask_lt())] = (uint16_t)claimed;
}

// Decision from the reduced results (identical in every lane of the group).
__device__ __forceinline__ int32_t decide(int64_t best_s, int32_t best_id, int64_t stay, bool iso_ok, int32_t c) {
  if (iso_ok && (best_s == INT64_MIN || 0 > best_s)) {
    best_s = 0;
    best_id = ISO_ID;
  }
  if (best_s != INT64_MIN && best_s > stay) return best_id == ISO_ID ? -1 : best_id;
  return c;
}

// Block-wide sum of the counters; one atomic per counter per block, spread
// over NSPREAD copies.
template <int NT, int NV = 3>
__device__ __forceinline__ void flush_counters(int64_t *ctr, int64_t movers, int64_t cands, int64_t marcs,
                                               int64_t rows = 0, int64_t row_arcs = 0) {
  __shared__ int64_t red[NV][NT / WAVE];
  int64_t x[5] = {movers, cands, marcs, rows, row_arcs};
  const int w = threadIdx.x / WAVE;
#pragma unroll
  for (int k = 0; k < NV; k++) {
    const int64_t t = wave_sum(x[k]);
    if (lane_id() == 0) red[k][w] = t;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    int64_t s = 0;
    for (int i = 0; i < NT / WAVE; i++) s += red[threadIdx.x][i];
    // counters 0-2, then (NV = 5) 4-5: slot 3 holds capacity errors
    const int slot = threadIdx.x < 3 ? threadIdx.x : threadIdx.x + 1;
    if (s) atomic_add_i64(&ctr[(blockIdx.x % NSPREAD) * NCTR + slot], s);
  }
}

// Reduces (best score, best id, own-cluster weight) over a block of NT
// threads; the result is valid in thread 0.
template <int NT>
__device__ __forceinline__ void block_best(int64_t &best_s, int32_t &best_id, int64_t &wc) {
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
  __shared__ int64_t rs[NT / WAVE];
  __shared__ int32_t rid[NT / WAVE];
  __shared__ int64_t rw[NT / WAVE];
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    rs[w] = best_s;
    rid[w] = best_id;
    rw[w] = wc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < NT / WAVE; i++) {
      if (better(rs[i], rid[i], best_s, best_id)) {
        best_s = rs[i];
        best_id = rid[i];
      }
      wc += rw[i];
    }
  }
}

// ---------------------------------------------------------- lane groups

// G lanes per vertex (G <= 64, inside one wavefront), a private LDS table of
// up to HMAX slots per vertex (2G slots when HMAX == 2G: one arc per lane).
template <int G, int HMAX, int WK, bool A32>
__global__ __launch_bounds__(BM_NT) void k_bm_group(AggArgs a) {
  using Acc = typename std::conditional<A32, int32_t, int64_t>::type;
  constexpr int GPB = BM_NT / G;
  constexpr bool ONE_PASS = HMAX == 2 * G;
  __shared__ int32_t hk[GPB * HMAX];
  __shared__ Acc hv[GPB * HMAX];
  const int t = threadIdx.x, grp = t / G, gl = t % G;
  const int32_t *list;
  int64_t count;
  work_of(a, list, count);
  int64_t c_movers = 0, c_cands = 0, c_marcs = 0, c_iso = 0;
  for (int64_t g0 = (int64_t)blockIdx.x * GPB; g0 < count; g0 += (int64_t)gridDim.x * GPB) {
    const int64_t gi = g0 + grp;
    const bool valid = gi < count;
    int32_t *keys = hk + grp * HMAX;
    Acc *vals = hv + grp * HMAX;
    int32_t v = 0, c = 0;
    int64_t beg = 0, end = 0;
    if (valid) {
      v = list[gi];
      beg = a.off[v];
      end = a.off[v + 1];
      c = a.C[v];
    }
    uint32_t H = HMAX;
    if constexpr (!ONE_PASS) {
      H = pow2_at_least(2 * (end - beg + 1));
      if (H > (uint32_t)HMAX) H = HMAX;
    }
    for (uint32_t j = gl; j < H; j += G) {
      keys[j] = -1;
      vals[j] = 0;
    }
    // loads the decision needs, issued before the row is walked
    int64_t kv = 0, Kc = 0;
    int32_t cntc = 0;
    if (valid) {
      kv = a.k[v];
      Kc = a.K[c];
      cntc = a.cnt[c];
    }
    __syncthreads();
    int32_t u0 = -1;
    if (valid) {
      if (gl == 0) lds_insert<Acc>(keys, vals, H, c, 0);
      if constexpr (ONE_PASS) {
        const int64_t e = beg + gl;
        if (e < end) {
          u0 = a.col[e];
          lds_insert<Acc>(keys, vals, H, a.C[u0], load_w<WK>(a.wt, e));
        }
      } else {
        for (int64_t base = beg + gl; base < end; base += 4 * G) {
          int32_t u[4], X[4];
          int64_t w[4];
#pragma unroll
          for (int j = 0; j < 4; j++) {
            const int64_t e = base + j * G;
            u[j] = e < end ? a.col[e] : -1;
            w[j] = e < end ? load_w<WK>(a.wt, e) : 0;
          }
#pragma unroll
          for (int j = 0; j < 4; j++) X[j] = u[j] >= 0 ? a.C[u[j]] : -1;
#pragma unroll
          for (int j = 0; j < 4; j++)
            if (X[j] >= 0) lds_insert<Acc>(keys, vals, H, X[j], w[j]);
        }
      }
    }
    __syncthreads();
    int64_t best_s = INT64_MIN, wc = 0, ncand = 0;
    int32_t best_id = ISO_ID;
    int64_t lp = 0, lq = 1;
    int32_t job = 0;
    if (valid) job_lambda(a, v, lp, lq, job);
    const int64_t pk = lp * kv;
    int64_t hw = INT64_MIN;
    int32_t hX = INT32_MAX;
    if (HMAX >= 512 && a.prune) {
      if (valid)
        for (uint32_t j = gl; j < H; j += G) {
          const int32_t X = keys[j];
          if (X >= 0 && X != c) heavier((int64_t)vals[j], X, hw, hX);
        }
      group_heaviest<G>(hw, hX);
    }
    if (valid) {
      const int64_t L = score_floor(a.K, lq, pk, hw, hX);
      const int64_t stay0 = lq * own_weight(keys, vals, H, c) - pk * (Kc - kv);
      for (uint32_t j = gl; j < H; j += G) {
        const int32_t X = keys[j];
        if (X < 0) continue;
        ncand++;
        const int64_t wx = (int64_t)vals[j];
        if (X == c) {
          wc = wx;
        } else if (lq * wx >= L && lq * wx > stay0) {
          const int64_t s = lq * wx - pk * a.K[X];
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
      const int64_t stay = lq * wc - pk * (Kc - kv);
      const int32_t d = decide(best_s, best_id, stay, a.allow_iso && cntc >= 2, c);
      moved = d != c;
      if (gl == 0) a.D[v] = d;
      if (moved && gl == 0 && a.left_flag) a.left_flag[c] = 1;
      if (moved && gl == 0 && a.Cw) own_move(a, v, c, d, kv, c_iso);
      if (moved && a.next_flag) {
        if constexpr (ONE_PASS) {
          if (u0 >= 0) a.next_flag[u0] = 1;
        } else {
          for (int64_t e = beg + gl; e < end; e += G) a.next_flag[a.col[e]] = 1;
        }
      }
    }
    c_movers += (moved && gl == 0) ? 1 : 0;
    c_cands += ncand;
    c_marcs += (moved && gl == 0) ? end - beg : 0;
    __syncthreads();  // the tables are cleared again for the next vertices
  }
  if (c_iso) atomic_add_i64(a.iso_ctr, c_iso);
  flush_counters<BM_NT>(a.ctr, c_movers, c_cands, c_marcs);
}

// ------------------------------------------------------- block per vertex

// One vertex per block, a table of min(hcap, pow2 >= 2(deg+1)) slots in
// dynamic LDS (keys then values).  The host admits a vertex only when its
// distinct clusters (<= deg + 1) fill at most 70% of hcap.
// TAG only separates launch classes in kernel traces (1 = small levels).
// With LIST, a slot is cleared the first time a vertex of the block reaches
// it; after that the slots a vertex filled (listed in occ, one uint16 per
// slot after the values) are all that scoring reads and all that is reset for
// the next vertex, so a row with few distinct clusters costs little in a large
// table.  Without LIST each vertex clears and scans its H slots (less LDS per
// block, so more resident blocks).
template <int NT, int WK, bool A32, int TAG = 0, bool LIST = true>
__global__ __launch_bounds__(NT) void k_bm_wide(AggArgs a) {
  using Acc = typename std::conditional<A32, int32_t, int64_t>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  int32_t *keys = reinterpret_cast<int32_t *>(smem);
  Acc *vals = reinterpret_cast<Acc *>(smem + ((a.hcap * 4 + 15) & ~15ll));
  uint16_t *occ = reinterpret_cast<uint16_t *>(smem + ((a.hcap * 4 + 15) & ~15ll) + a.hcap * sizeof(Acc));
  __shared__ int32_t sh_d, occ_n;
  const int t = threadIdx.x;
  const int32_t *list;
  int64_t count;
  work_of(a, list, count);
  if (t == 0) occ_n = 0;
  uint32_t clean = 0;  // slots [0, clean) hold no key (block-uniform)
  int64_t movers = 0, marcs = 0, cands = 0, niso = 0;
  if (a.Cw) replay_prev<NT>(a);
  for (int64_t vi = blockIdx.x; vi < count; vi += gridDim.x) {
    const int32_t v = list[vi];
    const int64_t beg = a.off[v], end = a.off[v + 1];
    const int32_t c = a.C[v];
    uint32_t H = pow2_at_least(2 * (end - beg + 1));
    if (H > (uint32_t)a.hcap) H = (uint32_t)a.hcap;
    const int64_t kv = a.k[v], Kc = a.K[c];
    const int32_t cntc = a.cnt[c];
    for (uint32_t j = (LIST ? clean : 0) + t; j < H; j += NT) {
      keys[j] = -1;
      vals[j] = 0;
    }
    if (H > clean) clean = H;
    __syncthreads();
    if (t == 0) {
      const int32_t h0 = lds_insert_claim<Acc>(keys, vals, H, c, 0);
      if (LIST && h0 >= 0) occ[atomicAdd(&occ_n, 1)] = (uint16_t)h0;
    }
    for (int64_t base = beg + t; base < end; base += 4 * NT) {
      int32_t u[4], X[4];
      int64_t w[4];
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int64_t e = base + j * NT;
        u[j] = e < end ? a.col[e] : -1;
        w[j] = e < end ? load_w<WK>(a.wt, e) : 0;
      }
#pragma unroll
      for (int j = 0; j < 4; j++) X[j] = u[j] >= 0 ? a.C[u[j]] : -1;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int32_t claimed = X[j] >= 0 ? lds_insert_claim<Acc>(keys, vals, H, X[j], w[j]) : -1;
        if constexpr (LIST) list_claims(claimed, occ, &occ_n);
      }
    }
    __syncthreads();
    int64_t lp, lq;
    int32_t job;
    job_lambda(a, v, lp, lq, job);
    const int64_t pk = lp * kv;
    int64_t best_s = INT64_MIN, wc = 0;
    int32_t best_id = ISO_ID;
    const int32_t nocc = LIST ? occ_n : (int32_t)H;
    int64_t hw = INT64_MIN;
    int32_t hX = INT32_MAX;
    if (a.prune) {  // uniform: a launch argument
      for (int32_t j = t; j < nocc; j += NT) {
        const uint32_t h = LIST ? occ[j] : (uint32_t)j;
        const int32_t X = keys[h];
        if (X >= 0 && X != c) heavier((int64_t)vals[h], X, hw, hX);
      }
      block_heaviest<NT>(hw, hX);
    }
    const int64_t L = score_floor(a.K, lq, pk, hw, hX);
    const int64_t stay0 = lq * own_weight(keys, vals, H, c) - pk * (Kc - kv);
    for (int32_t j = t; j < nocc; j += NT) {
      const uint32_t h = LIST ? occ[j] : (uint32_t)j;
      const int32_t X = keys[h];
      if (!LIST && X < 0) continue;
      cands++;
      const int64_t wx = (int64_t)vals[h];
      if (X == c) {
        wc = wx;
      } else if (lq * wx >= L && lq * wx > stay0) {
        const int64_t s = lq * wx - pk * a.K[X];
        if (better(s, X, best_s, best_id)) {
          best_s = s;
          best_id = X;
        }
      }
    }
    block_best<NT>(best_s, best_id, wc);
    if (t == 0) {
      const int64_t stay = lq * wc - pk * (Kc - kv);
      const int32_t d = decide(best_s, best_id, stay, a.allow_iso && cntc >= 2, c);
      a.D[v] = d;
      sh_d = d;
      if (d != c) {
        movers += 1;
        marcs += end - beg;
        if (a.left_flag) a.left_flag[c] = 1;
        if (a.Cw) own_move(a, v, c, d, kv, niso);
      }
    }
    __syncthreads();
    if (sh_d != c && a.next_flag)
      for (int64_t e = beg + t; e < end; e += NT) a.next_flag[a.col[e]] = 1;
    if constexpr (LIST) {  // leave the table clean for the next vertex
      for (int32_t j = t; j < nocc; j += NT) {
        keys[occ[j]] = -1;
        vals[occ[j]] = 0;
      }
    }
    __syncthreads();  // table, occ and sh_d are reused by the next vertex
    if (t == 0) occ_n = 0;
  }
  if (t == 0 && niso) atomic_add_i64(a.iso_ctr, niso);
  flush_counters<NT>(a.ctr, movers, cands, marcs);
}

// ------------------------------------- lambda sweep: shared level-0 rows

// A sweep runs up to SH_MAXJ clusterings of one graph (one per lambda) as a
// batch whose jobs are identical copies: job j owns vertices [j*n1, (j+1)*n1)
// and its rows are job 0's rows shifted by j*n1.  For rows of degree < 256 one
// launch serves every job: the block takes a vertex v, wave j aggregates job
// j's row of v, and the cluster ids of neighbor u for all jobs sit in one
// 64-byte line C16[u][0..15], so the 16 waves share each row read and each
// neighbor's line (fetched once into L1, hit by the other waves).  Decisions
// equal those of the per-job kernels: same table, same scores, same order.
constexpr int SH_MAXJ = 16;
constexpr int SH_BIN_HI = 4;   // bins 0..SH_BIN_HI (degree <= 255) share rows
constexpr int SH_SLOTS = 512;  // per-wave table: pow2 >= 2 (255 + 1)

// C16[v][j] = C[j*n1 + v] for j < J, -1 beyond: one thread per vertex writes
// its 64-byte line (reads of each job's C are coalesced across the wave).
__global__ void k_sh_transpose(const int32_t *__restrict__ C, int64_t n1, int32_t J, int32_t *__restrict__ C16) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n1; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t x[SH_MAXJ];
#pragma unroll
    for (int j = 0; j < SH_MAXJ; j++) x[j] = j < J ? C[(int64_t)j * n1 + v] : -1;
    int4 *line = reinterpret_cast<int4 *>(C16 + v * SH_MAXJ);
#pragma unroll
    for (int q = 0; q < SH_MAXJ / 4; q++) line[q] = make_int4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
  }
}

// From the sub-round's buckets b0 .. b1-1 (packed ids j*n1 + v): mask[v] |=
// 1 << j, and every v whose mask was empty is appended to one of NSPREAD
// list segments (segment k = blocks with blockIdx % NSPREAD == k, capacity n1
// each, count in seg_cnt[k]), one atomic per block and step.  The list order
// varies from run to run; nothing downstream depends on it.
__global__ __launch_bounds__(BM_NT) void k_sh_mask(const int32_t *__restrict__ list0,
                                                   const int64_t *__restrict__ dstart, int32_t b0, int32_t b1,
                                                   int64_t n1, uint32_t *__restrict__ mask,
                                                   int32_t *__restrict__ seglist, int64_t *__restrict__ seg_cnt) {
  __shared__ int32_t wcnt[BM_NT / WAVE];
  __shared__ int64_t bbase;
  const int64_t lo = dstart[b0], hi = dstart[b1];
  const int seg = blockIdx.x % NSPREAD, wv = threadIdx.x / WAVE;
  int32_t *out = seglist + (int64_t)seg * n1;
  for (int64_t base = lo + (int64_t)blockIdx.x * BM_NT; base < hi; base += (int64_t)gridDim.x * BM_NT) {
    const int64_t i = base + threadIdx.x;
    bool first = false;
    int32_t v = 0;
    if (i < hi) {
      const int32_t vp = list0[i];
      const int32_t j = (int32_t)(vp / n1);
      v = (int32_t)(vp - (int64_t)j * n1);
      first = atomicOr(&mask[v], 1u << j) == 0;
    }
    const uint64_t m = __ballot(first);
    if (lane_id() == 0) wcnt[wv] = (int32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t tot = 0;
      for (int w = 0; w < BM_NT / WAVE; w++) tot += wcnt[w];
      bbase = tot ? (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(&seg_cnt[seg]),
                                       (unsigned long long)tot)
                  : 0;
    }
    __syncthreads();
    if (first) {
      int64_t pos = bbase + __popcll(m & __lanemask_lt());
      for (int w = 0; w < wv; w++) pos += wcnt[w];
      out[pos] = v;
    }
    __syncthreads();  // wcnt and bbase are reused by the next step
  }
}

// The id of job j (wave-uniform) among the 16 ids of a neighbor's line.
__device__ __forceinline__ int32_t pick16(const int4 &a, const int4 &b, const int4 &c, const int4 &d, int j) {
  const int4 q = j < 8 ? (j < 4 ? a : b) : (j < 12 ? c : d);
  const int r = j & 3;
  return r == 0 ? q.x : r == 1 ? q.y : r == 2 ? q.z : q.w;
}

// One wave per listed vertex (SH_WPB waves per block, each on its own
// vertex and its own table).  The wave loads the row (from job 0, the first
// n1 vertices) and every neighbor's line of 16 ids once, into registers, then
// runs the jobs of the vertex's mask one after another: insert, score against
// job j's C, K and cnt, decide, mark job j's frontier.  The scoring scan
// resets each slot it reads, so the table is clean for the next job without a
// clearing pass.  The vertex's mask is cleared for the next sub-round.
constexpr int SH_WPB = BM_NT / WAVE;

template <int WK, bool A32>
__global__ __launch_bounds__(BM_NT) void k_bm_shared(AggArgs a, const int32_t *__restrict__ C16, int64_t n1,
                                                     uint32_t *__restrict__ mask, const int32_t *__restrict__ seglist,
                                                     const int64_t *__restrict__ seg_cnt) {
  using Acc = typename std::conditional<A32, int32_t, int64_t>::type;
  __shared__ int32_t hk[SH_WPB * SH_SLOTS];
  __shared__ Acc hv[SH_WPB * SH_SLOTS];
  const int wv = threadIdx.x / WAVE, gl = lane_id();
  int32_t *keys = hk + wv * SH_SLOTS;
  Acc *vals = hv + wv * SH_SLOTS;
  for (int s = gl; s < SH_SLOTS; s += WAVE) {
    keys[s] = -1;
    vals[s] = 0;
  }
  __builtin_amdgcn_wave_barrier();
  int64_t total = 0;
  for (int k = 0; k < NSPREAD; k++) total += seg_cnt[k];
  int64_t c_movers = 0, c_cands = 0, c_marcs = 0, c_rows = 0, c_rarcs = 0;
  for (int64_t vi = (int64_t)blockIdx.x * SH_WPB + wv; vi < total; vi += (int64_t)gridDim.x * SH_WPB) {
    int k = 0;
    int64_t r = vi;
    while (r >= seg_cnt[k]) r -= seg_cnt[k++];  // vi < total: ends at a segment below NSPREAD
    const int32_t v = seglist[(int64_t)k * n1 + r];
    const uint32_t m = mask[v];
    __builtin_amdgcn_wave_barrier();
    if (gl == 0) mask[v] = 0;
    const int64_t beg = a.off[v], end = a.off[v + 1];
    const uint32_t H = pow2_at_least(2 * (end - beg + 1));
    const int64_t kv = a.k[v];
    int32_t u[4];
    int64_t w[4];
    int4 q0[4], q1[4], q2[4], q3[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int64_t e = beg + gl + i * WAVE;
      u[i] = e < end ? a.col[e] : -1;
      w[i] = e < end ? load_w<WK>(a.wt, e) : 0;
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
      if (u[i] >= 0) {
        const int4 *line = reinterpret_cast<const int4 *>(C16 + (int64_t)u[i] * SH_MAXJ);
        q0[i] = line[0];
        q1[i] = line[1];
        q2[i] = line[2];
        q3[i] = line[3];
      } else {
        q0[i] = q1[i] = q2[i] = q3[i] = make_int4(-1, -1, -1, -1);
      }
    }
    // lane j < 16 fetches job j's cluster of v (from v's own line), its
    // total and its size: one round trip for all jobs
    int32_t cj = 0, cntj = 0;
    int64_t Kj = 0;
    if (gl < SH_MAXJ && ((m >> gl) & 1u)) {
      cj = C16[(int64_t)v * SH_MAXJ + gl];
      Kj = a.K[cj];
      cntj = a.cnt[cj];
    }
    for (uint32_t mm = m; mm; mm &= mm - 1) {
      const int j = __ffs((int)mm) - 1;
      const int64_t vp = (int64_t)j * n1 + v;
      const int32_t c = __shfl(cj, j, WAVE);
      const int64_t Kc = __shfl(Kj, j, WAVE);
      const int32_t cntc = __shfl(cntj, j, WAVE);
      if (gl == 0) lds_insert<Acc>(keys, vals, H, c, 0);
#pragma unroll
      for (int i = 0; i < 4; i++)
        if (u[i] >= 0) lds_insert<Acc>(keys, vals, H, pick16(q0[i], q1[i], q2[i], q3[i], j), w[i]);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const int64_t lp = a.jv.jp[j], lq = a.jv.jq[j];
      const int64_t pk = lp * kv;
      int64_t best_s = INT64_MIN, wc = 0;
      int32_t best_id = ISO_ID;
      const int64_t stay0 = lq * own_weight(keys, vals, H, c) - pk * (Kc - kv);  // (before the scan clears)
      int64_t hw = INT64_MIN;
      int32_t hX = INT32_MAX;
      if (a.prune) {
        for (uint32_t s = gl; s < H; s += WAVE) {
          const int32_t X = keys[s];
          if (X >= 0 && X != c) heavier((int64_t)vals[s], X, hw, hX);
        }
        group_heaviest<WAVE>(hw, hX);
      }
      const int64_t L = score_floor(a.K, lq, pk, hw, hX);
      for (uint32_t s = gl; s < H; s += WAVE) {
        const int32_t X = keys[s];
        if (X < 0) continue;
        const int64_t wx = (int64_t)vals[s];
        keys[s] = -1;
        vals[s] = 0;
        c_cands++;
        if (X == c) {
          wc = wx;
        } else if (lq * wx >= L && lq * wx > stay0) {
          const int64_t sc = lq * wx - pk * a.K[X];
          if (better(sc, X, best_s, best_id)) {
            best_s = sc;
            best_id = X;
          }
        }
      }
#pragma unroll
      for (int o = WAVE / 2; o > 0; o >>= 1) {
        const int64_t os = __shfl_xor(best_s, o, WAVE);
        const int32_t oid = __shfl_xor(best_id, o, WAVE);
        if (better(os, oid, best_s, best_id)) {
          best_s = os;
          best_id = oid;
        }
        wc += __shfl_xor(wc, o, WAVE);
      }
      const int64_t stay = lq * wc - pk * (Kc - kv);
      const int32_t d = decide(best_s, best_id, stay, a.allow_iso && cntc >= 2, c);
      if (gl == 0) a.D[vp] = d;
      if (d != c) {
        if (a.next_flag) {
          const int64_t jb = (int64_t)j * n1;
#pragma unroll
          for (int i = 0; i < 4; i++)
            if (u[i] >= 0) a.next_flag[jb + u[i]] = 1;
        }
        if (gl == 0) {
          c_movers++;
          c_marcs += end - beg;
          if (a.left_flag) a.left_flag[c] = 1;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();  // the table is clean for the next job
    }
    if (gl == 0) {
      c_rows++;
      c_rarcs += end - beg;
    }
  }
  flush_counters<BM_NT, 5>(a.ctr, c_movers, c_cands, c_marcs, c_rows, c_rarcs);
}


// ------------------------------------------------ first iteration, singletons

// First sub-round of a coarsening Best-Moves (C = identity) on rows without
// repeated neighbors: every neighbor u is its own cluster with K_u = k_u, so
// no aggregation is needed.  The best target is the neighbor maximizing
// q*w(v,u) - p*k_v*k_u (ties to the lowest id); staying scores 0 and
// isolation is not available (|c| = 1).  G lanes per vertex, or the whole
// block when G == NT.
template <int G, int NT, int WK, int TAG = 0>
__global__ __launch_bounds__(NT) void k_bm_single(AggArgs a) {
  constexpr int GPB = NT / G;
  __shared__ int32_t sh_d[GPB];
  const int t = threadIdx.x, grp = t / G, gl = t % G;
  const int32_t *list;
  int64_t count;
  work_of(a, list, count);
  int64_t c_movers = 0, c_cands = 0, c_marcs = 0, c_iso = 0;  // (singletons never isolate)
  if (a.Cw) replay_prev<NT>(a);
  for (int64_t g0 = (int64_t)blockIdx.x * GPB; g0 < count; g0 += (int64_t)gridDim.x * GPB) {
    const int64_t gi = g0 + grp;
    const bool valid = gi < count;
    int32_t v = 0;
    int64_t beg = 0, end = 0, kv = 0;
    if (valid) {
      v = list[gi];
      beg = a.off[v];
      end = a.off[v + 1];
      kv = a.k[v];
    }
    int64_t lp = 0, lq = 1;
    int32_t job = 0;
    if (valid) job_lambda(a, v, lp, lq, job);
    const int64_t pk = lp * kv;
    int64_t best_s = INT64_MIN, wc = 0;
    int32_t best_id = ISO_ID;
    for (int64_t base = beg + gl; base < end; base += 4 * G) {
      int32_t u[4];
      int64_t w[4], ku[4];
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int64_t e = base + j * G;
        u[j] = e < end ? a.col[e] : -1;
        w[j] = e < end ? load_w<WK>(a.wt, e) : 0;
      }
#pragma unroll
      for (int j = 0; j < 4; j++) ku[j] = u[j] >= 0 ? a.k[u[j]] : 0;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        if (u[j] < 0) continue;
        const int64_t sc = lq * w[j] - pk * ku[j];
        if (better(sc, u[j], best_s, best_id)) {
          best_s = sc;
          best_id = u[j];
        }
      }
    }
    int32_t d = v;
    if constexpr (G < NT) {
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) {
        int64_t os = __shfl_xor(best_s, o, WAVE);
        int32_t oid = __shfl_xor(best_id, o, WAVE);
        if (better(os, oid, best_s, best_id)) {
          best_s = os;
          best_id = oid;
        }
      }
      d = decide(best_s, best_id, 0, false, v);
    } else {
      block_best<NT>(best_s, best_id, wc);
      if (t == 0) sh_d[0] = decide(best_s, best_id, 0, false, v);
      __syncthreads();
      d = sh_d[0];
    }
    const bool moved = valid && d != v;
    if (valid && gl == 0) a.D[v] = d;
    if (moved && gl == 0 && a.Cw) own_move(a, v, v, d, kv, c_iso);
    if (moved && gl == 0 && a.left_flag) a.left_flag[v] = 1;
    if (moved && a.next_flag)
      for (int64_t e = beg + gl; e < end; e += G) a.next_flag[a.col[e]] = 1;
    c_movers += (moved && gl == 0) ? 1 : 0;
    c_cands += (valid && gl == 0) ? end - beg + 1 : 0;
    c_marcs += (moved && gl == 0) ? end - beg : 0;
    if constexpr (G == NT) __syncthreads();  // sh_d is reused by the next vertex
  }
  flush_counters<NT>(a.ctr, c_movers, c_cands, c_marcs);
}

// ------------------------------------------------------ flat hub aggregation

// Rows too wide for LDS are aggregated chunk-parallel: every row is cut into
// chunks of B7_CHUNK arcs, one block per chunk, so a 400k-neighbor row is
// spread over hundreds of blocks.  A chunk is first summed by cluster in an
// LDS table, then its distinct clusters go to the row's table of
// cap = pow2 >= 2(deg+1) slots in global memory, so repeated clusters cost
// one global atomic per chunk instead of one per arc.  A separate kernel
// then scores every row's table in segments of B7_SEG slots.
constexpr int B7_NT = 256;
constexpr int B7L_NT = 1024;
constexpr int64_t B7_SEG = 4096;
constexpr int64_t B7_CHUNK = 2048;
constexpr int B7_CHUNK_SLOTS = 4096;

// Layout of the bucket's hub rows, in one block: exclusive prefixes of the
// chunk counts (cstart), table capacities (tstart) and scoring segments
// (sstart), n7 + 1 entries each; tot = {chunks, slots, segments, n7}.

__global__ __launch_bounds__(B7L_NT) void k_b7_layout(AggArgs a, int64_t *__restrict__ cstart,
                                                      int64_t *__restrict__ tstart, int64_t *__restrict__ sstart,
                                                      int64_t *__restrict__ tot) {
  const int32_t *list;
  int64_t n7;
  work_of(a, list, n7);
  int64_t ca = 0, ct = 0, cs = 0;
  for (int64_t i0 = 0; i0 < n7; i0 += B7L_NT) {
    const int64_t i = i0 + threadIdx.x;
    int64_t nc = 0, cap = 0, ns = 0;
    if (i < n7) {
      const int32_t v = list[i];
      const int64_t d = a.off[v + 1] - a.off[v];
      nc = cdiv(d, B7_CHUNK);
      cap = pow2_at_least(2 * (d + 1));
      ns = cdiv(cap, B7_SEG);
    }
    int64_t td, tc, tn;
    const int64_t pd = block_excl_scan<int64_t, B7L_NT>(nc, &td);
    const int64_t pc = block_excl_scan<int64_t, B7L_NT>(cap, &tc);
    const int64_t pn = block_excl_scan<int64_t, B7L_NT>(ns, &tn);
    if (i < n7) {
      cstart[i] = ca + pd;
      tstart[i] = ct + pc;
      sstart[i] = cs + pn;
    }
    ca += td;
    ct += tc;
    cs += tn;
  }
  if (threadIdx.x == 0) {
    cstart[n7] = ca;
    tstart[n7] = ct;
    sstart[n7] = cs;
    tot[0] = ca;
    tot[1] = ct;
    tot[2] = cs;
    tot[3] = n7;
  }
}

// Packed tables (every row's sum of |w| below 2^31, so every partial sum
// fits 32 bits): one 64-bit slot holds the key (high half) and its weight
// sum (low half), so a new key is claimed with its first weight in one CAS
// and repeated keys add to the low half with a 32-bit atomic.
constexpr unsigned long long PK_EMPTY = 0xFFFFFFFF00000000ull;

template <bool PK>
__global__ void k_b7_clear(int32_t *__restrict__ keys, int64_t *__restrict__ vals, const int64_t *__restrict__ tot) {
  const int64_t total = tot[1];
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (int64_t)gridDim.x * blockDim.x) {
    if constexpr (PK) {
      reinterpret_cast<unsigned long long *>(vals)[j] = PK_EMPTY;
    } else {
      keys[j] = -1;
      vals[j] = 0;
    }
  }
}

// Adds w to key X in a global table of H slots (keys -1 = empty).  Keys and
// values only change through atomics inside this kernel.
__device__ __forceinline__ void global_insert(int32_t *keys, int64_t *vals, uint32_t H, int32_t X, int64_t w) {
  uint32_t h = slot_of(X, H);
  while (true) {
    int32_t cur = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == -1) {
      cur = atomicCAS(&keys[h], -1, X);
      if (cur == -1) cur = X;
    }
    if (cur == X) {
      if (w) atomic_add_i64(&vals[h], w);
      return;
    }
    h = (h + 1 == H) ? 0 : h + 1;
  }
}

__device__ __forceinline__ void global_insert_packed(unsigned long long *tab, uint32_t H, int32_t X, int32_t w) {
  uint32_t h = slot_of(X, H);
  const unsigned long long mine = ((unsigned long long)(uint32_t)X << 32) | (unsigned long long)(uint32_t)w;
  while (true) {
    unsigned long long cur = __hip_atomic_load(&tab[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == PK_EMPTY) {
      const unsigned long long old = atomicCAS(&tab[h], PK_EMPTY, mine);
      if (old == PK_EMPTY) return;  // claimed with the first weight
      cur = old;
    }
    if ((int32_t)(cur >> 32) == X) {
      // the low half (little-endian), never the key
      if (w) atomicAdd(reinterpret_cast<int32_t *>(&tab[h]), w);
      return;
    }
    h = (h + 1 == H) ? 0 : h + 1;
  }
}

// One block per chunk (cstart / tstart hold n7 + 1 entries): the chunk's
// arcs are summed by cluster in LDS, then each distinct cluster is added to
// the row's global table; the row's first chunk also enters its own cluster.
template <int WK, bool PK>
__global__ __launch_bounds__(B7_NT) void k_b7_insert(AggArgs a, const int64_t *__restrict__ tot,
                                                     const int64_t *__restrict__ cstart,
                                                     const int64_t *__restrict__ tstart) {
  __shared__ int32_t lk[B7_CHUNK_SLOTS];
  __shared__ int64_t lv[B7_CHUNK_SLOTS];
  __shared__ int64_t sh_row;
  const int32_t *list;
  int64_t cnt7;
  work_of(a, list, cnt7);
  const int64_t nch = tot[0], n7 = tot[3];
  const int t = threadIdx.x;
  for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
    if (t == 0) {  // row holding this chunk
      int64_t lo = 0, hi = n7 - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (cstart[mid] <= ch) lo = mid;
        else hi = mid - 1;
      }
      sh_row = lo;
    }
    for (int j = t; j < B7_CHUNK_SLOTS; j += B7_NT) {
      lk[j] = -1;
      lv[j] = 0;
    }
    __syncthreads();
    const int64_t i = sh_row;
    const int32_t v = list[i];
    const int64_t beg = a.off[v], end = a.off[v + 1];
    const int64_t e0 = beg + (ch - cstart[i]) * B7_CHUNK;
    const int64_t e1 = e0 + B7_CHUNK < end ? e0 + B7_CHUNK : end;
    if (e0 == beg && t == 0) lds_insert<int64_t>(lk, lv, B7_CHUNK_SLOTS, a.C[v], 0);
    for (int64_t base = e0 + t; base < e1; base += 4 * B7_NT) {
      int32_t u[4], X[4];
      int64_t w[4];
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int64_t e = base + j * B7_NT;
        u[j] = e < e1 ? a.col[e] : -1;
        w[j] = e < e1 ? load_w<WK>(a.wt, e) : 0;
      }
#pragma unroll
      for (int j = 0; j < 4; j++) X[j] = u[j] >= 0 ? a.C[u[j]] : -1;
#pragma unroll
      for (int j = 0; j < 4; j++)
        if (X[j] >= 0) lds_insert<int64_t>(lk, lv, B7_CHUNK_SLOTS, X[j], w[j]);
    }
    __syncthreads();
    const int64_t t0 = tstart[i];
    const uint32_t H = (uint32_t)(tstart[i + 1] - t0);
    for (int j = t; j < B7_CHUNK_SLOTS; j += B7_NT) {
      if (lk[j] < 0) continue;
      if constexpr (PK)
        global_insert_packed(reinterpret_cast<unsigned long long *>(a.gvals) + t0, H, lk[j], (int32_t)lv[j]);
      else
        global_insert(a.gkeys + t0, a.gvals + t0, H, lk[j], lv[j]);
    }
    __syncthreads();  // the LDS table and sh_row are reused by the next chunk
  }
}

// Scoring of the hub tables, one block per B7_SEG-slot segment (a row's
// table spans cdiv(cap, B7_SEG) segments, sstart = prefix of segment counts).

struct SegBest {
  int64_t best_s;
  int64_t wc;
  int64_t cands;
  int32_t best_id;
  int32_t pad;
};

template <bool PK>
__global__ __launch_bounds__(B7_NT) void k_b7_segscore(AggArgs a, const int64_t *__restrict__ tot,
                                                       const int64_t *__restrict__ tstart,
                                                       const int64_t *__restrict__ sstart,
                                                       SegBest *__restrict__ part) {
  const int32_t *list;
  int64_t cnt7;
  work_of(a, list, cnt7);
  const int64_t nsg = tot[2], n7 = tot[3];
  for (int64_t sg = blockIdx.x; sg < nsg; sg += gridDim.x) {
    // row owning this segment
    int64_t lo = 0, hi = n7 - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (sstart[mid] <= sg) lo = mid;
      else hi = mid - 1;
    }
    const int64_t i = lo;
    const int32_t v = list[i];
    const int32_t c = a.C[v];
    int64_t lp, lq;
    int32_t job;
    job_lambda(a, v, lp, lq, job);
    const int64_t pk = lp * a.k[v];
    const int64_t t0 = tstart[i], H = tstart[i + 1] - t0;
    const int64_t j0 = (sg - sstart[i]) * B7_SEG;
    const int64_t j1 = j0 + B7_SEG < H ? j0 + B7_SEG : H;
    int64_t best_s = INT64_MIN, wc = 0, cands = 0;
    int32_t best_id = ISO_ID;
    // the tables were filled by device-scope atomics in the previous kernel:
    // read them with device-scope loads as well
    for (int64_t j = j0 + threadIdx.x; j < j1; j += B7_NT) {
      int32_t X;
      int64_t wx;
      if constexpr (PK) {
        const unsigned long long sl = __hip_atomic_load(reinterpret_cast<unsigned long long *>(a.gvals) + t0 + j,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        X = (int32_t)(sl >> 32);
        wx = (int64_t)(int32_t)(uint32_t)sl;
      } else {
        X = __hip_atomic_load(&a.gkeys[t0 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (X >= 0) wx = __hip_atomic_load(&a.gvals[t0 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (X < 0) continue;
      cands++;
      if (X == c) {
        wc = wx;
      } else {
        const int64_t sc = lq * wx - pk * a.K[X];
        if (better(sc, X, best_s, best_id)) {
          best_s = sc;
          best_id = X;
        }
      }
    }
    cands = wave_sum(cands);
    __shared__ int64_t rc[B7_NT / WAVE];
    if (lane_id() == 0) rc[threadIdx.x / WAVE] = cands;
    block_best<B7_NT>(best_s, best_id, wc);
    if (threadIdx.x == 0) {
      int64_t tc = 0;
      for (int k = 0; k < B7_NT / WAVE; k++) tc += rc[k];
      part[sg] = SegBest{best_s, wc, tc, best_id, 0};
    }
    __syncthreads();  // rc is reused by the next segment
  }
}

// One block per row: combines the row's segments, decides, marks the frontier.
__global__ __launch_bounds__(B7_NT) void k_b7_final(AggArgs a, const int64_t *__restrict__ sstart,
                                                    const SegBest *__restrict__ part,
                                                    const uint8_t *__restrict__ done) {
  __shared__ int32_t sh_d;
  const int t = threadIdx.x;
  const int32_t *list;
  int64_t n7;
  work_of(a, list, n7);
  int64_t movers = 0, marcs = 0, cands = 0, niso = 0;
  for (int64_t i = blockIdx.x; i < n7; i += gridDim.x) {
    if (done && done[i]) continue;  // decided by k_hub_row (block-uniform)
    const int32_t v = list[i];
    const int64_t beg = a.off[v], end = a.off[v + 1];
    const int32_t c = a.C[v];
    const int64_t kv = a.k[v], Kc = a.K[c];
    const int32_t cntc = a.cnt[c];
    int64_t best_s = INT64_MIN, wc = 0;
    int32_t best_id = ISO_ID;
    for (int64_t sg = sstart[i] + t; sg < sstart[i + 1]; sg += B7_NT) {
      const SegBest b = part[sg];
      if (better(b.best_s, b.best_id, best_s, best_id)) {
        best_s = b.best_s;
        best_id = b.best_id;
      }
      wc += b.wc;
      cands += b.cands;
    }
    block_best<B7_NT>(best_s, best_id, wc);
    if (t == 0) {
      int64_t lp, lq;
      int32_t job;
      job_lambda(a, v, lp, lq, job);
      const int64_t stay = lq * wc - lp * kv * (Kc - kv);
      const int32_t d = decide(best_s, best_id, stay, a.allow_iso && cntc >= 2, c);
      a.D[v] = d;
      sh_d = d;
      if (d != c) {
        movers += 1;
        marcs += end - beg;
        if (a.left_flag) a.left_flag[c] = 1;
        if (a.Cw) own_move(a, v, c, d, kv, niso);
      }
    }
    __syncthreads();
    if (sh_d != c && a.next_flag)
      for (int64_t e = beg + t; e < end; e += B7_NT) a.next_flag[a.col[e]] = 1;
    __syncthreads();  // sh_d is reused by the next row
  }
  if (t == 0 && niso) atomic_add_i64(a.iso_ctr, niso);
  flush_counters<B7_NT>(a.ctr, movers, cands, marcs);
}

// ------------------------------------------- partitioned hub aggregation

// Hub rows without global atomics: every hub arc's cluster id is gathered
// once into a per-row buffer (xs), then each row is cut into P hash
// partitions of its clusters (a multiplier independent of the table hash),
// one 1024-thread block per partition, aggregated and scored in LDS.  P is
// chosen so that a partition expects half of HP_LIMIT distinct clusters.  A
// partition that meets more than the limit stops claiming slots before its
// table fills (so probing always ends) and counts an overflow; the host then
// redoes the whole Best-Moves call with the global tables, which give the
// same result.
constexpr int HP_NT = 1024;
constexpr int HP_SLOTS = 12288;
constexpr int HP_LIMIT = HP_SLOTS * 7 / 10;
constexpr int HP_STOP = HP_SLOTS - 2 * HP_NT;  // claims never exceed this
// Up to this widest row every partition reads its whole row (at most 16
// partitions); a level with wider rows first scatters each row's ids by
// partition (k_hps_count, k_hps_scatter), so a partition reads only its own.
constexpr int64_t HP_MAX_DEG = 65536;
// Partitions per row are capped (LDS histograms); a row so wide that its
// partitions then overflow takes the redo with the global tables.
constexpr int HPS_MAXP = 4096;

__host__ __device__ inline int64_t hp_parts(int64_t deg) {
  const int64_t p = cdiv(2 * (deg + 1), HP_LIMIT);
  return p < HPS_MAXP ? p : HPS_MAXP;
}

__device__ __forceinline__ uint32_t part_of(int32_t X, uint32_t P) {
  return (uint32_t)(((uint64_t)((uint32_t)X * 0x85EBCA6Bu) * (uint64_t)P) >> 32);
}

// Layout of the bucket's hub rows, in one block: prefixes of gather chunks
// (cstart), degrees (xoff) and partitions (pstart), n7 + 1 entries each;
// tot = {chunks, arcs, partitions, n7}.
__global__ __launch_bounds__(B7L_NT) void k_hp_layout(AggArgs a, int64_t *__restrict__ cstart,
                                                      int64_t *__restrict__ xoff, int64_t *__restrict__ pstart,
                                                      int64_t *__restrict__ tot, const uint8_t *__restrict__ done) {
  const int32_t *list;
  int64_t n7;
  work_of(a, list, n7);
  int64_t ca = 0, cx = 0, cp = 0;
  for (int64_t i0 = 0; i0 < n7; i0 += B7L_NT) {
    const int64_t i = i0 + threadIdx.x;
    int64_t nc = 0, d = 0, np = 0;
    if (i < n7 && !done[i]) {  // rows decided in one pass take no chunks or partitions
      const int32_t v = list[i];
      d = a.off[v + 1] - a.off[v];
      nc = cdiv(d, B7_CHUNK);
      np = hp_parts(d);
    }
    int64_t tc, tx, tp;
    const int64_t pc = block_excl_scan<int64_t, B7L_NT>(nc, &tc);
    const int64_t px = block_excl_scan<int64_t, B7L_NT>(d, &tx);
    const int64_t pp = block_excl_scan<int64_t, B7L_NT>(np, &tp);
    if (i < n7) {
      cstart[i] = ca + pc;
      xoff[i] = cx + px;
      pstart[i] = cp + pp;
    }
    ca += tc;
    cx += tx;
    cp += tp;
  }
  if (threadIdx.x == 0) {
    cstart[n7] = ca;
    xoff[n7] = cx;
    pstart[n7] = cp;
    tot[0] = ca;
    tot[1] = cx;
    tot[2] = cp;
    tot[3] = n7;
  }
}

// One block per chunk of B7_CHUNK arcs: xs[xoff[row] + j] = C[col[beg + j]].
__global__ __launch_bounds__(B7_NT) void k_hp_gather(AggArgs a, const int64_t *__restrict__ tot,
                                                     const int64_t *__restrict__ cstart,
                                                     const int64_t *__restrict__ xoff, int32_t *__restrict__ xs) {
  __shared__ int64_t sh_row;
  const int32_t *list;
  int64_t cnt7;
  work_of(a, list, cnt7);
  const int64_t nch = tot[0], n7 = tot[3];
  for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
    __syncthreads();  // sh_row is reused
    if (threadIdx.x == 0) {
      int64_t lo = 0, hi = n7 - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (cstart[mid] <= ch) lo = mid;
        else hi = mid - 1;
      }
      sh_row = lo;
    }
    __syncthreads();
    const int64_t i = sh_row;
    const int32_t v = list[i];
    const int64_t beg = a.off[v], end = a.off[v + 1];
    const int64_t e0 = beg + (ch - cstart[i]) * B7_CHUNK;
    const int64_t e1 = e0 + B7_CHUNK < end ? e0 + B7_CHUNK : end;
    int32_t *out = xs + xoff[i] - beg;
    for (int64_t base = e0 + threadIdx.x; base < e1; base += 4 * B7_NT) {
      int32_t u[4];
#pragma unroll
      for (int j = 0; j < 4; j++) u[j] = base + j * B7_NT < e1 ? a.col[base + j * B7_NT] : -1;
#pragma unroll
      for (int j = 0; j < 4; j++)
        if (u[j] >= 0) out[base + j * B7_NT] = a.C[u[j]];
    }
  }
}

// Adds w to key X unless the table already holds `stop` claims (then false).
template <class Acc>
__device__ __forceinline__ bool lds_insert_bounded(int32_t *keys, Acc *vals, int32_t X, int64_t w, int32_t *nclaim,
                                                   int32_t stop) {
  uint32_t h = slot_of(X, HP_SLOTS);
  while (true) {
    int32_t cur = keys[h];
    if (cur == -1) {
      if (atomicAdd(nclaim, 1) >= stop) return false;
      cur = atomicCAS(&keys[h], -1, X);
      if (cur == -1) {
        cur = X;
      } else {
        atomicSub(nclaim, 1);  // another key took the slot first
      }
    }
    if (cur == X) {
      if (w) {
        if constexpr (sizeof(Acc) == 8)
          atomicAdd(reinterpret_cast<unsigned long long *>(&vals[h]), (unsigned long long)w);
        else
          atomicAdd(&vals[h], (Acc)w);
      }
      return true;
    }
    h = (h + 1 == (uint32_t)HP_SLOTS) ? 0 : h + 1;
  }
}

// lds_insert_bounded that also reports a slot it claimed (-1 otherwise).
template <class Acc>
__device__ __forceinline__ bool lds_insert_bounded_claim(int32_t *keys, Acc *vals, int32_t X, int64_t w,
                                                         int32_t *nclaim, int32_t stop, int32_t &claimed) {
  uint32_t h = slot_of(X, HP_SLOTS);
  while (true) {
    int32_t cur = keys[h];
    if (cur == -1) {
      if (atomicAdd(nclaim, 1) >= stop) return false;
      cur = atomicCAS(&keys[h], -1, X);
      if (cur == -1) {
        cur = X;
        claimed = (int32_t)h;
      } else {
        atomicSub(nclaim, 1);  // another key took the slot first
      }
    }
    if (cur == X) {
      if (w) {
        if constexpr (sizeof(Acc) == 8)
          atomicAdd(reinterpret_cast<unsigned long long *>(&vals[h]), (unsigned long long)w);
        else
          atomicAdd(&vals[h], (Acc)w);
      }
      return true;
    }
    h = (h + 1 == (uint32_t)HP_SLOTS) ? 0 : h + 1;
  }
}

// One block per partition: its clusters' weights summed in LDS, then scored
// (as the per-row kernels do) into part[partition]; an overflow counts in
// counter 6 of the launch.  With 32-bit sums the table (96 KB) leaves room
// for a list of the claimed slots (24 KB): the table is cleared once per
// block, and scoring and the reset for the next partition touch only the
// listed slots, a few thousand instead of all 12288.
template <int WK, bool A32, bool SEG>
__global__ __launch_bounds__(HP_NT) void k_hp_part(AggArgs a, const int64_t *__restrict__ tot,
                                                   const int64_t *__restrict__ xoff,
                                                   const int64_t *__restrict__ pstart,
                                                   const int32_t *__restrict__ xs, SegBest *__restrict__ part,
                                                   const int64_t *__restrict__ segstart,
                                                   const int64_t *__restrict__ pcnt,
                                                   const int64_t *__restrict__ ws) {
  using Acc = typename std::conditional<A32, int32_t, int64_t>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  int32_t *keys = reinterpret_cast<int32_t *>(smem);
  Acc *vals = reinterpret_cast<Acc *>(smem + (size_t)HP_SLOTS * sizeof(int32_t));
  constexpr bool LIST = A32;
  uint16_t *occ = reinterpret_cast<uint16_t *>(smem + (size_t)HP_SLOTS * (sizeof(int32_t) + sizeof(Acc)));
  __shared__ int32_t nclaim, occ_n;
  __shared__ int64_t sh_row;
  const int t = threadIdx.x;
  const int32_t *list;
  int64_t cnt7;
  work_of(a, list, cnt7);
  const int64_t np = tot[2], n7 = tot[3];
  const int32_t limit = a.hub_limit > 0 ? a.hub_limit : HP_LIMIT;
  int64_t overflows = 0;
  if (LIST) {
    for (int s = t; s < HP_SLOTS; s += HP_NT) {
      keys[s] = -1;
      vals[s] = 0;
    }
    if (t == 0) occ_n = 0;
  }
  for (int64_t pi = blockIdx.x; pi < np; pi += gridDim.x) {
    __syncthreads();  // the table, nclaim and sh_row are reused
    if (!LIST)
      for (int s = t; s < HP_SLOTS; s += HP_NT) {
        keys[s] = -1;
        vals[s] = 0;
      }
    if (t == 0) {
      nclaim = 0;
      int64_t lo = 0, hi = n7 - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (pstart[mid] <= pi) lo = mid;
        else hi = mid - 1;
      }
      sh_row = lo;
    }
    __syncthreads();
    const int64_t i = sh_row;
    const int32_t v = list[i];
    const int64_t beg = a.off[v], deg = a.off[v + 1] - beg;
    const uint32_t P = (uint32_t)(pstart[i + 1] - pstart[i]), p = (uint32_t)(pi - pstart[i]);
    const int32_t c = a.C[v];
    const int32_t *x = SEG ? xs : xs + xoff[i];
    if (t == 0 && part_of(c, P) == p) {
      int32_t h0 = -1;
      lds_insert_bounded_claim<Acc>(keys, vals, c, 0, &nclaim, HP_STOP, h0);
      if (LIST && h0 >= 0) occ[atomicAdd(&occ_n, 1)] = (uint16_t)h0;
    }
    if constexpr (SEG) {  // this partition's ids and weights, scattered
      const int64_t s0 = segstart[pi], s1 = s0 + pcnt[pi];
      // every lane of a wave runs the same trips (the claims are listed per wave)
      for (int64_t j0 = s0; j0 < s1; j0 += HP_NT) {
        const int64_t j = j0 + t;
        int32_t h = -1;
        if (j < s1) lds_insert_bounded_claim<Acc>(keys, vals, xs[j], ws[j], &nclaim, HP_STOP, h);
        if (LIST) list_claims(h, occ, &occ_n);
      }
    } else {
      for (int64_t j0 = 0; j0 < deg; j0 += HP_NT) {
        const int64_t j = j0 + t;
        int32_t h = -1;
        if (j < deg) {
          const int32_t X = x[j];
          if (part_of(X, P) == p)
            lds_insert_bounded_claim<Acc>(keys, vals, X, load_w<WK>(a.wt, beg + j), &nclaim, HP_STOP, h);
        }
        if (LIST) list_claims(h, occ, &occ_n);
      }
    }
    __syncthreads();
    const int32_t nocc = LIST ? occ_n : HP_SLOTS;
    const bool over = nclaim > limit;  // block-uniform
    if (t == 0 && a.hub_seen) atomicAdd(&a.hub_seen[v], nclaim);
    int64_t lp, lq;
    int32_t job;
    job_lambda(a, v, lp, lq, job);
    const int64_t pk = lp * a.k[v];
    int64_t best_s = INT64_MIN, wc = 0, cands = 0;
    int32_t best_id = ISO_ID;
    // pruned as the per-row kernels are, against this partition's heaviest
    // candidate (a partition's best is exact; the row's is their maximum)
    int64_t hw = INT64_MIN;
    int32_t hX = INT32_MAX;
    if (a.prune) {
      if (!over)
        for (int j = t; j < nocc; j += HP_NT) {
          const int s = LIST ? occ[j] : j;
          const int32_t X = keys[s];
          if (X >= 0 && X != c) heavier((int64_t)vals[s], X, hw, hX);
        }
      block_heaviest<HP_NT>(hw, hX);
    }
    const int64_t L = score_floor(a.K, lq, pk, hw, hX);
    if (!over) {
      for (int j = t; j < nocc; j += HP_NT) {
        const int s = LIST ? occ[j] : j;
        const int32_t X = keys[s];
        if (X < 0) continue;
        cands++;
        const int64_t wx = (int64_t)vals[s];
        if (X == c) {
          wc = wx;
        } else if (lq * wx >= L) {
          const int64_t sc = lq * wx - pk * a.K[X];
          if (better(sc, X, best_s, best_id)) {
            best_s = sc;
            best_id = X;
          }
        }
      }
    }
    cands = wave_sum(cands);
    __shared__ int64_t rc[HP_NT / WAVE];
    if (lane_id() == 0) rc[t / WAVE] = cands;
    block_best<HP_NT>(best_s, best_id, wc);
    if (t == 0) {
      int64_t tc = 0;
      for (int k = 0; k < HP_NT / WAVE; k++) tc += rc[k];
      part[pi] = SegBest{best_s, wc, tc, best_id, 0};
      overflows += over ? 1 : 0;
    }
    if (LIST) {  // leave the table clean for the next partition (block_best passed a barrier)
      for (int j = t; j < nocc; j += HP_NT) {
        keys[occ[j]] = -1;
        vals[occ[j]] = 0;
      }
      if (t == 0) occ_n = 0;
    }
  }
  if (t == 0 && overflows) atomic_add_i64(&a.ctr[(blockIdx.x % NSPREAD) * NCTR + 6], overflows);
}

// Chunk-parallel, as k_hp_gather, and counts the chunk's arcs per partition
// of its row (LDS histogram, one global atomic per touched partition).
__global__ __launch_bounds__(B7_NT) void k_hps_count(AggArgs a, const int64_t *__restrict__ tot,
                                                     const int64_t *__restrict__ cstart,
                                                     const int64_t *__restrict__ xoff,
                                                     const int64_t *__restrict__ pstart, int32_t *__restrict__ xs,
                                                     int64_t *__restrict__ pcnt) {
  __shared__ int32_t hist[HPS_MAXP];
  __shared__ int64_t sh_row;
  const int32_t *list;
  int64_t cnt7;
  work_of(a, list, cnt7);
  const int64_t nch = tot[0], n7 = tot[3];
  const int t = threadIdx.x;
  for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
    __syncthreads();  // hist and sh_row are reused
    if (t == 0) {
      int64_t lo = 0, hi = n7 - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (cstart[mid] <= ch) lo = mid;
        else hi = mid - 1;
      }
      sh_row = lo;
    }
    __syncthreads();
    const int64_t i = sh_row;
    const int32_t v = list[i];
    const int64_t beg = a.off[v], end = a.off[v + 1];
    const int64_t e0 = beg + (ch - cstart[i]) * B7_CHUNK;
    const int64_t e1 = e0 + B7_CHUNK < end ? e0 + B7_CHUNK : end;
    const uint32_t P = (uint32_t)(pstart[i + 1] - pstart[i]);
    for (uint32_t k = t; k < P; k += B7_NT) hist[k] = 0;
    __syncthreads();
    int32_t *out = xs + xoff[i] - beg;
    for (int64_t e = e0 + t; e < e1; e += B7_NT) {
      const int32_t X = a.C[a.col[e]];
      out[e] = X;
      atomicAdd(&hist[part_of(X, P)], 1);
    }
    __syncthreads();
    for (uint32_t k = t; k < P; k += B7_NT)
      if (hist[k]) atomic_add_i64(&pcnt[pstart[i] + k], hist[k]);
  }
}

// Chunk-parallel: reserves the chunk's range in each touched partition's
// segment (one global atomic per partition) and places its ids and weights
// there by LDS rank (the order inside a segment is immaterial: integer sums).
template <int WK>
__global__ __launch_bounds__(B7_NT) void k_hps_scatter(AggArgs a, const int64_t *__restrict__ tot,
                                                       const int64_t *__restrict__ cstart,
                                                       const int64_t *__restrict__ xoff,
                                                       const int64_t *__restrict__ pstart,
                                                       const int32_t *__restrict__ xs,
                                                       const int64_t *__restrict__ segstart,
                                                       int64_t *__restrict__ cursor, int32_t *__restrict__ ys,
                                                       int64_t *__restrict__ ws) {
  __shared__ int32_t hist[HPS_MAXP];
  __shared__ int64_t base[HPS_MAXP];
  __shared__ int64_t sh_row;
  const int32_t *list;
  int64_t cnt7;
  work_of(a, list, cnt7);
  const int64_t nch = tot[0], n7 = tot[3];
  const int t = threadIdx.x;
  for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
    __syncthreads();
    if (t == 0) {
      int64_t lo = 0, hi = n7 - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (cstart[mid] <= ch) lo = mid;
        else hi = mid - 1;
      }
      sh_row = lo;
    }
    __syncthreads();
    const int64_t i = sh_row;
    const int32_t v = list[i];
    const int64_t beg = a.off[v], end = a.off[v + 1];
    const int64_t e0 = beg + (ch - cstart[i]) * B7_CHUNK;
    const int64_t e1 = e0 + B7_CHUNK < end ? e0 + B7_CHUNK : end;
    const uint32_t P = (uint32_t)(pstart[i + 1] - pstart[i]);
    const int64_t p0 = pstart[i];
    const int32_t *x = xs + xoff[i] - beg;
    for (uint32_t k = t; k < P; k += B7_NT) hist[k] = 0;
    __syncthreads();
    for (int64_t e = e0 + t; e < e1; e += B7_NT) atomicAdd(&hist[part_of(x[e], P)], 1);
    __syncthreads();
    for (uint32_t k = t; k < P; k += B7_NT) {
      const int32_t h = hist[k];
      if (h) base[k] = segstart[p0 + k] + (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(&cursor[p0 + k]),
                                                             (unsigned long long)h);
      hist[k] = 0;
    }
    __syncthreads();
    for (int64_t e = e0 + t; e < e1; e += B7_NT) {
      const int32_t X = x[e];
      const uint32_t k = part_of(X, P);
      const int64_t at = base[k] + atomicAdd(&hist[k], 1);
      ys[at] = X;
      ws[at] = load_w<WK>(a.wt, e);
    }
  }
}

// keys, values, and (32-bit sums) the claimed-slot list of k_hp_part
size_t hp_lds_bytes(bool a32) { return (size_t)HP_SLOTS * (sizeof(int32_t) + (a32 ? 4 + 2 : 8)); }

// Hub rows in one pass.  A row's degree bounds its distinct clusters, but
// once clusters have formed a hub row meets far fewer clusters than it has
// arcs (on a contracted power-law graph, a sixth or less after the first
// iteration), so most hub rows fit one block's LDS table after all.  One
// block per row streams the row once into a table of H slots whose claims
// stop at `limit` keys: a row that stays within the limit is scored and
// decided here exactly as the per-row kernels do (done[i] = 1); a row that
// meets more clusters stops reading at once and is left to the hash
// partitions (done[i] = 0), which k_hp_layout and k_b7_final then take alone.
// hub_seen[v] keeps the number of distinct clusters v's row met when it was
// last decided (here, or summed over its partitions by k_hp_part); a row
// that met more than the limit then goes straight to the partitions instead
// of reading most of itself again before it overflows.  The count is a hint
// about speed only: either way the row is decided the same.
__device__ __forceinline__ bool lds_insert_upto(int32_t *keys, int32_t *vals32, int64_t *vals64, bool a32,
                                                uint32_t H, int32_t X, int64_t w, int32_t *nclaim,
                                                int32_t stop) {
  uint32_t h = slot_of(X, H);
  while (true) {
    int32_t cur = keys[h];
    if (cur == -1) {
      if (atomicAdd(nclaim, 1) >= stop) return false;
      cur = atomicCAS(&keys[h], -1, X);
      if (cur == -1) {
        cur = X;
      } else {
        atomicSub(nclaim, 1);  // another key took the slot first
      }
    }
    if (cur == X) {
      if (w) {
        if (a32)
          atomicAdd(&vals32[h], (int32_t)w);
        else
          atomicAdd(reinterpret_cast<unsigned long long *>(&vals64[h]), (unsigned long long)w);
      }
      return true;
    }
    h = (h + 1 == H) ? 0 : h + 1;
  }
}

constexpr int HR_NT = 1024;

template <int WK, bool A32>
__global__ __launch_bounds__(HR_NT) void k_hub_row(AggArgs a, uint8_t *__restrict__ done, int32_t limit) {
  using Acc = typename std::conditional<A32, int32_t, int64_t>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t H = (uint32_t)a.hcap;
  int32_t *keys = reinterpret_cast<int32_t *>(smem);
  Acc *vals = reinterpret_cast<Acc *>(smem + ((a.hcap * 4 + 15) & ~15ll));
  __shared__ int32_t nclaim, sh_d;
  const int t = threadIdx.x;
  const int32_t *list;
  int64_t n7;
  work_of(a, list, n7);
  // claims stop one block's worth of inserts below the table size, so a
  // probe always meets an empty slot and every insert ends
  const int32_t stop = (int32_t)H - HR_NT;
  int64_t movers = 0, marcs = 0, cands = 0, niso = 0;
  for (int64_t i = blockIdx.x; i < n7; i += gridDim.x) {
    const int32_t v = list[i];
    if (a.hub_seen && a.hub_seen[v] > limit) {  // uniform: one address
      __syncthreads();  // every thread has read the hint before it is cleared
      if (t == 0) {
        done[i] = 0;
        a.hub_seen[v] = 0;  // k_hp_part adds this time's count
      }
      continue;
    }
    const int64_t beg = a.off[v], end = a.off[v + 1];
    const int32_t c = a.C[v];
    const int64_t kv = a.k[v], Kc = a.K[c];
    const int32_t cntc = a.cnt[c];
    for (uint32_t j = t; j < H; j += HR_NT) {
      keys[j] = -1;
      vals[j] = 0;
    }
    if (t == 0) nclaim = 0;
    __syncthreads();
    if (t == 0)
      lds_insert_upto(keys, reinterpret_cast<int32_t *>(vals), reinterpret_cast<int64_t *>(vals), A32, H, c, 0,
                      &nclaim, stop);
    bool ok = true;
    for (int64_t base = beg + t; base < end && ok; base += 4 * HR_NT) {
      int32_t u[4], X[4];
      int64_t w[4];
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int64_t e = base + j * HR_NT;
        u[j] = e < end ? a.col[e] : -1;
        w[j] = e < end ? load_w<WK>(a.wt, e) : 0;
      }
#pragma unroll
      for (int j = 0; j < 4; j++) X[j] = u[j] >= 0 ? a.C[u[j]] : -1;
#pragma unroll
      for (int j = 0; j < 4; j++)
        if (X[j] >= 0)
          ok = lds_insert_upto(keys, reinterpret_cast<int32_t *>(vals), reinterpret_cast<int64_t *>(vals), A32, H,
                               X[j], w[j], &nclaim, stop) && ok;
      // another lane's overflow ends this lane's reading too (a stale read
      // of the counter only delays that)
      ok = ok && *(volatile int32_t *)&nclaim <= limit;
    }
    __syncthreads();
    const bool fits = nclaim <= limit;  // block-uniform
    if (!fits) {
      if (t == 0) {
        done[i] = 0;
        if (a.hub_seen) a.hub_seen[v] = 0;  // k_hp_part adds this time's count
      }
      __syncthreads();  // the table and nclaim are reused by the next row
      continue;
    }
    if (t == 0 && a.hub_seen) a.hub_seen[v] = nclaim;
    int64_t lp, lq;
    int32_t job;
    job_lambda(a, v, lp, lq, job);
    const int64_t pk = lp * kv;
    int64_t best_s = INT64_MIN, wc = 0;
    int32_t best_id = ISO_ID;
    int64_t hw = INT64_MIN;
    int32_t hX = INT32_MAX;
    if (a.prune) {
      for (uint32_t j = t; j < H; j += HR_NT) {
        const int32_t X = keys[j];
        if (X >= 0 && X != c) heavier((int64_t)vals[j], X, hw, hX);
      }
      block_heaviest<HR_NT>(hw, hX);
    }
    const int64_t L = score_floor(a.K, lq, pk, hw, hX);
    const int64_t stay0 = lq * own_weight(keys, vals, H, c) - pk * (Kc - kv);
    for (uint32_t j = t; j < H; j += HR_NT) {
      const int32_t X = keys[j];
      if (X < 0) continue;
      cands++;
      const int64_t wx = (int64_t)vals[j];
      if (X == c) {
        wc = wx;
      } else if (lq * wx >= L && lq * wx > stay0) {
        const int64_t sc = lq * wx - pk * a.K[X];
        if (better(sc, X, best_s, best_id)) {
          best_s = sc;
          best_id = X;
        }
      }
    }
    block_best<HR_NT>(best_s, best_id, wc);
    if (t == 0) {
      const int64_t stay = lq * wc - pk * (Kc - kv);
      const int32_t d = decide(best_s, best_id, stay, a.allow_iso && cntc >= 2, c);
      a.D[v] = d;
      done[i] = 1;
      sh_d = d;
      if (d != c) {
        movers += 1;
        marcs += end - beg;
        if (a.left_flag) a.left_flag[c] = 1;
        if (a.Cw) own_move(a, v, c, d, kv, niso);
      }
    }
    __syncthreads();
    if (sh_d != c && a.next_flag)
      for (int64_t e = beg + t; e < end; e += HR_NT) a.next_flag[a.col[e]] = 1;
    __syncthreads();  // the table, nclaim and sh_d are reused by the next row
  }
  if (t == 0 && niso) atomic_add_i64(a.iso_ctr, niso);
  flush_counters<HR_NT>(a.ctr, movers, cands, marcs);
}

// Table of the one-pass hub kernel: as many slots as the per-block LDS holds
// beside its reduction arrays; rows may fill three quarters of it.
int64_t hub_row_slots(const Ctx &c, bool a32) {
  const int64_t budget = (int64_t)c.lds_per_block - 4096;
  return (budget - 16) / (a32 ? 8 : 12);
}


// ------------------------------------------ neighbors-of-clusters frontier

// End of an iteration under the neighbors-of-clusters rule (Sec. 3.2.2):
// every vertex v whose cluster (at the end of the iteration, before fresh
// ids are renamed) is one that a vertex moved out of during the iteration
// marks its neighbors in `next`.  Lane i of a wave tests vertex base + i;
// the wave then walks the rows of the marked vertices one after another,
// coalesced.  The left flags alternate between two arrays: this launch
// reads `left` and clears `left_next`, which the next iteration's moves fill
// (the previous iteration's launch, the last reader of left_next, is done).
constexpr int LN_NT = 256;
__global__ __launch_bounds__(LN_NT) void k_mark_left_nbrs(const int64_t *__restrict__ off,
                                                          const int32_t *__restrict__ col,
                                                          const int32_t *__restrict__ C, int64_t n,
                                                          const uint8_t *__restrict__ left,
                                                          uint8_t *__restrict__ left_next, uint8_t *__restrict__ next) {
  const int lane = lane_id();
  const int64_t stride = (int64_t)gridDim.x * LN_NT;
  for (int64_t base = (int64_t)blockIdx.x * LN_NT + (threadIdx.x - lane); base < n; base += stride) {
    const int64_t v = base + lane;
    bool mark = false;
    if (v < n) {
      left_next[v] = 0;
      const int32_t x = C[v];
      mark = x < n && left[x];
    }
    uint64_t m = __ballot(mark);
    while (m) {
      const int i = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const int64_t u = base + i;
      const int64_t e1 = off[u + 1];
      for (int64_t e = off[u] + lane; e < e1; e += WAVE) next[col[e]] = 1;
    }
  }
}

// ------------------------------------- neighbors-of-movers frontier, pulled

// End of an iteration under the neighbors-of-movers rule on levels above the
// small-level size (Sec. 3.2.2): next[u] = 1 for every u adjacent to a vertex
// that moved during the iteration (moved[v] = 1, set by k_bm_apply).  The
// deciding kernels do not mark neighbors on these levels; this launch builds
// the set in one of two ways, chosen from the iteration's mover count (the
// launches' counters, so every block takes the same branch):
// * many movers (at least 1/FR_DENSE of the vertices): every vertex looks
//   through its own row for a neighbor that moved and stops at the first
//   (a lane per vertex for the first arcs, a group of lanes for the rest
//   of a row).  When most vertices move, nearly every row has a mover among its
//   first arcs, so this reads a few arcs per vertex instead of storing one
//   flag per arc of every mover;
// * few movers: one wave takes 64 vertices, lists the movers among them by
//   ballot and marks each mover's row with all 64 lanes (what the deciding
//   kernels would store, without their lane-group shapes).
// Both give the same set because the graph is symmetric: u is adjacent to v
// exactly when v is adjacent to u.  Movers of degree 2048 or more are not
// flagged: they marked their neighbors as they decided, so both ways only
// add to `next` (cleared by the compaction of the previous iteration).
constexpr int FR_NT = 256;
constexpr int FR_FIRST = 4;  // arcs a lane checks alone before a group takes the row
constexpr int FR_G = 8;      // lanes per group walking the rest of a row
constexpr int64_t FR_DENSE = 8;

__global__ __launch_bounds__(FR_NT) void k_frontier(const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                    int64_t n, const uint8_t *__restrict__ moved,
                                                    const int64_t *__restrict__ lctr, int32_t nlaunch,
                                                    uint8_t *__restrict__ next) {
  __shared__ int sh_pull;
  __shared__ int64_t sh_m[FR_NT / WAVE];
  {
    // movers: counter 0 of every copy of every launch, summed by the block
    int64_t m = 0;
    for (int64_t i = threadIdx.x; i < (int64_t)nlaunch * NSPREAD; i += FR_NT) m += lctr[i * NCTR];
    m = wave_sum(m);
    if (lane_id() == 0) sh_m[threadIdx.x / WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t tot = 0;
      for (int w = 0; w < FR_NT / WAVE; w++) tot += sh_m[w];
      sh_pull = tot * FR_DENSE >= n ? 1 : 0;
    }
    __syncthreads();
  }
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * FR_NT + threadIdx.x) / WAVE;
  const int64_t nw = (int64_t)gridDim.x * FR_NT / WAVE;
  if (sh_pull) {
    // a lane checks its own vertex's first FR_FIRST arcs; the rows that
    // have more and no moved neighbor among those are then walked by groups
    // of FR_G lanes, FR_G rows at a time, each until a moved neighbor shows
    const int gi = lane / FR_G, gl = lane % FR_G;
    const uint64_t gmask = ((1ull << FR_G) - 1) << (gi * FR_G);
    for (int64_t v0 = wid * WAVE; v0 < n; v0 += nw * WAVE) {
      const int64_t v = v0 + lane;
      int64_t beg = 0, end = 0;
      if (v < n) {
        beg = off[v];
        end = off[v + 1];
      }
      int32_t u[FR_FIRST];
#pragma unroll
      for (int r = 0; r < FR_FIRST; r++) u[r] = beg + r < end ? col[beg + r] : -1;
      uint32_t mv = 0;  // every gather issued before any is tested
#pragma unroll
      for (int r = 0; r < FR_FIRST; r++) mv |= u[r] >= 0 ? (uint32_t)moved[u[r]] : 0u;
      const bool found = mv != 0;
      if (found) next[v] = 1;
      uint64_t mk = __ballot(!found && end - beg > FR_FIRST);
      while (mk) {
        // group gi takes the gi-th lowest listed row, if there is one
        uint64_t m2 = mk;
        for (int k = 0; k < gi && m2; k++) m2 &= m2 - 1;
        const int j = m2 ? __ffsll((unsigned long long)m2) - 1 : 0;
        for (int k = 0; k < WAVE / FR_G && mk; k++) mk &= mk - 1;
        const int64_t bj = __shfl(beg, j, WAVE), ej = __shfl(end, j, WAVE);
        const int64_t b = m2 ? bj + FR_FIRST : 0, e1 = m2 ? ej : 0;
        bool hit = false;
        for (int64_t e0 = b; e0 < e1 && !hit; e0 += FR_G)  // group-uniform trips
          hit = (__ballot(e0 + gl < e1 && moved[col[e0 + gl]] != 0) & gmask) != 0;
        if (hit && gl == 0) next[v0 + j] = 1;
      }
    }
  } else {
    for (int64_t v0 = wid * WAVE; v0 < n; v0 += nw * WAVE) {
      const int64_t v = v0 + lane;
      uint64_t mk = __ballot(v < n && moved[v] != 0);
      while (mk) {
        const int j = __ffsll((unsigned long long)mk) - 1;
        mk &= mk - 1;
        const int64_t beg = off[v0 + j], end = off[v0 + j + 1];
        for (int64_t e = beg + lane; e < end; e += 4 * WAVE) {
          int32_t u[4];
#pragma unroll
          for (int r = 0; r < 4; r++) u[r] = e + r * WAVE < end ? col[e + r * WAVE] : -1;
#pragma unroll
          for (int r = 0; r < 4; r++)
            if (u[r] >= 0) next[u[r]] = 1;
        }
      }
    }
  }
}


// -------------------------------------------------------------- apply

// Applies the sub-round's decisions; an isolating vertex v takes the fresh
// id n + v.  With `moved`, every mover of degree below 2048 is also flagged
// there (the frontier of the iteration is then built from these flags by
// k_frontier; wider rows marked their neighbors when they decided).
//
// Batched runs (jid set) also flag the jobs that moved: the list keeps vertex
// order within each bin, so a block's movers mostly share a few consecutive
// jobs; their flags gather in LDS and leave as one plain store per job
// instead of one global atomic per mover on a handful of addresses.
__global__ __launch_bounds__(BM_NT) void k_bm_apply(const int32_t *__restrict__ list0, int64_t count0,
                                                    const int64_t *__restrict__ dstart, int32_t bfirst, int32_t blast,
                                                    const int32_t *__restrict__ D, int32_t *__restrict__ C,
                                                    int64_t *__restrict__ K, int32_t *__restrict__ cnt,
                                                    const int64_t *__restrict__ k, int64_t n,
                                                    int64_t *__restrict__ iso_ctr, const int32_t *__restrict__ jid,
                                                    int64_t *__restrict__ jmoved, uint8_t *__restrict__ moved,
                                                    const int64_t *__restrict__ off) {
  constexpr int JW = 64;  // jobs flagged in LDS per block
  __shared__ int32_t j0;
  __shared__ int32_t jflag[JW];
  const int32_t *list = list0;
  int64_t count = count0;
  if (dstart) {  // the sub-round's buckets are contiguous in the list
    list = list0 + dstart[bfirst];
    count = dstart[blast] - dstart[bfirst];
  }
  int64_t niso = 0;
  for (int64_t base = (int64_t)blockIdx.x * BM_NT; base < count; base += (int64_t)gridDim.x * BM_NT) {
    const int64_t i = base + threadIdx.x;
    if (jid) {
      if (threadIdx.x == 0) j0 = jid[list[base]];
      if (threadIdx.x < JW) jflag[threadIdx.x] = 0;
      __syncthreads();
    }
    if (i < count) {
      const int32_t v = list[i];
      int32_t d = D[v];
      const int32_t c = C[v];
      if (d != c && jid) {
        const int32_t j = jid[v];
        if (j >= j0 && j - j0 < JW) jflag[j - j0] = 1;
        else jmoved[j] = 1;
      }
      if (d != c) {
        const int64_t kv = k[v];
        if (moved && off[v + 1] - off[v] <= bin_limit_fixed(5)) moved[v] = 1;
        if (d < 0) {
          d = (int32_t)(n + v);
          niso++;
        }
        if (kv) {
          atomic_add_i64(&K[c], -kv);
          atomic_add_i64(&K[d], kv);
        }
        atomicSub(&cnt[c], 1);
        atomicAdd(&cnt[d], 1);
        C[v] = d;
      }
    }
    if (jid) {
      __syncthreads();
      if (threadIdx.x < JW && jflag[threadIdx.x]) jmoved[j0 + threadIdx.x] = 1;
      __syncthreads();
    }
  }
  niso = wave_sum(niso);
  if (lane_id() == 0 && niso) atomic_add_i64(iso_ctr, niso);
}

// ------------------------------------------------ renaming fresh clusters

// Renaming is needed only after an iteration with an isolating vertex;
// device-driven iterations queue it always and let it skip itself.
__device__ __forceinline__ bool no_isolation(const int64_t *isoc, int S) {
  if (!isoc) return false;
  int64_t t = 0;
  for (int s = 0; s < S; s++) t += isoc[s];
  return t == 0;
}

// fresh[t] = cluster n + t is non-empty; empty[x] = cluster x (< n) is empty.
__global__ void k_fresh_flags(const int32_t *__restrict__ cnt, int64_t n, uint8_t *__restrict__ fresh,
                              uint8_t *__restrict__ empty, const int64_t *__restrict__ isoc, int S) {
  if (no_isolation(isoc, S)) return;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    fresh[x] = cnt[n + x] > 0;
    empty[x] = cnt[x] == 0;
  }
}

// Ranks are taken per job (one job: the whole id range).  rank_f / rank_e
// are exclusive prefix counts with the total stored at index n.  The empty id
// of local rank r inside job j is stored at elist[rank_f[base_j] + r], the
// slot of the job's r-th fresh cluster, for r below the job's fresh count.
__global__ void k_empty_list(const uint8_t *__restrict__ empty, const int32_t *__restrict__ rank_e,
                             const int32_t *__restrict__ rank_f, int64_t n, JobView jv,
                             int32_t *__restrict__ elist, const int64_t *__restrict__ isoc, int S) {
  if (no_isolation(isoc, S)) return;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    if (!empty[x]) continue;
    int64_t b = 0, e = n;
    if (jv.jid) {
      const int32_t j = jv.jid[x];
      b = jv.jbase[j];
      e = jv.jbase[j + 1];
    }
    const int32_t r = rank_e[x] - rank_e[b];
    if (r < rank_f[e] - rank_f[b]) elist[rank_f[b] + r] = (int32_t)x;
  }
}

// The r-th non-empty fresh cluster takes the r-th empty id (totals moved).
__global__ void k_fresh_move(const uint8_t *__restrict__ fresh, const int32_t *__restrict__ rank_f,
                             const int32_t *__restrict__ elist, int64_t n, int64_t *__restrict__ K,
                             int32_t *__restrict__ cnt, int32_t *__restrict__ newid, int64_t *__restrict__ err,
                             const int64_t *__restrict__ isoc, int S) {
  if (no_isolation(isoc, S)) return;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    if (!fresh[t]) continue;
    const int32_t x = elist[rank_f[t]];
    // by counting there are enough empty ids; a violation is reported
    // instead of indexing out of range
    if (x < 0 || (int64_t)x >= n) {
      atomic_add_i64(err, 1);
      continue;
    }
    newid[t] = x;
    K[x] = K[n + t];
    cnt[x] = cnt[n + t];
    K[n + t] = 0;
    cnt[n + t] = 0;
  }
}

__global__ void k_fresh_relabel(int32_t *__restrict__ C, int64_t n, const int32_t *__restrict__ newid,
                                const int64_t *__restrict__ isoc, int S) {
  if (no_isolation(isoc, S)) return;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = C[v];
    if (c >= n) C[v] = newid[c - n];
  }
}

// The same renaming in one block for small n (one launch): exclusive ranks
// of fresh and empty ids tile by tile, then the pairing, the moves and the
// relabel, each phase behind a block barrier.
constexpr int RN_NT = 1024;
constexpr int64_t RN_SMALL = 16384;

// One block of RN_NT threads (the caller checks that someone isolated).
__device__ __forceinline__ void rename_small_body(int32_t *__restrict__ C, int64_t n, int64_t *__restrict__ K,
                                                  int32_t *__restrict__ cnt, int32_t *__restrict__ rank_f,
                                                  int32_t *__restrict__ rank_e, int32_t *__restrict__ elist,
                                                  int32_t *__restrict__ newid, const JobView &jv,
                                                  int64_t *__restrict__ err) {
  int32_t carry_f = 0, carry_e = 0;
  for (int64_t x0 = 0; x0 < n; x0 += RN_NT) {
    const int64_t x = x0 + threadIdx.x;
    const int32_t f = x < n && cnt[n + x] > 0, e = x < n && cnt[x] == 0;
    int32_t tf, te;
    const int32_t pf = block_excl_scan<int32_t, RN_NT>(f, &tf), pe = block_excl_scan<int32_t, RN_NT>(e, &te);
    if (x < n) {
      rank_f[x] = carry_f + pf;
      rank_e[x] = carry_e + pe;
    }
    carry_f += tf;
    carry_e += te;
  }
  if (threadIdx.x == 0) {
    rank_f[n] = carry_f;
    rank_e[n] = carry_e;
  }
  __syncthreads();
  for (int64_t x = threadIdx.x; x < n; x += RN_NT) {
    if (cnt[x] != 0) continue;
    int64_t b = 0, e = n;
    if (jv.jid) {
      const int32_t j = jv.jid[x];
      b = jv.jbase[j];
      e = jv.jbase[j + 1];
    }
    const int32_t r = rank_e[x] - rank_e[b];
    if (r < rank_f[e] - rank_f[b]) elist[rank_f[b] + r] = (int32_t)x;
  }
  __syncthreads();
  for (int64_t t = threadIdx.x; t < n; t += RN_NT) {
    if (cnt[n + t] <= 0) continue;
    const int32_t x = elist[rank_f[t]];
    if (x < 0 || (int64_t)x >= n) {
      atomic_add_i64(err, 1);
      continue;
    }
    newid[t] = x;
    K[x] = K[n + t];
    cnt[x] = cnt[n + t];
    K[n + t] = 0;
    cnt[n + t] = 0;
  }
  __syncthreads();
  for (int64_t v = threadIdx.x; v < n; v += RN_NT) {
    const int32_t c = C[v];
    if (c >= n) C[v] = newid[c - n];
  }
}

__global__ __launch_bounds__(RN_NT) void k_rename_small(int32_t *__restrict__ C, int64_t n, int64_t *__restrict__ K,
                                                        int32_t *__restrict__ cnt, int32_t *__restrict__ rank_f,
                                                        int32_t *__restrict__ rank_e, int32_t *__restrict__ elist,
                                                        int32_t *__restrict__ newid, JobView jv,
                                                        int64_t *__restrict__ err, const int64_t *__restrict__ isoc,
                                                        int S) {
  if (no_isolation(isoc, S)) return;
  rename_small_body(C, n, K, cnt, rank_f, rank_e, elist, newid, jv, err);
}

// Per-job termination of a device-driven iteration: a running job counts the
// iteration and stops when none of its vertices moved.
__global__ void k_job_update(uint8_t *__restrict__ jrun, int64_t *__restrict__ jmoved, int32_t *__restrict__ iters,
                             uint8_t *__restrict__ moved_any, int64_t jobs) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < jobs; j += (int64_t)gridDim.x * blockDim.x) {
    if (jrun[j]) {
      iters[j]++;
      if (jmoved[j]) moved_any[j] = 1;
      else jrun[j] = 0;
    }
    jmoved[j] = 0;
  }
}

// Vertices and arcs per degree bin (upper bounds of every bucket of a
// Best-Moves call): hist[b], hist[NBINS + b].
__global__ __launch_bounds__(BM_NT) void k_bin_hist(const int64_t *__restrict__ off, int64_t n, int64_t wide_max,
                                                    int64_t *__restrict__ hist) {
  __shared__ int64_t lh[2 * NBINS];
  if (threadIdx.x < 2 * NBINS) lh[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t v = (int64_t)blockIdx.x * BM_NT + threadIdx.x; v < n; v += (int64_t)gridDim.x * BM_NT) {
    const int64_t d = off[v + 1] - off[v];
    const int b = bin_of(d, wide_max);
    atomicAdd(reinterpret_cast<unsigned long long *>(&lh[b]), 1ull);
    if (d) atomicAdd(reinterpret_cast<unsigned long long *>(&lh[NBINS + b]), (unsigned long long)d);
  }
  __syncthreads();
  if (threadIdx.x < 2 * NBINS && lh[threadIdx.x]) atomic_add_i64(&hist[threadIdx.x], lh[threadIdx.x]);
}

// --- partition of the active vertices into (sub-round, bin) buckets

// Vertices of stopped jobs get bucket NOBUCKET and are left out.
constexpr uint16_t NOBUCKET = 0xFFFF;

// Each block owns one contiguous range of the active list; a bucket holds the
// ranges' members in range order, so a launch walks the vertex ids roughly in
// ascending order (cluster ids of one job stay together in L2).
__device__ __forceinline__ int64_t active_count(int64_t na, const int64_t *na_dev) { return na_dev ? *na_dev : na; }

__device__ __forceinline__ void part_range(int64_t na, int64_t &beg, int64_t &end) {
  const int64_t per = cdiv(na, (int64_t)gridDim.x);
  beg = (int64_t)blockIdx.x * per;
  end = beg + per < na ? beg + per : na;
}

// Per block and bucket: members (blkcnt[b * grid + block]); per bucket: total
// members and arcs.
__global__ __launch_bounds__(BM_NT) void k_part_count(const int32_t *__restrict__ list, int64_t na0,
                                                      const int64_t *__restrict__ na_dev,
                                                      const int64_t *__restrict__ off, uint64_t h, int32_t S,
                                                      int64_t wide_max, JobView jv, uint16_t *__restrict__ bucket_of,
                                                      int32_t *__restrict__ blkcnt, int64_t *__restrict__ bcnt,
                                                      int64_t *__restrict__ barcs) {
  extern __shared__ int64_t sm[];
  const int NB = S * NBINS;
  int64_t *lc = sm;
  int64_t *la = sm + NB;
  for (int i = threadIdx.x; i < 2 * NB; i += BM_NT) sm[i] = 0;
  __syncthreads();
  const int64_t na = active_count(na0, na_dev);
  int64_t beg, end;
  part_range(na, beg, end);
  for (int64_t i = beg + threadIdx.x; i < end; i += BM_NT) {
    const int32_t v = list ? list[i] : (int32_t)i;
    int64_t local = v;
    if (jv.jid) {
      const int32_t j = jv.jid[v];
      if (!jv.jrun[j]) {
        bucket_of[i] = NOBUCKET;
        continue;
      }
      local = v - jv.jbase[j];
    }
    const int64_t deg = off[v + 1] - off[v];
    const int s = (int)(mix64(h ^ (uint64_t)local) % (uint64_t)S);
    const int b = s * NBINS + bin_of(deg, wide_max);
    bucket_of[i] = (uint16_t)b;
    atomicAdd(reinterpret_cast<unsigned long long *>(&lc[b]), 1ull);
    if (deg) atomicAdd(reinterpret_cast<unsigned long long *>(&la[b]), (unsigned long long)deg);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NB; i += BM_NT) {
    blkcnt[(int64_t)i * gridDim.x + blockIdx.x] = (int32_t)lc[i];
    if (lc[i]) atomic_add_i64(&bcnt[i], lc[i]);
    if (la[i]) atomic_add_i64(&barcs[i], la[i]);
  }
}

// Stable placement of one tile of NT consecutive items into NB buckets (b
// = NOBUCKET: not placed): returns run[b] plus the item's rank among the
// tile's earlier items of bucket b (-1 when not placed), then advances run[b]
// by the tile's count.  Ranks inside a wave come from ballots over the bits
// of b, waves are taken in order, so buckets keep the items' order and the
// partition is the same on every run.  wcnt (LDS, NT / WAVE x NB int32) is
// zero on entry and on exit.  Every thread of the block calls it.
template <int NT>
__device__ __forceinline__ int64_t tile_stable_pos(int b, int NB, int32_t *wcnt, int64_t *run) {
  constexpr int NW = NT / WAVE;
  const int w = threadIdx.x / WAVE;
  const bool valid = b != NOBUCKET;
  int bits = 1;
  while ((1 << bits) < NB) bits++;
  uint64_t peers = __ballot(valid);
  for (int k = 0; k < bits; k++) {
    const uint64_t bb = __ballot((b >> k) & 1);
    peers &= ((b >> k) & 1) ? bb : ~bb;
  }
  const int rank = __popcll(peers & __lanemask_lt());
  const int cntp = __popcll(peers);
  if (valid && rank == cntp - 1) wcnt[w * NB + b] = cntp;
  __syncthreads();
  int64_t pos = -1;
  if (valid) {
    pos = run[b] + rank;
    for (int q = 0; q < w; q++) pos += wcnt[q * NB + b];
  }
  __syncthreads();
  for (int x = threadIdx.x; x < NB; x += NT) {
    int32_t t = 0;
#pragma unroll
    for (int q = 0; q < NW; q++) {
      t += wcnt[q * NB + x];
      wcnt[q * NB + x] = 0;
    }
    run[x] += t;
  }
  __syncthreads();
  return pos;
}

// LDS of the stable placement: NB running positions and NT / WAVE x NB counts.
__host__ __device__ constexpr size_t stable_lds_bytes(int NB, int NT) {
  return (size_t)NB * sizeof(int64_t) + (size_t)(NT / WAVE) * NB * sizeof(int32_t);
}

// The partition of a small level in one block and one launch: bucket counts
// and arcs, bucket starts (NB + 1) and the bucket lists.
constexpr int PS_NT = 1024;
constexpr int64_t SMALL_LEVEL = LCC_SMALL_LEVEL_MAX;

// One block of PS_NT threads; sm holds 2 * NB int64 then the placement counts
// (part_small_lds_bytes).
__host__ __device__ constexpr size_t part_small_lds_bytes(int NB) {
  return (size_t)NB * sizeof(int64_t) + stable_lds_bytes(NB, PS_NT);
}
__device__ __forceinline__ void part_small_body(const int32_t *__restrict__ list, int64_t na0,
                                                const int64_t *__restrict__ na_dev, const int64_t *__restrict__ off,
                                                uint64_t h, int32_t S, int64_t wide_max, const JobView &jv,
                                                uint16_t *__restrict__ bucket_of, int64_t *__restrict__ bcnt,
                                                int64_t *__restrict__ barcs, int64_t *__restrict__ dstart,
                                                int32_t *__restrict__ out, int64_t *sm) {
  const int NB = S * NBINS;
  int64_t *lc = sm;       // members, then cursor
  int64_t *la = sm + NB;  // arcs
  int32_t *wcnt = reinterpret_cast<int32_t *>(sm + 2 * NB);
  for (int i = threadIdx.x; i < 2 * NB; i += PS_NT) sm[i] = 0;
  for (int i = threadIdx.x; i < (PS_NT / WAVE) * NB; i += PS_NT) wcnt[i] = 0;
  __syncthreads();
  const int64_t na = active_count(na0, na_dev);
  for (int64_t i = threadIdx.x; i < na; i += PS_NT) {
    const int32_t v = list ? list[i] : (int32_t)i;
    int64_t local = v;
    if (jv.jid) {
      const int32_t j = jv.jid[v];
      if (!jv.jrun[j]) {
        bucket_of[i] = NOBUCKET;
        continue;
      }
      local = v - jv.jbase[j];
    }
    const int64_t deg = off[v + 1] - off[v];
    const int sr = (int)(mix64(h ^ (uint64_t)local) % (uint64_t)S);
    const int b = sr * NBINS + bin_of(deg, wide_max);
    bucket_of[i] = (uint16_t)b;
    atomicAdd(reinterpret_cast<unsigned long long *>(&lc[b]), 1ull);
    if (deg) atomicAdd(reinterpret_cast<unsigned long long *>(&la[b]), (unsigned long long)deg);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int b = 0; b < NB; b++) {
      bcnt[b] = lc[b];
      barcs[b] = la[b];
      dstart[b] = t;
      const int64_t cb = lc[b];
      lc[b] = t;  // becomes the cursor
      t += cb;
    }
    dstart[NB] = t;
  }
  __syncthreads();
  for (int64_t x0 = 0; x0 < na; x0 += PS_NT) {
    const int64_t i = x0 + threadIdx.x;
    const int b = i < na ? (int)bucket_of[i] : (int)NOBUCKET;
    const int64_t pos = tile_stable_pos<PS_NT>(b, NB, wcnt, lc);
    if (pos >= 0) out[pos] = list ? list[i] : (int32_t)i;
  }
}

__global__ __launch_bounds__(PS_NT) void k_part_small(const int32_t *__restrict__ list, int64_t na0,
                                                      const int64_t *__restrict__ na_dev,
                                                      const int64_t *__restrict__ off, uint64_t h, int32_t S,
                                                      int64_t wide_max, JobView jv, uint16_t *__restrict__ bucket_of,
                                                      int64_t *__restrict__ bcnt, int64_t *__restrict__ barcs,
                                                      int64_t *__restrict__ dstart, int32_t *__restrict__ out) {
  extern __shared__ int64_t sm[];
  part_small_body(list, na0, na_dev, off, h, S, wide_max, jv, bucket_of, bcnt, barcs, dstart, out, sm);
}

// The second copy of a small level's state: C2 = C (n), K2 = K, cnt2 = cnt
// (2n: regular then fresh ids).
__global__ void k_copy_state(const int32_t *__restrict__ C, const int64_t *__restrict__ K,
                             const int32_t *__restrict__ cnt, int64_t n, int32_t *__restrict__ C2,
                             int64_t *__restrict__ K2, int32_t *__restrict__ cnt2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) C2[i] = C[i];
  if (i < 2 * n) {
    K2[i] = K[i];
    cnt2[i] = cnt[i];
  }
}

// The end of a small level's iteration in one block: the next frontier
// (compaction of the flags), the renaming of fresh clusters (when someone
// isolated), per-job termination in batches, then the partition of the next
// iteration (when there is one) into that iteration's counter block.
struct IterEndSmall {
  // the copy of (C, K, cnt) that missed the last sub-round's moves (its
  // buckets rb0 .. rb1-1 of blist, decisions in D), brought up to date
  const int32_t *D;
  const int64_t *k;
  const int64_t *dstart_cur;
  int32_t rb0, rb1;
  int32_t *Cl;
  int64_t *Kl;
  int32_t *cntl;
  // the second copy, renamed like the first
  int32_t *C2;
  int64_t *K2;
  int32_t *cnt2;
  // frontier
  uint8_t *next;
  int32_t *active;
  int64_t *nact;
  int32_t compact;
  // renaming
  int32_t *C;
  int64_t *K;
  int32_t *cnt;
  int32_t *rank_f, *rank_e, *elist, *newid;
  int64_t *err;
  const int64_t *isoc;
  // batches
  int32_t *jiters;
  uint8_t *jmoved_any;
  int64_t jobs;
  // next partition
  int32_t part;
  const int64_t *off;
  uint64_t h_next;
  int64_t wide_max;
  uint16_t *bucket_of;
  int64_t *bcnt, *barcs, *dstart;
  int32_t *blist;
};

__global__ __launch_bounds__(PS_NT) void k_iter_end_small(IterEndSmall e, int64_t n, int32_t S, JobView jv) {
  extern __shared__ int64_t sm[];
  if (e.Cl) {
    const int64_t lo = e.dstart_cur[e.rb0], hi = e.dstart_cur[e.rb1];
    for (int64_t i = lo + threadIdx.x; i < hi; i += PS_NT) {
      const int32_t v = e.blist[i];
      const int32_t d = e.D[v], c = e.Cl[v];
      if (d == c) continue;
      const int32_t t = d < 0 ? (int32_t)(n + v) : d;
      const int64_t kv = e.k[v];
      if (kv) {
        atomic_add_i64(&e.Kl[c], -kv);
        atomic_add_i64(&e.Kl[t], kv);
      }
      atomicSub(&e.cntl[c], 1);
      atomicAdd(&e.cntl[t], 1);
      e.Cl[v] = t;
    }
  }
  if (e.compact) compact_small_body(e.next, n, e.active, e.nact, 1);
  if (!no_isolation(e.isoc, S)) {
    __syncthreads();  // both copies are equal
    rename_small_body(e.C, n, e.K, e.cnt, e.rank_f, e.rank_e, e.elist, e.newid, jv, e.err);
    if (e.C2) {
      __syncthreads();  // the rank arrays are reused
      rename_small_body(e.C2, n, e.K2, e.cnt2, e.rank_f, e.rank_e, e.elist, e.newid, jv, e.err);
    }
  }
  if (e.jobs > 0) {
    uint8_t *jrun = const_cast<uint8_t *>(jv.jrun);
    for (int64_t j = threadIdx.x; j < e.jobs; j += PS_NT) {
      if (jrun[j]) {
        e.jiters[j]++;
        if (jv.jmoved[j]) e.jmoved_any[j] = 1;
        else jrun[j] = 0;
      }
      jv.jmoved[j] = 0;
    }
  }
  if (e.part) {
    __syncthreads();  // the active list, its count and the running flags are complete
    part_small_body(e.compact ? e.active : nullptr, n, e.compact ? e.nact : nullptr, e.off, e.h_next, S, e.wide_max,
                    jv, e.bucket_of, e.bcnt, e.barcs, e.dstart, e.blist, sm);
  }
}

// One block per bucket b: cursor[b * nblk + k] = start of bucket b + members
// of b in the ranges of blocks < k.
__global__ __launch_bounds__(BM_NT) void k_part_offsets(const int64_t *__restrict__ bcnt,
                                                        const int32_t *__restrict__ blkcnt, int64_t nblk,
                                                        int64_t *__restrict__ cursor, int64_t *__restrict__ dstart) {
  const int b = blockIdx.x;
  __shared__ int64_t base;
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int i = 0; i < b; i++) t += bcnt[i];
    base = t;
    // bucket starts for device-driven launches (NB + 1 entries)
    dstart[b] = t;
    if (b == (int)gridDim.x - 1) dstart[b + 1] = t + bcnt[b];
  }
  __syncthreads();
  int64_t carry = base;
  const int32_t *row = blkcnt + (int64_t)b * nblk;
  int64_t *out = cursor + (int64_t)b * nblk;
  for (int64_t k0 = 0; k0 < nblk; k0 += BM_NT) {
    const int64_t k = k0 + threadIdx.x;
    const int64_t x = k < nblk ? row[k] : 0;
    int64_t tot;
    const int64_t ex = block_excl_scan<int64_t, BM_NT>(x, &tot);
    if (k < nblk) out[k] = carry + ex;
    carry += tot;
  }
}

// Stable: a bucket lists its members in the order of the active list (no
// result depends on the order, but it makes the assignment of vertices to
// the blocks of the aggregation launches the same on every run).
__global__ __launch_bounds__(BM_NT) void k_part_scatter(const int32_t *__restrict__ list, int64_t na0,
                                                        const int64_t *__restrict__ na_dev,
                                                        const uint16_t *__restrict__ bucket_of, int32_t S,
                                                        const int64_t *__restrict__ cursor,
                                                        int32_t *__restrict__ out) {
  extern __shared__ int64_t sm[];
  const int NB = S * NBINS;
  int64_t *run = sm;  // next position per bucket
  int32_t *wcnt = reinterpret_cast<int32_t *>(sm + NB);
  for (int i = threadIdx.x; i < NB; i += BM_NT) run[i] = cursor[(int64_t)i * gridDim.x + blockIdx.x];
  for (int i = threadIdx.x; i < (BM_NT / WAVE) * NB; i += BM_NT) wcnt[i] = 0;
  __syncthreads();
  const int64_t na = active_count(na0, na_dev);
  int64_t beg, end;
  part_range(na, beg, end);
  for (int64_t i0 = beg; i0 < end; i0 += BM_NT) {
    const int64_t i = i0 + threadIdx.x;
    const int b = i < end ? (int)bucket_of[i] : (int)NOBUCKET;
    const int64_t pos = tile_stable_pos<BM_NT>(b, NB, wcnt, run);
    if (pos >= 0) out[pos] = list ? list[i] : (int32_t)i;
  }
}

// Orders each sub-round's hub bucket (rows wider than the degree-sized LDS
// bins) by decreasing degree, ties by list position.  The hub kernels give
// one block per row and blocks start in index order, so the longest rows now
// start first instead of ending the launch on one long row started last.
// Only the order of the list changes: every row is decided the same.  A
// bucket of at most `spread` rows (they all start at once) or more than
// HO_MAX rows keeps its order.  One block per sub-round.
constexpr int HO_NT = 1024;
constexpr int HO_MAX = 4096;
static_assert(HO_MAX == 1 << 12, "the sort key keeps the list position in its low 12 bits");
__global__ __launch_bounds__(HO_NT) void k_hub_order(const int64_t *__restrict__ dstart,
                                                     const int64_t *__restrict__ off, int64_t spread,
                                                     int32_t *__restrict__ blist) {
  __shared__ uint64_t key[HO_MAX];
  __shared__ int32_t vid[HO_MAX];
  const int t = threadIdx.x;
  const int b = blockIdx.x * NBINS + NBINS - 1;
  const int64_t beg = dstart[b], m = dstart[b + 1] - beg;
  if (m <= spread || m > HO_MAX) return;  // uniform
  int P = 1;
  while (P < m) P <<= 1;
  for (int i = t; i < P; i += HO_NT) {
    if (i < m) {
      const int32_t v = blist[beg + i];
      const int64_t deg = off[v + 1] - off[v];
      const int64_t d = deg < INT32_MAX ? deg : INT32_MAX;
      key[i] = ((uint64_t)(INT32_MAX - d) << 12) | (uint64_t)i;  // below 2^43, padding sorts last
      vid[i] = v;
    } else {
      key[i] = ~0ull;
    }
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = t; i < P; i += HO_NT) {
        const int x = i ^ j;
        if (x > i) {
          const uint64_t a = key[i], c = key[x];
          if ((a > c) == ((i & k) == 0)) {
            key[i] = c;
            key[x] = a;
          }
        }
      }
      __syncthreads();
    }
  for (int i = t; i < m; i += HO_NT) blist[beg + i] = vid[key[i] & (HO_MAX - 1)];
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
  size_t pending_idx;  // index into ctx.pending when timed
  int slot;
};

// Dynamic LDS for the wide kernels: keys (int32), 16-byte aligned values,
// then (list) the occupied-slot list (uint16, one entry per slot).
size_t wide_lds_bytes(int64_t slots, bool a32, bool list = true) {
  return (size_t)((slots * 4 + 15) & ~15ll) + (size_t)slots * (a32 ? 4 : 8) + (list ? (size_t)slots * 2 : 0);
}

// Largest table (slots) that fits the per-block LDS beside the kernel's own
// reduction arrays.
int64_t wide_slots(const Ctx &c, bool a32) {
  const int64_t budget = (int64_t)c.lds_per_block - 4096;
  const int64_t slots = (budget - 16) / (a32 ? 10 : 14);
  return slots < 65536 ? slots : 65535;  // occupied-slot indices are uint16
}

// Raises a kernel's dynamic-LDS limit once per context.
template <class F> void allow_lds(Ctx &c, F kernel, size_t bytes) {
  const void *f = reinterpret_cast<const void *>(kernel);
  for (const void *x : c.lds_raised)
    if (x == f) return;
  HIPCHECK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  c.lds_raised.push_back(f);
}

// Vertices one block of a bin's kernel handles at a time.
int bin_vpb(int bin) {
  static const int group[NBINS] = {BM_NT / 8, BM_NT / 16, BM_NT / 32, BM_NT / 64, BM_NT / 64, 1, 1, 1};
  return group[bin];
}

// Grid of a bin launch: one pass when the count is known, else a resident
// grid that loops over the bucket (device-driven launches).
int64_t bin_grid(const Ctx &c, int bin, int64_t count, bool exact) {
  const int64_t need = std::max<int64_t>(1, cdiv(count, bin_vpb(bin)));
  if (exact) return need;
  const int64_t cap = (int64_t)c.num_cu * (bin < 5 ? 8 : bin == 5 ? 4 : 2);
  return std::min(need, cap);
}

template <int WK, bool A32>
void launch_bin(Ctx &c, int bin, AggArgs a, int64_t grid) {
  const dim3 gr((unsigned)grid);
  switch (bin) {
    case 0: c.launch(k_bm_group<8, 16, WK, A32>, gr, dim3(BM_NT), 0, a); break;
    case 1: c.launch(k_bm_group<16, 32, WK, A32>, gr, dim3(BM_NT), 0, a); break;
    case 2: c.launch(k_bm_group<32, 64, WK, A32>, gr, dim3(BM_NT), 0, a); break;
    case 3: c.launch(k_bm_group<64, 128, WK, A32>, gr, dim3(BM_NT), 0, a); break;
    case 4: c.launch(k_bm_group<64, 512, WK, A32>, gr, dim3(BM_NT), 0, a); break;
    case 5: {  // without the slot list: 48 KB of LDS keeps 3 blocks per CU
      a.hcap = MID_SLOTS;
      const size_t bytes = wide_lds_bytes(MID_SLOTS, A32, false);
      c.launch(k_bm_wide<BM_NT, WK, A32, 0, false>, gr, dim3(BM_NT), bytes, a);
      break;
    }
    case 6: {
      a.hcap = wide_slots(c, A32);
      const size_t bytes = wide_lds_bytes(a.hcap, A32);
      allow_lds(c, k_bm_wide<WIDE_NT, WK, A32>, bytes);
      c.launch(k_bm_wide<WIDE_NT, WK, A32>, gr, dim3(WIDE_NT), bytes, a);
      break;
    }
    default:
      fail(LCC_ERR_DEVICE, "internal: the flat bin is launched by launch_flat_pk");
  }
  LAUNCHCHECK();
}

// Singleton first iteration: lanes per vertex follow the degree bin.
template <int WK> void launch_single(Ctx &c, int bin, AggArgs a, int64_t grid) {
  const dim3 gr((unsigned)grid);
  switch (bin) {
    case 0: c.launch(k_bm_single<8, BM_NT, WK>, gr, dim3(BM_NT), 0, a); break;
    case 1: c.launch(k_bm_single<16, BM_NT, WK>, gr, dim3(BM_NT), 0, a); break;
    case 2: c.launch(k_bm_single<32, BM_NT, WK>, gr, dim3(BM_NT), 0, a); break;
    case 3:
    case 4: c.launch(k_bm_single<64, BM_NT, WK>, gr, dim3(BM_NT), 0, a); break;
    case 5: c.launch(k_bm_single<BM_NT, BM_NT, WK>, gr, dim3(BM_NT), 0, a); break;
    default: c.launch(k_bm_single<WIDE_NT, WIDE_NT, WK>, gr, dim3(WIDE_NT), 0, a);
  }
  LAUNCHCHECK();
}

// Flat aggregation of the rows of bin 7 (see k_b7_insert).  Sizes are upper
// bounds (at most n7_ub rows holding at most a7_ub arcs); the kernels read
// the actual ones from the layout, so nothing is read back.
template <int WK, bool PK> void launch_flat_pk(Ctx &c, AggArgs a, int64_t n7_ub, int64_t a7_ub) {
  n7_ub = std::max<int64_t>(n7_ub, 1);
  int64_t *cstart = c.buf<int64_t>("b7.cstart", (size_t)n7_ub + 1);
  int64_t *tstart = c.buf<int64_t>("b7.tstart", (size_t)n7_ub + 1);
  int64_t *sstart = c.buf<int64_t>("b7.sstart", (size_t)n7_ub + 1);
  int64_t *tot = c.buf<int64_t>("b7.tot", 4);
  // capacities: pow2 >= 2(deg + 1) <= 4(deg + 1)
  const size_t slots = (size_t)(4 * (a7_ub + n7_ub));
  a.gkeys = c.buf<int32_t>("b7.keys", slots);
  a.gvals = c.buf<int64_t>("b7.vals", slots);
  const int64_t max_seg = (int64_t)slots / B7_SEG + n7_ub;
  SegBest *part = c.buf<SegBest>("b7.part", (size_t)max_seg);
  hipLaunchKernelGGL(k_b7_layout, dim3(1), dim3(B7L_NT), 0, c.stream, a, cstart, tstart, sstart, tot);
  LAUNCHCHECK();
  hipLaunchKernelGGL(k_b7_clear<PK>, dim3((unsigned)c.num_cu * 8), dim3(256), 0, c.stream, a.gkeys, a.gvals, tot);
  LAUNCHCHECK();
  // chunks: at most a7_ub / B7_CHUNK + n7_ub
  const int64_t chunks = a7_ub / B7_CHUNK + n7_ub;
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(chunks, (int64_t)c.num_cu * 4));
  hipLaunchKernelGGL((k_b7_insert<WK, PK>), dim3((unsigned)grid), dim3(B7_NT), 0, c.stream, a, tot, cstart, tstart);
  LAUNCHCHECK();
  hipLaunchKernelGGL(k_b7_segscore<PK>, dim3((unsigned)std::min<int64_t>(max_seg, (int64_t)c.num_cu * 8)), dim3(B7_NT), 0,
                     c.stream, a, tot, tstart, sstart, part);
  LAUNCHCHECK();
  hipLaunchKernelGGL(k_b7_final, dim3((unsigned)std::min<int64_t>(n7_ub, (int64_t)c.num_cu * 4)), dim3(B7_NT), 0,
                     c.stream, a, sstart, part, (const uint8_t *)nullptr);
  LAUNCHCHECK();
}

// Rows beyond the LDS tables through hash partitions in LDS (see k_hp_part),
// reading whole rows or (c.hub_scatter) their ids scattered by partition.
template <int WK> void launch_hub_part(Ctx &c, AggArgs a, int64_t n7_ub, int64_t a7_ub, bool a32) {
  n7_ub = std::max<int64_t>(n7_ub, 1);
  const int64_t a7 = std::max<int64_t>(a7_ub, 1);
  int64_t *cstart = c.buf<int64_t>("hp.cstart", (size_t)n7_ub + 1);
  int64_t *xoff = c.buf<int64_t>("hp.xoff", (size_t)n7_ub + 1);
  int64_t *pstart = c.buf<int64_t>("hp.pstart", (size_t)n7_ub + 1);
  int64_t *tot = c.buf<int64_t>("hp.tot", 4);
  int32_t *xs = c.buf<int32_t>("hp.xs", (size_t)a7);
  // partitions: at most cdiv(2 (d + 1), HP_LIMIT) <= 2 (d + 1) / HP_LIMIT + 1 per row
  const int64_t parts_ub = 2 * (a7_ub + n7_ub) / HP_LIMIT + n7_ub + 1;
  SegBest *part = c.buf<SegBest>("hp.part", (size_t)parts_ub);
  // first every row in one pass where its clusters fit one block's table
  uint8_t *done = c.buf<uint8_t>("hp.done", (size_t)n7_ub);
  if (a.hub_row_limit < 0) {  // every row takes the partitions
    HIPCHECK(hipMemsetAsync(done, 0, (size_t)n7_ub, c.stream));
    a.hub_seen = nullptr;
  } else {
    AggArgs ah = a;
    ah.hcap = hub_row_slots(c, a32);
    int32_t limit = (int32_t)(ah.hcap * 3 / 4);
    if (a.hub_row_limit > 0 && a.hub_row_limit < limit) limit = a.hub_row_limit;
    const size_t bytes = wide_lds_bytes(ah.hcap, a32, false);
    const dim3 gh((unsigned)std::min<int64_t>(n7_ub, (int64_t)1 << 20));
    if (a32) {
      allow_lds(c, k_hub_row<WK, true>, bytes);
      hipLaunchKernelGGL((k_hub_row<WK, true>), gh, dim3(HR_NT), bytes, c.stream, ah, done, limit);
    } else {
      allow_lds(c, k_hub_row<WK, false>, bytes);
      hipLaunchKernelGGL((k_hub_row<WK, false>), gh, dim3(HR_NT), bytes, c.stream, ah, done, limit);
    }
    LAUNCHCHECK();
  }
  hipLaunchKernelGGL(k_hp_layout, dim3(1), dim3(B7L_NT), 0, c.stream, a, cstart, xoff, pstart, tot,
                     (const uint8_t *)done);
  LAUNCHCHECK();
  const int64_t chunks = a7_ub / B7_CHUNK + n7_ub;
  const dim3 gc((unsigned)std::max<int64_t>(1, std::min<int64_t>(chunks, (int64_t)c.num_cu * 8)));
  const bool seg = c.hub_scatter;
  int64_t *pcnt = nullptr, *segstart = nullptr, *ws = nullptr;
  int32_t *ys = xs;
  if (!seg) {
    hipLaunchKernelGGL(k_hp_gather, gc, dim3(B7_NT), 0, c.stream, a, (const int64_t *)tot, (const int64_t *)cstart,
                       (const int64_t *)xoff, xs);
    LAUNCHCHECK();
  } else {
    pcnt = c.buf<int64_t>("hps.cnt", (size_t)parts_ub);
    int64_t *cursor = c.buf<int64_t>("hps.cur", (size_t)parts_ub);
    segstart = c.buf<int64_t>("hps.seg", (size_t)parts_ub);
    ys = c.buf<int32_t>("hps.ys", (size_t)a7);
    ws = c.buf<int64_t>("hps.ws", (size_t)a7);
    HIPCHECK(hipMemsetAsync(pcnt, 0, (size_t)parts_ub * sizeof(int64_t), c.stream));
    HIPCHECK(hipMemsetAsync(cursor, 0, (size_t)parts_ub * sizeof(int64_t), c.stream));
    hipLaunchKernelGGL(k_hps_count, gc, dim3(B7_NT), 0, c.stream, a, (const int64_t *)tot, (const int64_t *)cstart,
                       (const int64_t *)xoff, (const int64_t *)pstart, xs, pcnt);
    LAUNCHCHECK();
    scan<int64_t, int64_t>(c, pcnt, segstart, parts_ub, false, (int64_t *)nullptr);
    hipLaunchKernelGGL((k_hps_scatter<WK>), gc, dim3(B7_NT), 0, c.stream, a, (const int64_t *)tot,
                       (const int64_t *)cstart, (const int64_t *)xoff, (const int64_t *)pstart, (const int32_t *)xs,
                       (const int64_t *)segstart, cursor, ys, ws);
    LAUNCHCHECK();
  }
  const size_t bytes = hp_lds_bytes(a32);
  const dim3 gp((unsigned)std::max<int64_t>(1, std::min<int64_t>(parts_ub, (int64_t)c.num_cu * 2)));
#define LCC_HP_PART(A32_, SEG_)                                                                                  \
  do {                                                                                                          \
    allow_lds(c, k_hp_part<WK, A32_, SEG_>, bytes);                                                            \
    hipLaunchKernelGGL((k_hp_part<WK, A32_, SEG_>), gp, dim3(HP_NT), bytes, c.stream, a, (const int64_t *)tot,  \
                       (const int64_t *)xoff, (const int64_t *)pstart, (const int32_t *)ys, part,               \
                       (const int64_t *)segstart, (const int64_t *)pcnt, (const int64_t *)ws);                  \
  } while (0)
  if (a32 && seg) LCC_HP_PART(true, true);
  else if (a32) LCC_HP_PART(true, false);
  else if (seg) LCC_HP_PART(false, true);
  else LCC_HP_PART(false, false);
#undef LCC_HP_PART
  LAUNCHCHECK();
  hipLaunchKernelGGL(k_b7_final, dim3((unsigned)std::min<int64_t>(n7_ub, (int64_t)c.num_cu * 4)), dim3(B7_NT), 0,
                     c.stream, a, (const int64_t *)pstart, (const SegBest *)part, (const uint8_t *)done);
  LAUNCHCHECK();
}

// ub_count / ub_arcs: upper bounds of the bucket's vertices and arcs.
template <int WK>
void launch_any(Ctx &c, int bin, bool a32, bool single, int64_t ub_count, int64_t ub_arcs, AggArgs a,
                int64_t grid) {
  if (single) launch_single<WK>(c, bin, a, grid);
  else if (bin == NBINS - 1 && c.hub_partition) launch_hub_part<WK>(c, a, ub_count, ub_arcs, a32);
  else if (bin == NBINS - 1 && a32) launch_flat_pk<WK, true>(c, a, ub_count, ub_arcs);
  else if (bin == NBINS - 1) launch_flat_pk<WK, false>(c, a, ub_count, ub_arcs);
  else if (a32) launch_bin<WK, true>(c, bin, a, grid);
  else launch_bin<WK, false>(c, bin, a, grid);
}

int64_t pow2_host(int64_t x) {
  int64_t h = 1;
  while (h < x) h <<= 1;
  return h;
}

template <int WK>
void launch_shared_wk(Ctx &c, bool a32, const AggArgs &a, const int32_t *C16, int64_t n1, uint32_t *mask,
                      const int32_t *seglist, const int64_t *seg_cnt, int64_t grid) {
  if (a32)
    c.launch(k_bm_shared<WK, true>, dim3((unsigned)grid), dim3(BM_NT), 0, a, C16, n1, mask, seglist, seg_cnt);
  else
    c.launch(k_bm_shared<WK, false>, dim3((unsigned)grid), dim3(BM_NT), 0, a, C16, n1, mask, seglist, seg_cnt);
  LAUNCHCHECK();
}

void launch_shared(Ctx &c, int wk, bool a32, const AggArgs &a, const int32_t *C16, int64_t n1, uint32_t *mask,
                   const int32_t *seglist, const int64_t *seg_cnt, int64_t grid) {
  switch (wk) {
    case LCC_WT_UNIT: launch_shared_wk<LCC_WT_UNIT>(c, a32, a, C16, n1, mask, seglist, seg_cnt, grid); break;
    case LCC_WT_I16: launch_shared_wk<LCC_WT_I16>(c, a32, a, C16, n1, mask, seglist, seg_cnt, grid); break;
    case LCC_WT_I32: launch_shared_wk<LCC_WT_I32>(c, a32, a, C16, n1, mask, seglist, seg_cnt, grid); break;
    default: launch_shared_wk<LCC_WT_I64>(c, a32, a, C16, n1, mask, seglist, seg_cnt, grid); break;
  }
}

// A small level's sub-round: one block per vertex, the degree bins below
// 2048 in one launch (256 threads, MID_SLOTS table) and the wider bin in a
// second one (WIDE_NT threads, table up to `slots`) when the level has such
// rows.  The singleton sub-round needs no table.
template <int NT, int WK> void launch_small_wk(Ctx &c, bool a32, bool single, AggArgs a, int64_t slots, int64_t grid) {
  const dim3 gr((unsigned)grid);
  if (single) {
    c.launch(k_bm_single<NT, NT, WK, 1>, gr, dim3(NT), 0, a);
  } else if (a32) {
    a.hcap = slots;
    const size_t bytes = wide_lds_bytes(slots, true);
    allow_lds(c, k_bm_wide<NT, WK, true, 1>, bytes);
    c.launch(k_bm_wide<NT, WK, true, 1>, gr, dim3(NT), bytes, a);
  } else {
    a.hcap = slots;
    const size_t bytes = wide_lds_bytes(slots, false);
    allow_lds(c, k_bm_wide<NT, WK, false, 1>, bytes);
    c.launch(k_bm_wide<NT, WK, false, 1>, gr, dim3(NT), bytes, a);
  }
  LAUNCHCHECK();
}

void launch_small(Ctx &c, int wk, bool wide_rows, bool a32, bool single, const AggArgs &a, int64_t slots,
                  int64_t grid) {
  if (wide_rows) {
    switch (wk) {
      case LCC_WT_UNIT: launch_small_wk<WIDE_NT, LCC_WT_UNIT>(c, a32, single, a, slots, grid); break;
      case LCC_WT_I16: launch_small_wk<WIDE_NT, LCC_WT_I16>(c, a32, single, a, slots, grid); break;
      case LCC_WT_I32: launch_small_wk<WIDE_NT, LCC_WT_I32>(c, a32, single, a, slots, grid); break;
      default: launch_small_wk<WIDE_NT, LCC_WT_I64>(c, a32, single, a, slots, grid); break;
    }
  } else {
    switch (wk) {
      case LCC_WT_UNIT: launch_small_wk<BM_NT, LCC_WT_UNIT>(c, a32, single, a, slots, grid); break;
      case LCC_WT_I16: launch_small_wk<BM_NT, LCC_WT_I16>(c, a32, single, a, slots, grid); break;
      case LCC_WT_I32: launch_small_wk<BM_NT, LCC_WT_I32>(c, a32, single, a, slots, grid); break;
      default: launch_small_wk<BM_NT, LCC_WT_I64>(c, a32, single, a, slots, grid); break;
    }
  }
}

void launch_agg(Ctx &c, int wk, int bin, bool a32, bool single, int64_t ub_count, int64_t ub_arcs,
                const AggArgs &a, int64_t grid) {
  switch (wk) {
    case LCC_WT_UNIT: launch_any<LCC_WT_UNIT>(c, bin, a32, single, ub_count, ub_arcs, a, grid); break;
    case LCC_WT_I16: launch_any<LCC_WT_I16>(c, bin, a32, single, ub_count, ub_arcs, a, grid); break;
    case LCC_WT_I32: launch_any<LCC_WT_I32>(c, bin, a32, single, ub_count, ub_arcs, a, grid); break;
    default: launch_any<LCC_WT_I64>(c, bin, a32, single, ub_count, ub_arcs, a, grid); break;
  }
}

const char *bin_name(int b) {
  static const char *names[NBINS] = {"bm_aggregate_g8",  "bm_aggregate_g16",  "bm_aggregate_g32",
                                     "bm_aggregate_g64", "bm_aggregate_g64w", "bm_aggregate_block",
                                     "bm_aggregate_wide", "bm_aggregate_global"};
  return names[b];
}

// Renames the non-empty fresh clusters to the smallest empty ids (see the
// file comment).  With `isoc` (device-driven iterations) the kernels skip
// themselves after an iteration without isolation and a pairing error stays
// in `err` for the caller's next read; without it the error is checked here.
void rename_fresh(Ctx &c, int64_t n, int32_t *C, int64_t *K, int32_t *cnt, int64_t *err, const JobView &jv,
                  const int64_t *isoc = nullptr, int S = 0) {
  Ctx::Timer tm(&c, "bm_rename", 0.0, (double)n);
  const size_t nn = (size_t)n;
  int32_t *rank_f = c.buf<int32_t>("rn.rankf", nn + 1);
  int32_t *rank_e = c.buf<int32_t>("rn.ranke", nn + 1);
  int32_t *elist = c.buf<int32_t>("rn.elist", nn);
  int32_t *newid = c.buf<int32_t>("rn.newid", nn);
  if (n <= RN_SMALL) {
    hipLaunchKernelGGL(k_rename_small, dim3(1), dim3(RN_NT), 0, c.stream, C, n, K, cnt, rank_f, rank_e, elist, newid,
                       jv, err, isoc, S);
    LAUNCHCHECK();
  } else {
    uint8_t *fresh = c.buf<uint8_t>("rn.fresh", nn);
    uint8_t *empty = c.buf<uint8_t>("rn.empty", nn);
    const unsigned grid = (unsigned)std::min<int64_t>(cdiv(n, 256), 65536);
    hipLaunchKernelGGL(k_fresh_flags, dim3(grid), dim3(256), 0, c.stream, cnt, n, fresh, empty, isoc, S);
    LAUNCHCHECK();
    // (after an iteration without isolation the flags are stale and every
    // kernel reading the ranks skips itself)
    scan<uint8_t, int32_t>(c, fresh, rank_f, n, false, rank_f + n);
    scan<uint8_t, int32_t>(c, empty, rank_e, n, false, rank_e + n);
    hipLaunchKernelGGL(k_empty_list, dim3(grid), dim3(256), 0, c.stream, empty, rank_e, rank_f, n, jv, elist, isoc,
                       S);
    LAUNCHCHECK();
    hipLaunchKernelGGL(k_fresh_move, dim3(grid), dim3(256), 0, c.stream, fresh, rank_f, elist, n, K, cnt, newid, err,
                       isoc, S);
    LAUNCHCHECK();
    hipLaunchKernelGGL(k_fresh_relabel, dim3(grid), dim3(256), 0, c.stream, C, n, newid, isoc, S);
    LAUNCHCHECK();
  }
  if (!isoc) {
    int64_t e = 0;
    d2h(c, &e, err, sizeof(e));
    if (e) fail(LCC_ERR_DEVICE, "internal: fresh clusters outnumbered the empty cluster ids");
  }
}

}  // namespace

void best_moves_run(Ctx &c, const lcc_graph &g, int64_t p, int64_t q, const lcc_params &prm, int32_t level,
                    int32_t phase, int32_t *C, const BMShape &shape, lcc_bm_stats &st, const BatchLevel *bl) {
  JobView jv;
  int64_t J = 0;
  std::vector<uint8_t> hrun;
  if (bl) {
    J = bl->jobs;
    jv.jid = bl->jid;
    jv.jbase = bl->jbase;
    jv.jp = bl->jp;
    jv.jq = bl->jq;
    jv.jrun = c.buf<uint8_t>("bt.run", (size_t)J);
    jv.jmoved = c.buf<int64_t>("bt.moved", (size_t)J);
    hrun.assign(bl->active, bl->active + J);
    h2d(c, const_cast<uint8_t *>(jv.jrun), hrun.data(), (size_t)J);
    HIPCHECK(hipMemsetAsync(jv.jmoved, 0, (size_t)J * sizeof(int64_t), c.stream));
    std::fill(bl->iters, bl->iters + J, 0);
    std::fill(bl->moved_any, bl->moved_any + J, 0);
  }
  const bool identity = shape.identity, acc32 = shape.acc32;
  std::memset(&st, 0, sizeof(st));
  st.term = LCC_TERM_NUM_ITER;
  const int64_t n = g.n;
  const int S = prm.S;
  const int NB = S * NBINS;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  int32_t *D = c.buf<int32_t>("bm.D", nn);
  // cluster totals cover the regular ids [0, n) and the fresh ids [n, 2n)
  int64_t *K = c.buf<int64_t>("bm.K", 2 * nn);
  int32_t *cnt = c.buf<int32_t>("bm.cnt", 2 * nn);
  uint8_t *next = c.buf<uint8_t>("bm.next", nn);
  int32_t *active = c.buf<int32_t>("bm.active", nn);
  int32_t *blist = c.buf<int32_t>("bm.blist", nn);
  uint16_t *bucket_of = c.buf<uint16_t>("bm.bucket", nn);
  if (n > 0) {
    HIPCHECK(hipMemsetAsync(next, 0, nn, c.stream));
    HIPCHECK(hipMemsetAsync(K + n, 0, nn * sizeof(int64_t), c.stream));
    HIPCHECK(hipMemsetAsync(cnt + n, 0, nn * sizeof(int32_t), c.stream));
    if (identity) {
      hipLaunchKernelGGL(k_init_identity, dim3((unsigned)std::min<int64_t>(cdiv(n, 256), 65535)), dim3(256), 0,
                         c.stream, g.k, K, cnt, n);
      LAUNCHCHECK();
    } else {
      cluster_totals(c, n, C, g.k, K, cnt);
    }
  }
  // bin 6 takes rows whose distinct clusters fill at most 70% of the LDS table
  const int64_t wslots = wide_slots(c, acc32);
  const int64_t wide_max = wslots * 7 / 10 - 1;
  const int wb = wt_bytes(g.wt_kind);
  // a frontier list after the first iteration (neighbors of movers, or of
  // the clusters movers left); movers mark neighbors, or the left clusters
  const bool nbr = prm.frontier != LCC_FRONTIER_ALL;
  const bool mark_left = prm.frontier == LCC_FRONTIER_CLUSTERS;
  // asynchronous moves: every deciding launch applies its moves to the one
  // state (no apply launch, no second copy, no singleton shortcut)
  const bool async = prm.async_moves != 0;
  uint8_t *left = nullptr, *left_cur = nullptr;
  if (mark_left) {
    left = c.buf<uint8_t>("bm.left", 2 * nn);
    HIPCHECK(hipMemsetAsync(left, 0, nn, c.stream));
  }
  // marks the neighbors of the vertices in a left cluster (end of iteration it)
  auto mark_left_nbrs = [&](const int32_t *Cnow, int32_t it) {
    uint8_t *cur = left + (size_t)(it & 1) * nn, *other = left + (size_t)((it + 1) & 1) * nn;
    Ctx::Timer tm(&c, "bm_frontier_clusters", 0.0, (double)n, true);
    c.launch(k_mark_left_nbrs, dim3((unsigned)std::min<int64_t>(cdiv(n, LN_NT), (int64_t)c.num_cu * 8)),
             dim3(LN_NT), 0, g.off, g.col, Cnow, n, (const uint8_t *)cur, other, next);
    LAUNCHCHECK();
  };
  const int LC = NSPREAD * NCTR;
  static const char *wk_tag[4] = {"_unit", "_i16", "_i32", "_i64"};
  // neighbors-of-movers frontier built at the end of each iteration by
  // k_frontier (device-driven iterations on levels above the small size)
  // instead of by the deciding kernels
  bool pulled_front = false;

  // Per-iteration device counters: bucket counts, bucket arcs, bucket starts
  // (NB + 1), per-launch counters, per-sub-round isolations, next-frontier
  // size, pairing errors.
  const int64_t o_bcnt = 0, o_barcs = NB, o_start = 2 * NB, o_lctr = 3 * NB + 1;
  // (then NSPREAD list-segment counts per sub-round for the shared-row launch)
  const int64_t o_isoc = o_lctr + (int64_t)LC * NB, o_nact = o_isoc + S, o_err = o_nact + 1, o_seg = o_err + 1,
                IB = o_seg + (int64_t)NSPREAD * S;
  const int64_t part_grid = std::min<int64_t>(std::max<int64_t>(1, cdiv(n, BM_NT * 8)), (int64_t)c.num_cu * 8);
  int32_t *blkcnt = c.buf<int32_t>("bm.pblk", (size_t)(part_grid * NB));
  int64_t *pcur = c.buf<int64_t>("bm.pcur", (size_t)(part_grid * NB));
  const size_t part_smem = (size_t)2 * NB * sizeof(int64_t);  // k_part_count
  const size_t scatter_smem = stable_lds_bytes(NB, BM_NT);      // k_part_scatter
  const size_t small_smem = part_small_lds_bytes(NB);           // k_part_small, k_iter_end_small

  // rows beyond the LDS tables remember how many clusters they met (k_hub_row)
  int32_t *hub_seen = nullptr;
  if (n > 0 && shape.maxdeg > wide_max) {
    hub_seen = c.buf<int32_t>("bm.hubseen", nn);
    HIPCHECK(hipMemsetAsync(hub_seen, 0, nn * sizeof(int32_t), c.stream));
  }
  auto agg_args = [&](int bi, const int64_t *dstart, int64_t *ctr) {
    AggArgs a;
    std::memset(&a, 0, sizeof(a));
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
    a.hub_limit = prm.hub_limit;
    a.hub_row_limit = prm.hub_row_limit;
    a.prune = prm.score_pruning > 0 || (prm.score_pruning == 0 && g.n >= PRUNE_MIN_N) ? 1 : 0;
    a.hub_seen = hub_seen;
    a.list = blist;
    a.D = D;
    // (with the pulled frontier, rows of 2048 arcs or more still mark their
    // neighbors as they decide: their kernels spread a row over a whole block,
    // which one wave of k_frontier could not)
    a.next_flag = prm.frontier == LCC_FRONTIER_NBR && (!pulled_front || bi % NBINS >= 6) ? next : nullptr;
    a.left_flag = left_cur;
    if (async) {
      a.Cw = C;
      a.Kw = K;
      a.cntw = cnt;
      a.nlev = n;
    }
    a.ctr = ctr + (size_t)LC * bi;
    a.jv = jv;
    a.dstart = dstart;
    a.bucket = bi;
    a.nbuckets = 1;
    return a;
  };
  auto class_name = [&](int b, bool single) {
    return std::string(single ? "bm_single" : (b == NBINS - 1 ? "bm_flat_seq" : bin_name(b))) + wk_tag[g.wt_kind];
  };
  // Sums of the NSPREAD copies of a launch's counters.
  auto launch_sums = [&](const int64_t *lctr, int bi, int k) {
    int64_t t = 0;
    for (int r = 0; r < NSPREAD; r++) t += lctr[(size_t)bi * LC + r * NCTR + k];
    return t;
  };

  // Device-driven iterations: every kernel takes its bucket from device
  // memory, so the host queues iterations without waiting and reads the
  // counters back once per chunk of iterations.  An iteration queued after
  // the one that ended the call changes nothing (no vertex moves against an
  // unchanged state, and an empty frontier has no work), so only the
  // counters up to the stopping iteration are used.  Rows wider than the
  // LDS tables (the flat path sizes its tables on the host) and stopping
  // inside an iteration take the host-driven path below.
  const bool dd = n > 0 && prm.stop_after_subrounds == 0;
  if (dd) {
    // Small levels: one block partitions, and one block-per-vertex launch per
    // sub-round covers every degree bin (fewer launches where the host's
    // launch rate, not the work, sets the pace).  Larger levels: one launch
    // per degree bin present in the level.
    const int64_t small_max = prm.small_level > 0 ? prm.small_level : SMALL_LEVEL;
    const bool small = !async && n <= small_max && shape.maxdeg <= wide_max;
    pulled_front = !small && !async && prm.frontier == LCC_FRONTIER_NBR;
    uint8_t *moved = pulled_front ? c.buf<uint8_t>("bm.moved", nn) : nullptr;
    // degree histogram of the level (larger levels launch one kernel per
    // non-empty bin); a small level needs only the largest degree: its
    // narrow launch (degree < 2048) always runs, empty or not
    int64_t hist[2 * NBINS] = {0};
    if (!small) {
      int64_t *hist_d = c.buf<int64_t>("bm.hist", 2 * NBINS);
      HIPCHECK(hipMemsetAsync(hist_d, 0, 2 * NBINS * sizeof(int64_t), c.stream));
      hipLaunchKernelGGL(k_bin_hist, dim3((unsigned)std::min<int64_t>(cdiv(n, BM_NT), (int64_t)c.num_cu * 4)),
                         dim3(BM_NT), 0, c.stream, g.off, n, wide_max, hist_d);
      LAUNCHCHECK();
      d2h(c, hist, hist_d, sizeof(hist));
    }
    // tables of the small-level kernels: MID_SLOTS below degree 2048, else
    // room for the widest row of the level
    const bool wide_rows = small ? shape.maxdeg > bin_limit_fixed(5) : hist[6] > 0;
    // (a small level whose shortest row has 2048 arcs or more skips the narrow launch)
    bool narrow_rows = small && shape.mindeg <= bin_limit_fixed(5);
    for (int b = 0; b < 6; b++) narrow_rows = narrow_rows || hist[b] > 0;
    const int64_t small_slots = std::min<int64_t>(pow2_host(2 * (shape.maxdeg + 1)), wslots);
    // lambda sweeps: rows of degree < 256 read once for all jobs (see k_bm_shared)
    bool shared_rows = false;
    for (int b = 0; b <= SH_BIN_HI; b++) shared_rows = shared_rows || hist[b] > 0;
    shared_rows = shared_rows && bl && bl->shared_n > 0 && !small && !async && J >= 2 && J <= SH_MAXJ &&
                  J * bl->shared_n == n;
    const int64_t n1 = shared_rows ? bl->shared_n : 0;
    // rows of degree < 256 (bins 0-4): one launch when they are few
    int64_t low_rows = 0;
    int low_bins = 0;
    for (int b = 0; b <= SH_BIN_HI; b++) {
      low_rows += hist[b];
      low_bins += hist[b] > 0;
    }
    const bool low_merged = !small && low_bins > 1 && low_rows <= (prm.low_merge > 0 ? prm.low_merge : 32768);
    int32_t *C16 = nullptr, *seglist = nullptr;
    uint32_t *shmask = nullptr;
    if (shared_rows) {
      C16 = c.buf<int32_t>("sh.C16", (size_t)(n1 * SH_MAXJ));
      seglist = c.buf<int32_t>("sh.seglist", (size_t)(n1 * NSPREAD));
      shmask = c.buf<uint32_t>("sh.mask", (size_t)n1);
      HIPCHECK(hipMemsetAsync(shmask, 0, (size_t)n1 * sizeof(uint32_t), c.stream));
    }
    // renaming buffers of the small-level iteration end (as rename_fresh's),
    // and the second copy of the state (sub-rounds alternate between them)
    int32_t *rn_rank_f = nullptr, *rn_rank_e = nullptr, *rn_elist = nullptr, *rn_newid = nullptr;
    int32_t *C2 = nullptr, *cnt2 = nullptr;
    int64_t *K2 = nullptr;
    if (small) {
      C2 = c.buf<int32_t>("bm.C2", nn);
      K2 = c.buf<int64_t>("bm.K2", 2 * nn);
      cnt2 = c.buf<int32_t>("bm.cnt2", 2 * nn);
      hipLaunchKernelGGL(k_copy_state, dim3((unsigned)cdiv(2 * n, 1024)), dim3(1024), 0, c.stream,
                         (const int32_t *)C, (const int64_t *)K, (const int32_t *)cnt, n, C2, K2, cnt2);
      LAUNCHCHECK();
      rn_rank_f = c.buf<int32_t>("rn.rankf", nn + 1);
      rn_rank_e = c.buf<int32_t>("rn.ranke", nn + 1);
      rn_elist = c.buf<int32_t>("rn.elist", nn);
      rn_newid = c.buf<int32_t>("rn.newid", nn);
    }
    const int32_t NI = std::max<int32_t>(prm.num_iter, 1);
    int64_t *ctrs = c.buf<int64_t>("bm.ctrs", (size_t)(NI * IB));
    HIPCHECK(hipMemsetAsync(ctrs, 0, (size_t)(NI * IB) * sizeof(int64_t), c.stream));
    int32_t *jiters = nullptr;
    uint8_t *jmoved_any = nullptr;
    if (bl) {
      jiters = c.buf<int32_t>("bt.iters", (size_t)J);
      jmoved_any = c.buf<uint8_t>("bt.movedany", (size_t)J);
      HIPCHECK(hipMemsetAsync(jiters, 0, (size_t)J * sizeof(int32_t), c.stream));
      HIPCHECK(hipMemsetAsync(jmoved_any, 0, (size_t)J, c.stream));
    }
    const int64_t apply_grid = std::min<int64_t>(cdiv(n, BM_NT), (int64_t)c.num_cu * 8);
    struct Timed {
      size_t idx;
      int32_t it, bi, nb;
      bool single;
      int32_t shared_s = -1;  // sub-round of a shared-row launch
    };
    std::vector<Timed> timed;
    std::vector<int64_t> h((size_t)(NI * IB));
    // (with the all-vertices rule an iteration past the end redoes all the
    // work, so only the neighbor frontier queues ahead)
    const bool fixed_chunk = prm.queue_ahead > 0;
    int32_t queued = 0,
            chunk = fixed_chunk ? prm.queue_ahead : small && nbr ? std::max<int32_t>(1, c.small_iter_hint[phase & 1]) : 1;
    bool done = false;
    // a small level's chunk of iterations is a fixed sequence of launches
    // through c.launch: recorded, and replayed as a graph when repeated
    const bool replay = small && !c.timing && !prm.no_graph_replay;
    while (!done && queued < prm.num_iter) {
      const int32_t first = queued, last = std::min<int32_t>(prm.num_iter, queued + chunk);
      if (replay) c.begin_record();
      for (int32_t it = first; it < last; it++) {
        int64_t *blk = ctrs + (size_t)it * IB;
        if (mark_left) left_cur = left + (size_t)(it & 1) * nn;
        const uint64_t hh = round_hash(prm.seed, level, phase, it);
        if (moved) HIPCHECK(hipMemsetAsync(moved, 0, nn, c.stream));
        // the first iteration and the "all vertices" rule take every vertex
        const bool all = it == 0 || !nbr;
        const int32_t *list = all ? nullptr : active;
        const int64_t *na_dev = all ? nullptr : blk - IB + o_nact;
        if (small) {
          // later iterations were partitioned at the end of the previous one
          if (it == 0) {
            c.launch(k_part_small, dim3(1), dim3(PS_NT), small_smem, list, (int64_t)n, na_dev,
                     (const int64_t *)g.off, hh, (int32_t)S, wide_max, jv, bucket_of, blk + o_bcnt, blk + o_barcs,
                     blk + o_start, blist);
            LAUNCHCHECK();
          }
        } else {
          hipLaunchKernelGGL(k_part_count, dim3((unsigned)part_grid), dim3(BM_NT), part_smem, c.stream, list, n,
                             na_dev, g.off, hh, S, wide_max, jv, bucket_of, blkcnt, blk + o_bcnt, blk + o_barcs);
          LAUNCHCHECK();
          hipLaunchKernelGGL(k_part_offsets, dim3((unsigned)NB), dim3(BM_NT), 0, c.stream, blk + o_bcnt, blkcnt,
                             part_grid, pcur, blk + o_start);
          LAUNCHCHECK();
          hipLaunchKernelGGL(k_part_scatter, dim3((unsigned)part_grid), dim3(BM_NT), scatter_smem, c.stream, list, n,
                             na_dev, bucket_of, S, pcur, blist);
          LAUNCHCHECK();
          if (shape.maxdeg > wide_max) {
            hipLaunchKernelGGL(k_hub_order, dim3((unsigned)S), dim3(HO_NT), 0, c.stream,
                               (const int64_t *)(blk + o_start), g.off, (int64_t)c.num_cu, blist);
            LAUNCHCHECK();
          }
        }
        for (int s = 0; s < S; s++) {
          const bool single = it == 0 && s == 0 && identity && shape.simple && !async;
          if (small) {
            // bins 0-5 (degree < 2048), then bin 6 if the level has wider rows
            // sub-round s reads copy s % 2 and applies to the other, into
            // which its first launch replays sub-round s - 1
            const bool odd = s % 2 == 1;
            bool replay = s > 0;
            for (int part = 0; part < 2; part++) {
              if (part == 0 ? !narrow_rows : !wide_rows) continue;
              const int bi = s * NBINS + (part ? 6 : 0);
              AggArgs a = agg_args(bi, blk + o_start, blk + o_lctr);
              a.nbuckets = part ? 1 : 6;
              a.C = odd ? C2 : C;
              a.K = odd ? K2 : K;
              a.cnt = odd ? cnt2 : cnt;
              a.Cw = odd ? C : C2;
              a.Kw = odd ? K : K2;
              a.cntw = odd ? cnt : cnt2;
              a.nlev = n;
              a.iso_ctr = blk + o_isoc + s;
              if (replay) {
                a.rb0 = (s - 1) * NBINS;
                a.rb1 = s * NBINS;
                replay = false;
              }
              const size_t pidx = c.pending.size();
              {
                Ctx::Timer tm(&c, (std::string(single ? "bm_single_small" : "bm_aggregate_small") +
                                   (part ? "_wide" : "") + wk_tag[g.wt_kind]).c_str(),
                              0.0, 0.0, true);
                launch_small(c, g.wt_kind, part == 1, acc32, single, a, part ? small_slots : MID_SLOTS,
                             std::min<int64_t>(n, (int64_t)c.num_cu * (part ? 2 : 4)));
              }
              if (c.timing) timed.push_back({pidx, it, bi, a.nbuckets, single});
            }
          }
          const bool sh_now = shared_rows && !single;
          if (sh_now) {
            const int32_t b0 = s * NBINS, b1 = s * NBINS + SH_BIN_HI + 1;
            {
              Ctx::Timer tm(&c, "bm_shared_transpose", 8.0 * (double)n, (double)n, true);
              c.launch(k_sh_transpose, dim3((unsigned)std::min<int64_t>(cdiv(n1, 256), 65536)), dim3(256), 0,
                       (const int32_t *)C, n1, (int32_t)J, C16);
              LAUNCHCHECK();
            }
            {
              Ctx::Timer tm(&c, "bm_shared_mask", 0.0, 0.0, true);
              c.launch(k_sh_mask, dim3((unsigned)std::min<int64_t>(cdiv(n, BM_NT), (int64_t)c.num_cu * 8)),
                       dim3(BM_NT), 0, (const int32_t *)blist, (const int64_t *)(blk + o_start), b0, b1, n1, shmask,
                       seglist, blk + o_seg + (int64_t)NSPREAD * s);
              LAUNCHCHECK();
            }
            const int bi = s * NBINS;
            const AggArgs a = agg_args(bi, blk + o_start, blk + o_lctr);
            const size_t pidx = c.pending.size();
            {
              Ctx::Timer tm(&c, (std::string("bm_aggregate_shared") + wk_tag[g.wt_kind]).c_str(), 0.0, 0.0, true);
              launch_shared(c, g.wt_kind, acc32, a, C16, n1, shmask, seglist, blk + o_seg + (int64_t)NSPREAD * s,
                            std::min<int64_t>(cdiv(n1, SH_WPB), (int64_t)c.num_cu * 8));
            }
            if (c.timing) {
              Timed t{pidx, it, bi, SH_BIN_HI + 1, false};
              t.shared_s = s;
              timed.push_back(t);
            }
          }
          for (int b = 0; b < NBINS && !small; b++) {
            if (!hist[b] || (sh_now && b <= SH_BIN_HI)) continue;
            const int bi = s * NBINS + b;
            AggArgs a = agg_args(bi, blk + o_start, blk + o_lctr);
            if (async) a.iso_ctr = blk + o_isoc + s;
            // few rows below degree 256 in the level: their buckets (consecutive)
            // go to bin 4's kernel in one launch
            const bool merged = b <= SH_BIN_HI && !sh_now && low_merged;
            const int lb = merged ? SH_BIN_HI : b;
            if (merged) a.nbuckets = SH_BIN_HI + 1 - b;
            const size_t pidx = c.pending.size();
            {
              Ctx::Timer tm(&c, class_name(lb, single).c_str(), 0.0, 0.0, single || lb != NBINS - 1);
              launch_agg(c, g.wt_kind, lb, acc32, single, merged ? low_rows : hist[b], hist[NBINS + b], a,
                         bin_grid(c, lb, merged ? low_rows : hist[b], false));
            }
            if (c.timing) timed.push_back({pidx, it, bi, a.nbuckets, single});
            if (merged) b = SH_BIN_HI;
          }
          if (!small && !async) {
            Ctx::Timer tm(&c, "bm_apply", 0.0, 0.0, true);
            c.launch(k_bm_apply, dim3((unsigned)apply_grid), dim3(BM_NT), 0, (const int32_t *)blist, (int64_t)0,
                     (const int64_t *)(blk + o_start), (int32_t)(s * NBINS), (int32_t)((s + 1) * NBINS),
                     (const int32_t *)D, C, K, cnt, g.k, n, blk + o_isoc + s, jv.jid, jv.jmoved, moved,
                     (const int64_t *)g.off);
            LAUNCHCHECK();
          }
        }
        if (moved) {
          Ctx::Timer tm(&c, "bm_frontier", 0.0, (double)n, true);
          c.launch(k_frontier, dim3((unsigned)std::min<int64_t>(cdiv(n, FR_NT), (int64_t)c.num_cu * 16)),
                   dim3(FR_NT), 0, (const int64_t *)g.off, (const int32_t *)g.col, n, (const uint8_t *)moved,
                   (const int64_t *)(blk + o_lctr), (int32_t)NB, next);
          LAUNCHCHECK();
        }
        // (on small levels the state copy the last sub-round wrote)
        if (mark_left) mark_left_nbrs(small && (S - 1) % 2 == 0 ? C2 : C, it);
        if (small) {
          IterEndSmall e;
          std::memset(&e, 0, sizeof(e));
          // the last sub-round S - 1 read copy (S - 1) % 2 and applied to the
          // other, so copy (S - 1) % 2 lags by that sub-round's moves
          const bool lag_first = (S - 1) % 2 == 0;
          e.D = D;
          e.k = g.k;
          e.dstart_cur = blk + o_start;
          e.rb0 = (S - 1) * NBINS;
          e.rb1 = S * NBINS;
          e.Cl = lag_first ? C : C2;
          e.Kl = lag_first ? K : K2;
          e.cntl = lag_first ? cnt : cnt2;
          e.blist = blist;
          e.C2 = C2;
          e.K2 = K2;
          e.cnt2 = cnt2;
          e.next = next;
          e.active = active;
          e.nact = blk + o_nact;
          e.compact = nbr;
          e.C = C;
          e.K = K;
          e.cnt = cnt;
          e.rank_f = rn_rank_f;
          e.rank_e = rn_rank_e;
          e.elist = rn_elist;
          e.newid = rn_newid;
          e.err = blk + o_err;
          e.isoc = blk + o_isoc;
          e.jiters = jiters;
          e.jmoved_any = jmoved_any;
          e.jobs = bl ? J : 0;
          e.part = it + 1 < prm.num_iter;
          if (e.part) {
            int64_t *nb = blk + IB;  // the next iteration's counter block
            e.off = g.off;
            e.h_next = round_hash(prm.seed, level, phase, it + 1);
            e.wide_max = wide_max;
            e.bucket_of = bucket_of;
            e.bcnt = nb + o_bcnt;
            e.barcs = nb + o_barcs;
            e.dstart = nb + o_start;
          }
          Ctx::Timer tm(&c, "bm_iter_end_small", 0.0, (double)n, true);
          c.launch(k_iter_end_small, dim3(1), dim3(PS_NT), small_smem, e, n, (int32_t)S, jv);
          LAUNCHCHECK();
        } else {
          if (nbr) compact_flags(c, next, n, active, blk + o_nact, true, "bm.cmp");
          rename_fresh(c, n, C, K, cnt, blk + o_err, jv, blk + o_isoc, S);
          if (bl) {
            hipLaunchKernelGGL(k_job_update, dim3((unsigned)std::min<int64_t>(cdiv(J, 256), 1024)), dim3(256), 0,
                               c.stream, const_cast<uint8_t *>(jv.jrun), jv.jmoved, jiters, jmoved_any, J);
            LAUNCHCHECK();
          }
        }
      }
      if (replay) c.end_record();
      queued = last;
      d2h(c, h.data() + (size_t)first * IB, ctrs + (size_t)first * IB, (size_t)(last - first) * IB * sizeof(int64_t));
      for (int32_t it = first; it < last && !done; it++) {
        const int64_t *hb = h.data() + (size_t)it * IB;
        const int64_t *hl = hb + o_lctr;
        int64_t moved_it = 0, cap_err = 0, hub_over = 0;
        for (int bi = 0; bi < NB; bi++) {
          moved_it += launch_sums(hl, bi, 0);
          st.candidates += launch_sums(hl, bi, 1);
          cap_err += launch_sums(hl, bi, 3);
          hub_over += launch_sums(hl, bi, 6);
          st.vertices_processed += hb[o_bcnt + bi];
          st.arcs_scanned += hb[o_barcs + bi];
        }
        if (hub_over) throw HubOverflow{};
        if (cap_err)
          fail(LCC_ERR_DEVICE, "internal: a vertex degree exceeded the hash capacity sized from the maximum degree");
        if (hb[o_err]) fail(LCC_ERR_DEVICE, "internal: fresh clusters outnumbered the empty cluster ids");
        if (it < LCC_MAX_ITER_STATS) {
          st.active_per_iter[it] = (it == 0 || !nbr) ? n : h[(size_t)(it - 1) * IB + o_nact];
          st.moves_per_iter[it] = moved_it;
        }
        st.iterations++;
        st.subrounds += S;
        st.moves += moved_it;
        if (moved_it) st.moved_any = 1;
        if (moved_it == 0) {
          st.term = LCC_TERM_NO_MOVES;
          done = true;
        }
      }
      // later chunks are longer only where a finished call leaves no work
      if (nbr && !fixed_chunk) chunk++;
    }
    if (c.timing) {
      for (const Timed &t : timed) {
        if (t.idx >= c.pending.size()) continue;
        const int64_t *hb = h.data() + (size_t)t.it * IB;
        double cntb = 0, arcs = 0;
        for (int k = 0; k < t.nb; k++) {
          cntb += (double)hb[o_bcnt + t.bi + k];
          arcs += (double)hb[o_barcs + t.bi + k];
        }
        const double per_arc = t.single ? 12.0 + wb : 8.0 + wb;
        // candidates gather K (8 B each); movers store one flag per neighbor
        const double extra = 8.0 * (double)launch_sums(hb + o_lctr, t.bi, 1) +
                             (pulled_front ? 0.0 : (double)launch_sums(hb + o_lctr, t.bi, 2));
        if (t.shared_s >= 0) {
          // per listed vertex: list, mask, offsets, k (32 B); per row arc,
          // once for all jobs: col, weight, the 64-byte id line; per (vertex,
          // job): C, K and size of its cluster, D (20 B)
          const double uv = (double)launch_sums(hb + o_lctr, t.bi, 4), ua = (double)launch_sums(hb + o_lctr, t.bi, 5);
          c.pending[t.idx].bytes = uv * 32.0 + ua * (4.0 + wb + 4.0 * SH_MAXJ) + cntb * 20.0 + extra;
        } else {
          c.pending[t.idx].bytes = cntb * 48.0 + arcs * per_arc + extra;
        }
        c.pending[t.idx].items = arcs;
      }
    }
    if (small && nbr) c.small_iter_hint[phase & 1] = st.iterations;
    if (bl) {
      d2h(c, bl->iters, jiters, (size_t)J * sizeof(int32_t));
      d2h(c, bl->moved_any, jmoved_any, (size_t)J);
    }
    if (c.timing) c.collect_timing();
    return;
  }

  // Host-driven iterations: bucket sizes are read back before the launches.
  const size_t nctr = (size_t)IB;
  int64_t *dctr = c.buf<int64_t>("bm.ctr", nctr);
  int64_t *bcnt = dctr + o_bcnt, *barcs = dctr + o_barcs, *dstart = dctr + o_start, *lctr = dctr + o_lctr;
  int64_t *isoc = dctr + o_isoc, *nact = dctr + o_nact, *iso_err = dctr + o_err;
  std::vector<int64_t> hctr(nctr);
  const int32_t *list = nullptr;  // nullptr = every vertex
  int64_t na = n;
  if (bl) c.sync();
  bool stopped = false;
  for (int32_t it = 0; it < prm.num_iter && !stopped; it++) {
    const uint64_t hh = round_hash(prm.seed, level, phase, it);
    if (mark_left) left_cur = left + (size_t)(it & 1) * nn;
    st.iterations++;
    HIPCHECK(hipMemsetAsync(dctr, 0, nctr * sizeof(int64_t), c.stream));
    if (bl) {
      HIPCHECK(hipMemsetAsync(jv.jmoved, 0, (size_t)J * sizeof(int64_t), c.stream));
      for (int64_t j = 0; j < J; j++)
        if (hrun[j]) bl->iters[j]++;
    }
    if (na > 0) {
      hipLaunchKernelGGL(k_part_count, dim3((unsigned)part_grid), dim3(BM_NT), part_smem, c.stream, list, na,
                         (const int64_t *)nullptr, g.off, hh, S, wide_max, jv, bucket_of, blkcnt, bcnt, barcs);
      LAUNCHCHECK();
      hipLaunchKernelGGL(k_part_offsets, dim3((unsigned)NB), dim3(BM_NT), 0, c.stream, bcnt, blkcnt, part_grid, pcur,
                         dstart);
      LAUNCHCHECK();
      hipLaunchKernelGGL(k_part_scatter, dim3((unsigned)part_grid), dim3(BM_NT), scatter_smem, c.stream, list, na,
                         (const int64_t *)nullptr, bucket_of, S, pcur, blist);
      LAUNCHCHECK();
      if (shape.maxdeg > wide_max) {
        hipLaunchKernelGGL(k_hub_order, dim3((unsigned)S), dim3(HO_NT), 0, c.stream, (const int64_t *)dstart, g.off,
                           (int64_t)c.num_cu, blist);
        LAUNCHCHECK();
      }
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
        AggArgs a = agg_args(bi, nullptr, lctr);
        a.list = blist + start[bi];
        a.count = cntb;
        if (async) a.iso_ctr = isoc + s;
        const int64_t arcs_i = hctr[NB + bi];
        const double arcs_b = (double)arcs_i;
        // first sub-round from singletons on rows without repeats: no
        // aggregation (later sub-rounds see the moves of earlier ones)
        const bool single = it == 0 && s == 0 && identity && shape.simple && !async;
        size_t pidx = c.pending.size();
        {
          // algorithmic bytes: per vertex list, offsets, C, k, K, cnt, D (48 B);
          // per arc col, C[u] (or k[u] for singletons) and the weight.  The
          // flat bin is a sequence of kernels: timed as one class, never taken
          // as "the" kernel of a roofline
          const double per_arc = single ? 12.0 + wb : 8.0 + wb;
          Ctx::Timer tm(&c, class_name(b, single).c_str(), (double)cntb * 48.0 + arcs_b * per_arc, arcs_b,
                        single || b != NBINS - 1);
          launch_agg(c, g.wt_kind, b, acc32, single, cntb, arcs_i, a, bin_grid(c, b, cntb, true));
        }
        launches.push_back({c.timing ? pidx : (size_t)-1, bi});
        st.vertices_processed += cntb;
        st.arcs_scanned += hctr[NB + bi];
      }
      if (total_s > 0 && !async) {
        Ctx::Timer tm(&c, "bm_apply", (double)total_s * 12.0, (double)total_s);
        hipLaunchKernelGGL(k_bm_apply, dim3((unsigned)cdiv(total_s, BM_NT)), dim3(BM_NT), 0, c.stream,
                           blist + start[s * NBINS], total_s, (const int64_t *)nullptr, 0, 0, D, C, K, cnt, g.k, n,
                           isoc + s, jv.jid, jv.jmoved, (uint8_t *)nullptr, (const int64_t *)nullptr);
        LAUNCHCHECK();
      }
      st.subrounds++;
    }
    // next frontier
    if (mark_left && !stopped && n > 0) mark_left_nbrs(C, it);
    if (nbr && n > 0) compact_flags(c, next, n, active, nact, true, "bm.cmp");
    d2h(c, hctr.data() + o_lctr, lctr, (size_t)(LC * NB + S + 2) * sizeof(int64_t));
    const int64_t *hl = hctr.data() + o_lctr;
    int64_t moved_it = 0, cap_err = 0, hub_over = 0;
    for (int bi = 0; bi < NB; bi++) {
      moved_it += launch_sums(hl, bi, 0);
      st.candidates += launch_sums(hl, bi, 1);
      cap_err += launch_sums(hl, bi, 3);
      hub_over += launch_sums(hl, bi, 6);
    }
    if (hub_over) throw HubOverflow{};
    const int64_t hl_nact = hctr[o_nact];
    int64_t isolated = 0;
    for (int s = 0; s < S; s++) isolated += hctr[o_isoc + s];
    if (cap_err)
      fail(LCC_ERR_DEVICE, "internal: a vertex degree exceeded the hash capacity sized from the maximum degree");
    if (isolated) rename_fresh(c, n, C, K, cnt, iso_err, jv);
    if (bl) {
      // per-job termination: a job without moves in this iteration stops
      std::vector<int64_t> hm((size_t)J);
      d2h(c, hm.data(), jv.jmoved, (size_t)J * sizeof(int64_t));
      bool changed = false;
      for (int64_t j = 0; j < J; j++) {
        if (!hrun[j]) continue;
        if (hm[j]) bl->moved_any[j] = 1;
        if (!hm[j] && !stopped) {
          hrun[j] = 0;
          changed = true;
        }
      }
      if (changed) {
        h2d(c, const_cast<uint8_t *>(jv.jrun), hrun.data(), (size_t)J);
        c.sync();
      }
    }
    if (c.timing) {
      for (auto &L : launches) {
        if (L.pending_idx < c.pending.size()) {
          // candidates gather K (8 B each); movers store one flag per neighbor
          c.pending[L.pending_idx].bytes +=
              8.0 * (double)launch_sums(hl, L.slot, 1) + (double)launch_sums(hl, L.slot, 2);
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
    if (nbr) {
      na = hl_nact;
      list = active;
    } else {
      na = n;
      list = nullptr;
    }
  }
  if (c.timing) c.collect_timing();
}

__global__ void k_copy_i32(const int32_t *__restrict__ a, int32_t *__restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// A call whose rows beyond the LDS tables go through hash partitions keeps
// a copy of C: if a partition overflowed (k_hp_part), the call is redone from
// that copy with the global tables, so the result never depends on it.
void best_moves(Ctx &c, const lcc_graph &g, int64_t p, int64_t q, const lcc_params &prm, int32_t level,
                int32_t phase, int32_t *C, const BMShape &shape, lcc_bm_stats &st, const BatchLevel *bl) {
  const int64_t wide_max = wide_slots(c, shape.acc32) * 7 / 10 - 1;
  c.hub_partition = false;
  c.hub_scatter = shape.maxdeg > HP_MAX_DEG;
  if (g.n <= 0 || shape.maxdeg <= wide_max) {
    best_moves_run(c, g, p, q, prm, level, phase, C, shape, st, bl);
    return;
  }
  const unsigned grid = (unsigned)std::min<int64_t>(cdiv(g.n, 256), 65536);
  int32_t *snap = c.buf<int32_t>("bm.Csnap", (size_t)g.n);
  hipLaunchKernelGGL(k_copy_i32, dim3(grid), dim3(256), 0, c.stream, (const int32_t *)C, snap, g.n);
  LAUNCHCHECK();
  c.hub_partition = true;
  try {
    best_moves_run(c, g, p, q, prm, level, phase, C, shape, st, bl);
    c.hub_partition = false;
  } catch (const HubOverflow &) {
    c.hub_partition = false;
    c.sync();
    hipLaunchKernelGGL(k_copy_i32, dim3(grid), dim3(256), 0, c.stream, (const int32_t *)snap, C, g.n);
    LAUNCHCHECK();
    best_moves_run(c, g, p, q, prm, level, phase, C, shape, st, bl);
  } catch (...) {
    c.hub_partition = false;
    throw;
  }
}

}  // namespace lcc
