// prims.hpp -- data-parallel primitives for gfx950 used by the best-move,
// compress and objective kernels: block/wave scans, a three-phase exclusive
// scan over int64 lengths, order-preserving flag compaction, and a stable LSD
// radix sort (8-bit digits, 64-wide wavefronts, ballot-based stable ranks).
#pragma once

#include "common.hpp"

namespace lcc {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Inclusive scan over the 64 lanes of a wavefront.
template <class T> __device__ __forceinline__ T wave_incl_scan(T x) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    T y = __shfl_up(x, o, WAVE);
    if (l >= o) x += y;
  }
  return x;
}

template <class T> __device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, WAVE);
  return x;
}

// Exclusive scan of one value per thread over a block of NT threads.
// Returns the exclusive prefix; *total receives the block total.
template <class T, int NT> __device__ __forceinline__ T block_excl_scan(T x, T *total) {
  static_assert(NT % WAVE == 0, "block must be whole waves");
  constexpr int NW = NT / WAVE;
  __shared__ T wsum[NW];
  const int w = threadIdx.x / WAVE;
  T inc = wave_incl_scan(x);
  if (lane_id() == WAVE - 1) wsum[w] = inc;
  __syncthreads();
  T before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; i++) {
    T s = wsum[i];
    if (i < w) before += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return before + inc - x;
}

// ------------------------------------------------------------------- scan

constexpr int SCAN_NT = 256;
constexpr int SCAN_IPT = 8;
constexpr int SCAN_TILE = SCAN_NT * SCAN_IPT;

template <class TIn, class TOut>
__global__ __launch_bounds__(SCAN_NT) void k_scan_reduce(const TIn *__restrict__ in, int64_t n,
                                                          TOut *__restrict__ partial) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  TOut s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; i++) {
    int64_t idx = base + (int64_t)i * SCAN_NT + threadIdx.x;
    if (idx < n) s += (TOut)in[idx];
  }
  s = wave_sum(s);
  __shared__ TOut ws[SCAN_NT / WAVE];
  if (lane_id() == 0) ws[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    TOut t = 0;
    for (int i = 0; i < SCAN_NT / WAVE; i++) t += ws[i];
    partial[blockIdx.x] = t;
  }
}

// Scans one tile with an optional carry-in per tile.  Items are loaded
// striped (coalesced) into LDS and scanned in a blocked arrangement.
template <class TIn, class TOut>
__global__ __launch_bounds__(SCAN_NT) void k_scan_down(const TIn *__restrict__ in, TOut *__restrict__ out,
                                                        int64_t n, const TOut *__restrict__ carry,
                                                        int inclusive, TOut *__restrict__ total) {
  __shared__ TOut tile[SCAN_TILE];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; i++) {
    int j = i * SCAN_NT + threadIdx.x;
    int64_t idx = base + j;
    tile[j] = idx < n ? (TOut)in[idx] : (TOut)0;
  }
  __syncthreads();
  TOut v[SCAN_IPT];
  TOut s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_IPT; i++) {
    v[i] = tile[threadIdx.x * SCAN_IPT + i];
    s += v[i];
  }
  TOut tot;
  TOut pre = block_excl_scan<TOut, SCAN_NT>(s, &tot);
  if (carry) pre += carry[blockIdx.x];
#pragma unroll
  for (int i = 0; i < SCAN_IPT; i++) {
    TOut x = v[i];
    tile[threadIdx.x * SCAN_IPT + i] = inclusive ? pre + x : pre;
    pre += x;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < SCAN_IPT; i++) {
    int j = i * SCAN_NT + threadIdx.x;
    int64_t idx = base + j;
    if (idx < n) out[idx] = tile[j];
  }
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
    *total = (carry ? carry[blockIdx.x] : (TOut)0) + tot;
}

// out = exclusive (or inclusive) prefix sum of in over n items (in == out
// allowed).  `total` (device, nullable) receives the sum of all items.  Uses
// the context's scratch names "scan.<depth>".
template <class TIn, class TOut>
void scan(Ctx &c, const TIn *in, TOut *out, int64_t n, bool inclusive, TOut *total, int depth = 0) {
  if (n <= 0) {
    if (total) HIPCHECK(hipMemsetAsync(total, 0, sizeof(TOut), c.stream));
    return;
  }
  int64_t nb = cdiv(n, SCAN_TILE);
  if (nb == 1) {
    hipLaunchKernelGGL((k_scan_down<TIn, TOut>), dim3(1), dim3(SCAN_NT), 0, c.stream, in, out, n,
                       (const TOut *)nullptr, (int)inclusive, total);
    LAUNCHCHECK();
    return;
  }
  TOut *part = c.buf<TOut>("scan." + std::to_string(depth), (size_t)nb);
  hipLaunchKernelGGL((k_scan_reduce<TIn, TOut>), dim3((unsigned)nb), dim3(SCAN_NT), 0, c.stream, in, n, part);
  LAUNCHCHECK();
  scan<TOut, TOut>(c, part, part, nb, false, (TOut *)nullptr, depth + 1);
  hipLaunchKernelGGL((k_scan_down<TIn, TOut>), dim3((unsigned)nb), dim3(SCAN_NT), 0, c.stream, in, out, n,
                     (const TOut *)part, (int)inclusive, total);
  LAUNCHCHECK();
}

// ------------------------------------------------------------- compaction

constexpr int CMP_NT = 256;
constexpr int CMP_IPT = 16;
constexpr int CMP_TILE = CMP_NT * CMP_IPT;

static __global__ __launch_bounds__(CMP_NT) void k_flag_count(const uint8_t *__restrict__ flags, int64_t n,
                                                       int64_t *__restrict__ partial) {
  const int64_t base = (int64_t)blockIdx.x * CMP_TILE + (int64_t)threadIdx.x * CMP_IPT;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < CMP_IPT; i++) s += (base + i < n) ? (flags[base + i] != 0) : 0;
  s = wave_sum(s);
  __shared__ int64_t ws[CMP_NT / WAVE];
  if (lane_id() == 0) ws[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int i = 0; i < CMP_NT / WAVE; i++) t += ws[i];
    partial[blockIdx.x] = t;
  }
}

// Writes the indices of set flags in ascending order; optionally clears them.
static __global__ __launch_bounds__(CMP_NT) void k_flag_scatter(uint8_t *__restrict__ flags, int64_t n,
                                                         const int64_t *__restrict__ offs,
                                                         int32_t *__restrict__ list, int clear) {
  const int64_t base = (int64_t)blockIdx.x * CMP_TILE + (int64_t)threadIdx.x * CMP_IPT;
  uint8_t f[CMP_IPT];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < CMP_IPT; i++) {
    f[i] = (base + i < n) ? flags[base + i] : 0;
    s += f[i] != 0;
  }
  int64_t tot;
  int64_t pos = block_excl_scan<int64_t, CMP_NT>(s, &tot) + offs[blockIdx.x];
#pragma unroll
  for (int i = 0; i < CMP_IPT; i++) {
    if (f[i]) {
      list[pos++] = (int32_t)(base + i);
      if (clear) flags[base + i] = 0;
    }
  }
}

// Small inputs in one block and one launch: tiles of CMP_SMALL_NT flags in order.
constexpr int CMP_SMALL_NT = 1024;
constexpr int64_t CMP_SMALL = 16384;

// One block of CMP_SMALL_NT threads: list <- ascending i with flags[i] != 0.
__device__ __forceinline__ void compact_small_body(uint8_t *__restrict__ flags, int64_t n, int32_t *__restrict__ list,
                                                   int64_t *__restrict__ count, int clear) {
  int64_t carry = 0;
  for (int64_t x0 = 0; x0 < n; x0 += CMP_SMALL_NT) {
    const int64_t x = x0 + threadIdx.x;
    const int64_t f = x < n && flags[x] != 0;
    int64_t tot;
    const int64_t pos = carry + block_excl_scan<int64_t, CMP_SMALL_NT>(f, &tot);
    if (f) {
      list[pos] = (int32_t)x;
      if (clear) flags[x] = 0;
    }
    carry += tot;
  }
  if (threadIdx.x == 0) *count = carry;
}

static __global__ __launch_bounds__(CMP_SMALL_NT) void k_flag_compact_small(uint8_t *__restrict__ flags, int64_t n,
                                                                            int32_t *__restrict__ list,
                                                                            int64_t *__restrict__ count, int clear) {
  compact_small_body(flags, n, list, count, clear);
}

// list <- ascending indices i with flags[i] != 0; *count_dev <- their number.
inline void compact_flags(Ctx &c, uint8_t *flags, int64_t n, int32_t *list, int64_t *count_dev, bool clear,
                          const char *tag = "cmp") {
  if (n <= 0) {
    HIPCHECK(hipMemsetAsync(count_dev, 0, sizeof(int64_t), c.stream));
    return;
  }
  if (n <= CMP_SMALL) {
    hipLaunchKernelGGL(k_flag_compact_small, dim3(1), dim3(CMP_SMALL_NT), 0, c.stream, flags, n, list, count_dev,
                       (int)clear);
    LAUNCHCHECK();
    return;
  }
  int64_t nb = cdiv(n, CMP_TILE);
  int64_t *part = c.buf<int64_t>(std::string(tag) + ".part", (size_t)nb);
  hipLaunchKernelGGL(k_flag_count, dim3((unsigned)nb), dim3(CMP_NT), 0, c.stream, flags, n, part);
  LAUNCHCHECK();
  scan<int64_t, int64_t>(c, part, part, nb, false, count_dev, 1);
  hipLaunchKernelGGL(k_flag_scatter, dim3((unsigned)nb), dim3(CMP_NT), 0, c.stream, flags, n, part, list,
                     (int)clear);
  LAUNCHCHECK();
}

// ------------------------------------------------------------- radix sort

constexpr int RS_NT = 256;
constexpr int RS_BITS = 8;
constexpr int RS_BINS = 1 << RS_BITS;

template <class K>
__global__ __launch_bounds__(RS_NT) void k_rs_hist(const K *__restrict__ keys, int64_t n, int shift,
                                                   int64_t per_block, int64_t *__restrict__ hist) {
  __shared__ int cnt[RS_BINS];
  for (int i = threadIdx.x; i < RS_BINS; i += RS_NT) cnt[i] = 0;
  __syncthreads();
  const int64_t beg = (int64_t)blockIdx.x * per_block;
  const int64_t end = beg + per_block < n ? beg + per_block : n;
  for (int64_t i = beg + threadIdx.x; i < end; i += RS_NT) {
    int d = (int)((keys[i] >> shift) & (RS_BINS - 1));
    atomicAdd(&cnt[d], 1);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < RS_BINS; d += RS_NT) hist[(int64_t)d * gridDim.x + blockIdx.x] = cnt[d];
}

// Stable scatter: every block walks its contiguous range in order, in tiles
// of RS_TILE keys.  Wave w of the block takes the w-th contiguous part of a
// tile (RS_IPT rows of 64 keys, lane l holding key row * 64 + l), so the
// order (wave, row, lane) is the input order.  A wave ranks its keys among
// equal digits by itself: per row, the lanes of one digit find each other
// with RS_BITS ballots, and a per-wave LDS counter per digit carries the
// count of earlier rows (one wave executes its LDS reads and writes in
// program order, so no barrier is needed inside the row loop).  The tile
// start of each digit and each wave's offset inside it then come from one
// scan over the per-wave counts; keys are placed in LDS in digit order and
// written out run by run, so consecutive threads store consecutive addresses
// of one digit's output range.
constexpr int RS_IPT = 8;
constexpr int RS_TILE = RS_NT * RS_IPT;
static_assert(RS_NT == RS_BINS, "one thread per digit in the per-tile scan");

template <class K, class V, bool HASV>
__global__ __launch_bounds__(RS_NT) void k_rs_scatter(const K *__restrict__ keys, const V *__restrict__ vals,
                                                      K *__restrict__ okeys, V *__restrict__ ovals, int64_t n,
                                                      int shift, int64_t per_block,
                                                      const int64_t *__restrict__ offs) {
  constexpr int NW = RS_NT / WAVE;
  constexpr int WKEYS = RS_IPT * WAVE;  // keys of one wave's part of a tile
  __shared__ int64_t base[RS_BINS];     // output position of the block's next key of digit d
  __shared__ int cnt[RS_BINS];          // keys of digit d in the tile
  __shared__ int tstart[RS_BINS];       // first tile slot of digit d
  __shared__ int wcnt[NW][RS_BINS];     // per wave: keys of digit d so far, then the wave's offset
  __shared__ K sk[RS_TILE];
  __shared__ V sv[HASV ? RS_TILE : 1];
  const int t = threadIdx.x, w = t / WAVE, l = lane_id();
  for (int d = t; d < RS_BINS; d += RS_NT) base[d] = offs[(int64_t)d * gridDim.x + blockIdx.x];
  const int64_t beg = (int64_t)blockIdx.x * per_block;
  const int64_t end = beg + per_block < n ? beg + per_block : n;
  const uint64_t lt = __lanemask_lt();
  for (int64_t tb = beg; tb < end; tb += RS_TILE) {
    const int tn = (int)(end - tb < RS_TILE ? end - tb : RS_TILE);
    for (int d = t; d < RS_BINS; d += RS_NT)
      for (int q = 0; q < NW; q++) wcnt[q][d] = 0;
    __syncthreads();
    K key[RS_IPT];
    int rank[RS_IPT];
#pragma unroll
    for (int j = 0; j < RS_IPT; j++) {
      const int r = w * WKEYS + j * WAVE + l;
      const bool valid = r < tn;
      key[j] = valid ? keys[tb + r] : (K)0;
      const int d = (int)((key[j] >> shift) & (RS_BINS - 1));
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < RS_BITS; b++) {
        const uint64_t bb = __ballot((d >> b) & 1);
        peers &= ((d >> b) & 1) ? bb : ~bb;
      }
      const int below = __popcll(peers & lt);
      const int before = valid ? wcnt[w][d] : 0;
      rank[j] = before + below;
      if (valid && below == __popcll(peers) - 1) wcnt[w][d] = before + below + 1;
    }
    __syncthreads();
    // per digit: the tile count, and each wave's offset among the digit's keys
    int c = 0;
    if (t < RS_BINS)
      for (int q = 0; q < NW; q++) {
        const int x = wcnt[q][t];
        wcnt[q][t] = c;
        c += x;
      }
    {
      int tot;
      const int pre = block_excl_scan<int, RS_NT>(t < RS_BINS ? c : 0, &tot);
      if (t < RS_BINS) {
        tstart[t] = pre;
        cnt[t] = c;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RS_IPT; j++) {
      const int r = w * WKEYS + j * WAVE + l;
      if (r < tn) {
        const int d = (int)((key[j] >> shift) & (RS_BINS - 1));
        const int pos = tstart[d] + wcnt[w][d] + rank[j];
        sk[pos] = key[j];
        if constexpr (HASV) sv[pos] = vals[tb + r];
      }
    }
    __syncthreads();
    for (int p = t; p < tn; p += RS_NT) {
      const K k2 = sk[p];
      const int d = (int)((k2 >> shift) & (RS_BINS - 1));
      const int64_t at = base[d] + (p - tstart[d]);
      okeys[at] = k2;
      if constexpr (HASV) ovals[at] = sv[p];
    }
    __syncthreads();
    for (int d = t; d < RS_BINS; d += RS_NT) base[d] += cnt[d];
  }
}

// Stable LSD sort of n keys on bits [lo, bits), carrying vals when HASV.
// Sorts between (keys, vals) and (tk, tv); returns true when the sorted data
// ended in (tk, tv).
template <class K, class V, bool HASV>
bool radix_sort(Ctx &c, K *keys, V *vals, K *tk, V *tv, int64_t n, int bits, const char *tag = "rs", int lo = 0) {
  if (n <= 1 || bits <= lo) return false;
  int64_t P = cdiv(n, 4096);
  int64_t maxP = (int64_t)c.num_cu * 8;
  if (P > maxP) P = maxP;
  if (P < 1) P = 1;
  int64_t per = cdiv(cdiv(n, P), RS_NT) * RS_NT;
  P = cdiv(n, per);
  int64_t *hist = c.buf<int64_t>(std::string(tag) + ".hist", (size_t)(P * RS_BINS));
  bool flip = false;
  K *ka = keys, *kb = tk;
  V *va = vals, *vb = tv;
  for (int shift = lo; shift < bits; shift += RS_BITS) {
    hipLaunchKernelGGL((k_rs_hist<K>), dim3((unsigned)P), dim3(RS_NT), 0, c.stream, ka, n, shift, per, hist);
    LAUNCHCHECK();
    scan<int64_t, int64_t>(c, hist, hist, P * RS_BINS, false, (int64_t *)nullptr, 1);
    hipLaunchKernelGGL((k_rs_scatter<K, V, HASV>), dim3((unsigned)P), dim3(RS_NT), 0, c.stream, ka, va, kb, vb,
                       n, shift, per, hist);
    LAUNCHCHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
    flip = !flip;
  }
  return flip;
}

inline int bits_for(int64_t maxval) {
  int b = 0;
  while (b < 63 && ((int64_t)1 << b) <= maxval) b++;
  return b;
}

}  // namespace lcc
