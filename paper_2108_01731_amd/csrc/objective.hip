// objective.hip -- exact objective of a clustering (paper Sec. 2), summed over
// unordered pairs:  N = q*(sum s + W_in) - p * sum_X (K_X^2 - KK_X) / 2.
// K_X and KK_X come from a stable sort of the vertices by cluster and prefix-
// sum differences; the per-cluster squares and the intra-cluster arc weights
// are accumulated in 128-bit integers (block partials, summed on the host).
#include "ops.hpp"
#include "prims.hpp"

namespace lcc {

constexpr int OB_NT = 256;

// Block partial of sum over clusters x < n of (K[x]^2 - KK[x]).
__global__ __launch_bounds__(OB_NT) void k_obj_pairs(const int64_t *__restrict__ K, const int64_t *__restrict__ KK,
                                                     int64_t n, u128 *__restrict__ part) {
  __shared__ i128 red[OB_NT];
  i128 s = 0;
  for (int64_t x = (int64_t)blockIdx.x * OB_NT + threadIdx.x; x < n; x += (int64_t)gridDim.x * OB_NT) {
    const i128 kx = K[x];
    s += kx * kx - (i128)KK[x];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    i128 t = 0;
    for (int i = 0; i < OB_NT; i++) t += red[i];
    part[blockIdx.x] = (u128)t;
  }
}

// Block partial of sum over arcs inside clusters of w, plus sum of s.
template <int WK>
__global__ __launch_bounds__(OB_NT) void k_obj_intra(const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                     const void *__restrict__ wt, const int64_t *__restrict__ s,
                                                     const int32_t *__restrict__ C, int64_t n,
                                                     u128 *__restrict__ part_w, u128 *__restrict__ part_s) {
  __shared__ i128 rw[OB_NT];
  __shared__ i128 rs[OB_NT];
  i128 aw = 0, as = 0;
  // one wave per vertex, lanes stride the row
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * OB_NT + threadIdx.x) / WAVE;
  const int64_t nwaves = ((int64_t)gridDim.x * OB_NT) / WAVE;
  for (int64_t v = wave; v < n; v += nwaves) {
    const int32_t cv = C[v];
    int64_t acc = 0;
    for (int64_t e = off[v] + lane; e < off[v + 1]; e += WAVE)
      if (C[col[e]] == cv) acc += load_w<WK>(wt, e);
    aw += acc;
    if (lane == 0 && s) as += s[v];
  }
  rw[threadIdx.x] = aw;
  rs[threadIdx.x] = as;
  __syncthreads();
  if (threadIdx.x == 0) {
    i128 t = 0, u = 0;
    for (int i = 0; i < OB_NT; i++) {
      t += rw[i];
      u += rs[i];
    }
    part_w[blockIdx.x] = (u128)t;
    part_s[blockIdx.x] = (u128)u;
  }
}

void launch_objective_partials(hipStream_t stream, const lcc_graph &g, const int32_t *C, const int64_t *K,
                               const int64_t *KK, int64_t nb, u128 *part) {
  const int64_t n = g.n;
  hipLaunchKernelGGL(k_obj_pairs, dim3((unsigned)nb), dim3(OB_NT), 0, stream, K, KK, n, part);
  LAUNCHCHECK();
  switch (g.wt_kind) {
    case LCC_WT_UNIT:
      hipLaunchKernelGGL((k_obj_intra<LCC_WT_UNIT>), dim3((unsigned)nb), dim3(OB_NT), 0, stream, g.off, g.col, g.wt,
                         g.s, C, n, part + nb, part + 2 * nb);
      break;
    case LCC_WT_I16:
      hipLaunchKernelGGL((k_obj_intra<LCC_WT_I16>), dim3((unsigned)nb), dim3(OB_NT), 0, stream, g.off, g.col, g.wt,
                         g.s, C, n, part + nb, part + 2 * nb);
      break;
    case LCC_WT_I32:
      hipLaunchKernelGGL((k_obj_intra<LCC_WT_I32>), dim3((unsigned)nb), dim3(OB_NT), 0, stream, g.off, g.col, g.wt,
                         g.s, C, n, part + nb, part + 2 * nb);
      break;
    default:
      hipLaunchKernelGGL((k_obj_intra<LCC_WT_I64>), dim3((unsigned)nb), dim3(OB_NT), 0, stream, g.off, g.col, g.wt,
                         g.s, C, n, part + nb, part + 2 * nb);
  }
  LAUNCHCHECK();
}

i128 objective_from_sums(int64_t p, int64_t q, i128 pairs2, i128 win2, i128 ssum) {
  return (i128)q * (ssum + win2 / 2) - (i128)p * (pairs2 / 2);
}

ObjectiveParts objective_parts(Ctx &c, const lcc_graph &g, const int32_t *C) {
  ObjectiveParts r;
  const int64_t n = g.n;
  if (n <= 0) return r;
  Ctx::Timer tm(&c, "objective", (double)n * 36.0 + (double)g.arcs * (8.0 + wt_bytes(g.wt_kind)), (double)g.arcs);
  int64_t *K = c.buf<int64_t>("ob.K", (size_t)n);
  int64_t *KK = c.buf<int64_t>("ob.KK", (size_t)n);
  cluster_sums_k_kk(c, g, C, K, KK);
  const int64_t nb = std::min<int64_t>(cdiv(n, OB_NT), (int64_t)c.num_cu * 4);
  u128 *part = c.buf<u128>("ob.part", (size_t)(3 * nb));
  launch_objective_partials(c.stream, g, C, K, KK, nb, part);
  std::vector<u128> h((size_t)(3 * nb));
  d2h(c, h.data(), part, h.size() * sizeof(u128));
  for (int64_t i = 0; i < nb; i++) {
    r.pairs2 += (i128)h[i];
    r.win2 += (i128)h[nb + i];
    r.ssum += (i128)h[2 * nb + i];
  }
  return r;
}

i128 objective_num(Ctx &c, const lcc_graph &g, int64_t p, int64_t q, const int32_t *C) {
  const ObjectiveParts r = objective_parts(c, g, C);
  return objective_from_sums(p, q, r.pairs2, r.win2, r.ssum);
}

// ------------------------------------------- objective after a refinement

// Intra-cluster arc weight gained going from clustering P to clustering F of
// the same graph: sum over arcs u -> v of w * ([F u = F v] - [P u = P v]).
// Only arcs with a changed endpoint (F != P) contribute; the kernel walks the
// rows of the changed vertices (a wave lists the changed ones among 64
// vertices by ballot and takes their rows one after another) and counts an
// arc to an unchanged neighbor twice, once for itself and once for the
// reverse arc in that neighbor's row (the graph is symmetric with equal
// weights both ways).  Block partials in 128-bit integers.
template <int WK>
__global__ __launch_bounds__(OB_NT) void k_obj_delta(const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                     const void *__restrict__ wt, const int32_t *__restrict__ P,
                                                     const int32_t *__restrict__ F, int64_t n,
                                                     u128 *__restrict__ part) {
  __shared__ i128 red[OB_NT];
  i128 acc = 0;
  const int lane = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * OB_NT + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * OB_NT) / WAVE;
  for (int64_t v0 = wid * WAVE; v0 < n; v0 += nw * WAVE) {
    const int64_t v = v0 + lane;
    uint64_t mk = __ballot(v < n && F[v] != P[v]);
    while (mk) {
      const int j = __ffsll((unsigned long long)mk) - 1;
      mk &= mk - 1;
      const int64_t u = v0 + j;
      const int32_t fu = F[u], pu = P[u];
      int64_t a = 0;
      for (int64_t e = off[u] + lane; e < off[u + 1]; e += WAVE) {
        const int32_t x = col[e];
        const int32_t fx = F[x], px = P[x];
        const int64_t d = (int64_t)(fx == fu) - (int64_t)(px == pu);
        if (d) a += d * load_w<WK>(wt, e) * (fx != px ? 1 : 2);
      }
      acc += a;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    i128 t = 0;
    for (int i = 0; i < OB_NT; i++) t += red[i];
    part[blockIdx.x] = (u128)t;
  }
}

i128 objective_after_refine(Ctx &c, const lcc_graph &g, int64_t p, int64_t q, const int32_t *P, const int32_t *F,
                            const ObjectiveParts &before) {
  const int64_t n = g.n;
  if (n <= 0) return 0;
  Ctx::Timer tm(&c, "objective", (double)n * 32.0, (double)n);
  // the volume term of F: per-cluster sums of k and kk
  int64_t *K = c.buf<int64_t>("ob.K", (size_t)n);
  int64_t *KK = c.buf<int64_t>("ob.KK", (size_t)n);
  cluster_sums_k_kk(c, g, F, K, KK);
  const int64_t nb = std::min<int64_t>(cdiv(n, OB_NT), (int64_t)c.num_cu * 4);
  u128 *part = c.buf<u128>("ob.part", (size_t)(2 * nb));
  hipLaunchKernelGGL(k_obj_pairs, dim3((unsigned)nb), dim3(OB_NT), 0, c.stream, (const int64_t *)K,
                     (const int64_t *)KK, n, part);
  LAUNCHCHECK();
  switch (g.wt_kind) {
    case LCC_WT_UNIT:
      hipLaunchKernelGGL((k_obj_delta<LCC_WT_UNIT>), dim3((unsigned)nb), dim3(OB_NT), 0, c.stream, g.off, g.col, g.wt,
                         P, F, n, part + nb);
      break;
    case LCC_WT_I16:
      hipLaunchKernelGGL((k_obj_delta<LCC_WT_I16>), dim3((unsigned)nb), dim3(OB_NT), 0, c.stream, g.off, g.col, g.wt,
                         P, F, n, part + nb);
      break;
    case LCC_WT_I32:
      hipLaunchKernelGGL((k_obj_delta<LCC_WT_I32>), dim3((unsigned)nb), dim3(OB_NT), 0, c.stream, g.off, g.col, g.wt,
                         P, F, n, part + nb);
      break;
    default:
      hipLaunchKernelGGL((k_obj_delta<LCC_WT_I64>), dim3((unsigned)nb), dim3(OB_NT), 0, c.stream, g.off, g.col, g.wt,
                         P, F, n, part + nb);
  }
  LAUNCHCHECK();
  std::vector<u128> h((size_t)(2 * nb));
  d2h(c, h.data(), part, h.size() * sizeof(u128));
  i128 pairs2 = 0, dwin2 = 0;
  for (int64_t i = 0; i < nb; i++) {
    pairs2 += (i128)h[i];
    dwin2 += (i128)h[nb + i];
  }
  return objective_from_sums(p, q, pairs2, before.win2 + dwin2, before.ssum);
}

}  // namespace lcc
