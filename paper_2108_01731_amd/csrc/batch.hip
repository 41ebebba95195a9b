// batch.hip -- kernels for batched runs: many independent jobs packed
// block-diagonally into one graph (job j owns vertices [start_j, start_{j+1})
// and its arcs stay inside that range).  Per-job sums are formed per chunk of
// at most BATCH_CHUNK vertices (a chunk never spans two jobs) and combined
// per job on the host, so no job's result depends on its neighbours in the
// batch.
#include "ops.hpp"
#include "prims.hpp"

namespace lcc {

constexpr int BT_NT = 256;

__global__ void k_fill_jid(const int64_t *__restrict__ jstart, int64_t jobs, int64_t n, int32_t *__restrict__ jid) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = jobs - 1;
    while (lo < hi) {  // last job whose start <= v
      const int64_t mid = (lo + hi + 1) >> 1;
      if (jstart[mid] <= v) lo = mid;
      else hi = mid - 1;
    }
    jid[v] = (int32_t)lo;
  }
}


template <class T, class F> __device__ __forceinline__ T block_reduce(T x, F op) {
  __shared__ T red[BT_NT / WAVE];
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) x = op(x, __shfl_xor(x, o, WAVE));
  if (lane_id() == 0) red[threadIdx.x / WAVE] = x;
  __syncthreads();
  T r = red[0];
  for (int i = 1; i < BT_NT / WAVE; i++) r = op(r, red[i]);
  __syncthreads();
  return r;
}

// Per chunk: sum |w| over the rows (saturating), sum k, sum kk (k^2 when
// absent), sum |s|, negative-weight flag, and a flag for arcs that leave the
// job.  part[chunk * 6 + i].  Unit weights without `check` skip the arcs.
template <int WK>
__global__ __launch_bounds__(BT_NT) void k_job_vsums(const int64_t *__restrict__ chunks, const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ col, const void *__restrict__ wt,
                                                     const int64_t *__restrict__ k, const int64_t *__restrict__ kk,
                                                     const int64_t *__restrict__ s, const int64_t *__restrict__ jstart,
                                                     int check, uint64_t *__restrict__ part) {
  const int64_t job = chunks[3 * blockIdx.x], vb = chunks[3 * blockIdx.x + 1], ve = chunks[3 * blockIdx.x + 2];
  const int64_t lo = jstart[job], hi = jstart[job + 1];
  uint64_t wabs = 0, kt = 0, kks = 0, sabs = 0, neg = 0, cross = 0;
  // one wave per vertex, lanes stride the row
  const int lane = lane_id();
  for (int64_t v = vb + threadIdx.x / WAVE; v < ve; v += BT_NT / WAVE) {
    if (WK == LCC_WT_UNIT && !check) {
      if (lane == 0) wabs = sat_add(wabs, (uint64_t)(off[v + 1] - off[v]));
    } else {
      for (int64_t e = off[v] + lane; e < off[v + 1]; e += WAVE) {
        const int32_t u = col[e];
        if ((int64_t)u < lo || (int64_t)u >= hi) cross = 1;
        const int64_t w = load_w<WK>(wt, e);
        if (w < 0) {
          neg = 1;
          wabs = sat_add(wabs, w == INT64_MIN ? (1ull << 63) : (uint64_t)(-w));
        } else {
          wabs = sat_add(wabs, (uint64_t)w);
        }
      }
    }
    if (lane == 0) {
      const uint64_t kv = (uint64_t)k[v];
      kt = sat_add(kt, kv);
      kks = sat_add(kks, kk ? (uint64_t)kk[v] : (kv > 0xFFFFFFFFull ? ~0ull : kv * kv));
      if (s) {
        const int64_t sv = s[v];
        if (sv < 0) neg = 1;
        sabs = sat_add(sabs, sv < 0 ? (sv == INT64_MIN ? (1ull << 63) : (uint64_t)(-sv)) : (uint64_t)sv);
      }
    }
  }
  auto sat = [](uint64_t a, uint64_t b) { return sat_add(a, b); };
  auto orr = [](uint64_t a, uint64_t b) { return a | b; };
  wabs = block_reduce<uint64_t>(wabs, sat);
  kt = block_reduce<uint64_t>(kt, sat);
  kks = block_reduce<uint64_t>(kks, sat);
  sabs = block_reduce<uint64_t>(sabs, sat);
  neg = block_reduce<uint64_t>(neg, orr);
  cross = block_reduce<uint64_t>(cross, orr);
  if (threadIdx.x == 0) {
    uint64_t *o = part + 6 * (int64_t)blockIdx.x;
    o[0] = wabs;
    o[1] = kt;
    o[2] = kks;
    o[3] = sabs;
    o[4] = neg;
    o[5] = cross;
  }
}

// C[v] = Cn[map[v]] moved from the job's range at the coarser level to its
// range at this level (job-local ids are what the job alone would hold);
// vertices with map < 0 (jobs that stopped coarsening here) keep C[v].
__global__ void k_flatten_jobs(const int32_t *__restrict__ map, const int32_t *__restrict__ Cn,
                               const int32_t *__restrict__ jid, const int64_t *__restrict__ jbase,
                               const int64_t *__restrict__ jbase_next, int64_t n, int32_t *__restrict__ C) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t m = map[v];
    if (m < 0) continue;
    const int32_t j = jid[v];
    C[v] = (int32_t)((int64_t)Cn[m] - jbase_next[j] + jbase[j]);
  }
}

// labels[v] = global label - global label of the job's first vertex.
__global__ void k_local_labels(const int32_t *__restrict__ glab, const int32_t *__restrict__ jid,
                               const int64_t *__restrict__ jstart, int64_t n, int32_t *__restrict__ labels) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    labels[v] = glab[v] - glab[jstart[jid[v]]];
}

// First global label of every non-empty job.
__global__ void k_job_first_label(const int32_t *__restrict__ glab, const int64_t *__restrict__ jstart, int64_t jobs,
                                  int32_t *__restrict__ first) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < jobs; j += (int64_t)gridDim.x * blockDim.x)
    first[j] = jstart[j] < jstart[j + 1] ? glab[jstart[j]] : -1;
}

// Per chunk of vertices: sum over arcs inside clusters of w, and sum of s
// (objective, Sec. 2).  part[2 * chunk + {0, 1}] as 128-bit integers.
template <int WK>
__global__ __launch_bounds__(BT_NT) void k_job_obj_intra(const int64_t *__restrict__ chunks,
                                                         const int64_t *__restrict__ off, const int32_t *__restrict__ col,
                                                         const void *__restrict__ wt, const int64_t *__restrict__ s,
                                                         const int32_t *__restrict__ C, u128 *__restrict__ part) {
  const int64_t vb = chunks[3 * blockIdx.x + 1], ve = chunks[3 * blockIdx.x + 2];
  __shared__ i128 rw[BT_NT], rs[BT_NT];
  i128 aw = 0, as = 0;
  const int lane = lane_id();
  for (int64_t v = vb + threadIdx.x / WAVE; v < ve; v += BT_NT / WAVE) {
    const int32_t cv = C[v];
    for (int64_t e = off[v] + lane; e < off[v + 1]; e += WAVE)
      if (C[col[e]] == cv) aw += load_w<WK>(wt, e);
    if (lane == 0 && s) as += s[v];
  }
  rw[threadIdx.x] = aw;
  rs[threadIdx.x] = as;
  __syncthreads();
  if (threadIdx.x == 0) {
    i128 tw = 0, ts = 0;
    for (int i = 0; i < BT_NT; i++) {
      tw += rw[i];
      ts += rs[i];
    }
    part[2 * (int64_t)blockIdx.x] = (u128)tw;
    part[2 * (int64_t)blockIdx.x + 1] = (u128)ts;
  }
}

// Per chunk of cluster ids: sum of K_X^2 - KK_X.
__global__ __launch_bounds__(BT_NT) void k_job_obj_pairs(const int64_t *__restrict__ chunks,
                                                         const int64_t *__restrict__ K, const int64_t *__restrict__ KK,
                                                         u128 *__restrict__ part) {
  const int64_t xb = chunks[3 * blockIdx.x + 1], xe = chunks[3 * blockIdx.x + 2];
  __shared__ i128 r[BT_NT];
  i128 a = 0;
  for (int64_t x = xb + threadIdx.x; x < xe; x += BT_NT) {
    const i128 kx = K[x];
    a += kx * kx - (i128)KK[x];
  }
  r[threadIdx.x] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    i128 t = 0;
    for (int i = 0; i < BT_NT; i++) t += r[i];
    part[blockIdx.x] = (u128)t;
  }
}

// ------------------------------------------------------------------- host

static unsigned bt_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 65536)); }

void batch_fill_jid(Ctx &c, const int64_t *jstart, int64_t jobs, int64_t n, int32_t *jid) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_jid, dim3(bt_grid(n)), dim3(256), 0, c.stream, jstart, jobs, n, jid);
  LAUNCHCHECK();
}

std::vector<uint64_t> batch_vertex_sums(Ctx &c, const lcc_graph &g, const int64_t *jstart,
                                        const std::vector<int64_t> &chunks, bool check_arcs) {
  const int64_t nc = (int64_t)chunks.size() / 3;
  std::vector<uint64_t> h((size_t)(6 * nc), 0);
  if (nc == 0) return h;
  int64_t *dch = c.buf<int64_t>("bt.vchunks", chunks.size());
  h2d(c, dch, chunks.data(), chunks.size() * sizeof(int64_t));
  uint64_t *part = c.buf<uint64_t>("bt.vsums", (size_t)(6 * nc));
  switch (g.wt_kind) {
    case LCC_WT_UNIT:
      hipLaunchKernelGGL((k_job_vsums<LCC_WT_UNIT>), dim3((unsigned)nc), dim3(BT_NT), 0, c.stream, dch, g.off, g.col,
                         g.wt, g.k, g.kk, g.s, jstart, (int)check_arcs, part);
      break;
    case LCC_WT_I16:
      hipLaunchKernelGGL((k_job_vsums<LCC_WT_I16>), dim3((unsigned)nc), dim3(BT_NT), 0, c.stream, dch, g.off, g.col,
                         g.wt, g.k, g.kk, g.s, jstart, (int)check_arcs, part);
      break;
    case LCC_WT_I32:
      hipLaunchKernelGGL((k_job_vsums<LCC_WT_I32>), dim3((unsigned)nc), dim3(BT_NT), 0, c.stream, dch, g.off, g.col,
                         g.wt, g.k, g.kk, g.s, jstart, (int)check_arcs, part);
      break;
    default:
      hipLaunchKernelGGL((k_job_vsums<LCC_WT_I64>), dim3((unsigned)nc), dim3(BT_NT), 0, c.stream, dch, g.off, g.col,
                         g.wt, g.k, g.kk, g.s, jstart, (int)check_arcs, part);
  }
  LAUNCHCHECK();
  d2h(c, h.data(), part, h.size() * sizeof(uint64_t));
  return h;
}

void batch_flatten(Ctx &c, int64_t n, const int32_t *map, const int32_t *Cnext, const int32_t *jid,
                   const int64_t *jbase, const int64_t *jbase_next, int32_t *C) {
  if (n <= 0) return;
  Ctx::Timer tm(&c, "flatten", 28.0 * (double)n, (double)n);
  hipLaunchKernelGGL(k_flatten_jobs, dim3(bt_grid(n)), dim3(256), 0, c.stream, map, Cnext, jid, jbase, jbase_next, n,
                     C);
  LAUNCHCHECK();
}

void batch_local_labels(Ctx &c, const int32_t *glab, const int32_t *jid, const int64_t *jstart, int64_t n,
                        int32_t *labels) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_local_labels, dim3(bt_grid(n)), dim3(256), 0, c.stream, glab, jid, jstart, n, labels);
  LAUNCHCHECK();
}

std::vector<int32_t> batch_first_labels(Ctx &c, const int32_t *glab, const int64_t *jstart, int64_t jobs) {
  std::vector<int32_t> h((size_t)jobs);
  int32_t *d = c.buf<int32_t>("bt.firstlab", (size_t)jobs);
  hipLaunchKernelGGL(k_job_first_label, dim3(bt_grid(jobs)), dim3(256), 0, c.stream, glab, jstart, jobs, d);
  LAUNCHCHECK();
  d2h(c, h.data(), d, h.size() * sizeof(int32_t));
  return h;
}

void batch_objective_parts(Ctx &c, const lcc_graph &g, const int32_t *C, const std::vector<int64_t> &vchunks,
                           const int64_t *K, const int64_t *KK, const std::vector<int64_t> &cchunks,
                           std::vector<i128> &intra, std::vector<i128> &self, std::vector<i128> &pairs) {
  const int64_t nv = (int64_t)vchunks.size() / 3, nc = (int64_t)cchunks.size() / 3;
  intra.assign((size_t)nv, 0);
  self.assign((size_t)nv, 0);
  pairs.assign((size_t)nc, 0);
  if (nv > 0) {
    int64_t *dch = c.buf<int64_t>("bt.vchunks", vchunks.size());
    h2d(c, dch, vchunks.data(), vchunks.size() * sizeof(int64_t));
    u128 *part = c.buf<u128>("bt.objv", (size_t)(2 * nv));
    switch (g.wt_kind) {
      case LCC_WT_UNIT:
        hipLaunchKernelGGL((k_job_obj_intra<LCC_WT_UNIT>), dim3((unsigned)nv), dim3(BT_NT), 0, c.stream, dch, g.off,
                           g.col, g.wt, g.s, C, part);
        break;
      case LCC_WT_I16:
        hipLaunchKernelGGL((k_job_obj_intra<LCC_WT_I16>), dim3((unsigned)nv), dim3(BT_NT), 0, c.stream, dch, g.off,
                           g.col, g.wt, g.s, C, part);
        break;
      case LCC_WT_I32:
        hipLaunchKernelGGL((k_job_obj_intra<LCC_WT_I32>), dim3((unsigned)nv), dim3(BT_NT), 0, c.stream, dch, g.off,
                           g.col, g.wt, g.s, C, part);
        break;
      default:
        hipLaunchKernelGGL((k_job_obj_intra<LCC_WT_I64>), dim3((unsigned)nv), dim3(BT_NT), 0, c.stream, dch, g.off,
                           g.col, g.wt, g.s, C, part);
    }
    LAUNCHCHECK();
    std::vector<u128> h((size_t)(2 * nv));
    d2h(c, h.data(), part, h.size() * sizeof(u128));
    for (int64_t i = 0; i < nv; i++) {
      intra[(size_t)i] = (i128)h[(size_t)(2 * i)];
      self[(size_t)i] = (i128)h[(size_t)(2 * i + 1)];
    }
  }
  if (nc > 0) {
    int64_t *dcc = c.buf<int64_t>("bt.cchunks", cchunks.size());
    h2d(c, dcc, cchunks.data(), cchunks.size() * sizeof(int64_t));
    u128 *part = c.buf<u128>("bt.objc", (size_t)nc);
    hipLaunchKernelGGL(k_job_obj_pairs, dim3((unsigned)nc), dim3(BT_NT), 0, c.stream, dcc, K, KK, part);
    LAUNCHCHECK();
    std::vector<u128> h((size_t)nc);
    d2h(c, h.data(), part, h.size() * sizeof(u128));
    for (int64_t i = 0; i < nc; i++) pairs[(size_t)i] = (i128)h[(size_t)i];
  }
}

// ------------------------------------------------------------- replication

// off[j*n1 + v] = j*arcs1 + off1[v] for the J copies, and off[J*n1] = J*arcs1.
__global__ void k_rep_off(const int64_t *__restrict__ off1, int64_t n1, int64_t arcs1, int64_t J,
                          int64_t *__restrict__ off) {
  const int64_t total = J * n1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= total; i += (int64_t)gridDim.x * blockDim.x) {
    if (i == total) {
      off[i] = J * arcs1;
    } else {
      const int64_t j = i / n1;
      off[i] = j * arcs1 + off1[i - j * n1];
    }
  }
}

// col[j*arcs1 + e] = col1[e] + j*n1.
__global__ void k_rep_col(const int32_t *__restrict__ col1, int64_t arcs1, int64_t n1, int64_t J,
                          int32_t *__restrict__ col) {
  const int64_t total = J * arcs1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = i / arcs1;
    col[i] = col1[i - j * arcs1] + (int32_t)(j * n1);
  }
}

lcc_graph batch_replicate(Ctx &c, const lcc_graph &g1, int64_t J, OwnedGraph &out) {
  const int64_t n1 = g1.n, a1 = g1.arcs, n = J * n1, arcs = J * a1;
  out.n = n;
  out.arcs = arcs;
  out.wt_kind = g1.wt_kind;
  c.ensure(out.off, (size_t)(n + 1) * sizeof(int64_t));
  c.ensure(out.col, (size_t)(arcs > 0 ? arcs : 1) * sizeof(int32_t));
  const unsigned grid_v = (unsigned)std::min<int64_t>(std::max<int64_t>(1, cdiv(n + 1, BT_NT)), 65536);
  const unsigned grid_a = (unsigned)std::min<int64_t>(std::max<int64_t>(1, cdiv(arcs, BT_NT)), 65536);
  if (n1 > 0) {
    hipLaunchKernelGGL(k_rep_off, dim3(grid_v), dim3(BT_NT), 0, c.stream, g1.off, n1, a1, J, out.off.as<int64_t>());
    LAUNCHCHECK();
  } else {
    HIPCHECK(hipMemsetAsync(out.off.p, 0, sizeof(int64_t), c.stream));
  }
  if (arcs > 0) {
    hipLaunchKernelGGL(k_rep_col, dim3(grid_a), dim3(BT_NT), 0, c.stream, g1.col, a1, n1, J, out.col.as<int32_t>());
    LAUNCHCHECK();
  }
  lcc_graph g;
  std::memset(&g, 0, sizeof(g));
  g.n = n;
  g.arcs = arcs;
  g.off = out.off.as<int64_t>();
  g.col = out.col.as<int32_t>();
  g.wt_kind = g1.wt_kind;
  const size_t wb = (size_t)wt_bytes(g1.wt_kind);
  auto copies = [&](DevBuf &dst, const void *src, size_t each) {
    c.ensure(dst, each * (size_t)J);
    for (int64_t j = 0; j < J && each > 0; j++)
      HIPCHECK(hipMemcpyAsync(static_cast<char *>(dst.p) + (size_t)j * each, src, each, hipMemcpyDeviceToDevice,
                              c.stream));
    return dst.p;
  };
  if (g1.wt_kind != LCC_WT_UNIT) g.wt = copies(out.wt, g1.wt, (size_t)a1 * wb);
  g.k = static_cast<const int64_t *>(copies(out.k, g1.k, (size_t)n1 * sizeof(int64_t)));
  if (g1.s) g.s = static_cast<const int64_t *>(copies(out.s, g1.s, (size_t)n1 * sizeof(int64_t)));
  if (g1.kk) g.kk = static_cast<const int64_t *>(copies(out.kk, g1.kk, (size_t)n1 * sizeof(int64_t)));
  return g;
}

}  // namespace lcc
