// noalloc.hip -- the allocation-free objective behind lcc_objective_noalloc.
//
// Callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc) get lcc_objective's
// checks and exact result with every scratch array inside one static device
// array of this file, `scratch`, sized for graphs of at most
// LCC_NOALLOC_MAX_N vertices.  The kernels are lcc_objective's validation
// passes and objective partials; the per-cluster sums of k and kk come from
// integer atomics into two n-entry arrays (the sorting path of lcc_objective
// needs n-sized ping-pong buffers), and one-block kernels combine the block
// rows so that the host reads back a handful of values.
//
// Each device holds its own copy of the array at its own address.  In host
// code the array's name is only a stand-in: noalloc_setup asks the runtime
// for the device address once per device (lcc_ctx_create calls it with the
// device current) and every launch takes that address.  All calls on one
// device share the array, and each call clears what must start at zero, so
// calls that overlap on one device race.
#include <mutex>

#include "ops.hpp"
#include "prims.hpp"

namespace lcc {

constexpr int64_t NA_MAX_N = LCC_NOALLOC_MAX_N;
constexpr int64_t NA_BLOCKS = 1024;  // blocks of the row passes (grid-stride loops)
constexpr int NA_NT = 256;
constexpr int NA_MAX_DEVICES = 64;

// Byte offsets inside the array: K and KK (int64 per cluster id), the rows
// of the two validation passes, the objective partials, then the combined
// rows (each region 16-byte aligned).
constexpr size_t NA_K = 0;
constexpr size_t NA_KK = NA_K + sizeof(int64_t) * NA_MAX_N;
constexpr size_t NA_VROWS = NA_KK + sizeof(int64_t) * NA_MAX_N;
constexpr size_t NA_AROWS = NA_VROWS + sizeof(uint64_t) * VAL_VROW * NA_BLOCKS;
constexpr size_t NA_OPART = NA_AROWS + sizeof(uint64_t) * VAL_AROW * NA_BLOCKS;
constexpr size_t NA_TOTV = NA_OPART + sizeof(u128) * 3 * NA_BLOCKS;
constexpr size_t NA_TOTA = NA_TOTV + 64;
constexpr size_t NA_TOTO = NA_TOTA + 64;
constexpr size_t NA_BYTES = NA_TOTO + sizeof(u128) * 3;
static_assert(NA_OPART % 16 == 0 && NA_TOTO % 16 == 0, "u128 regions must be 16-byte aligned");
static_assert(sizeof(uint64_t) * VAL_VROW <= 64 && sizeof(uint64_t) * VAL_AROW <= 64, "combined rows fit");

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

static std::mutex na_mu;
static void *na_ptr[NA_MAX_DEVICES] = {};

void noalloc_setup(int device) {
  if (device < 0 || device >= NA_MAX_DEVICES) fail(LCC_ERR_UNSUPPORTED, "device index beyond the no-allocation table");
  std::lock_guard<std::mutex> lk(na_mu);
  if (na_ptr[device]) return;
  void *p = nullptr;
  HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) fail(LCC_ERR_DEVICE, "the no-allocation scratch has no device address");
  na_ptr[device] = p;
}

static unsigned char *na_base(int device) {
  std::lock_guard<std::mutex> lk(na_mu);
  if (device < 0 || device >= NA_MAX_DEVICES || !na_ptr[device])
    fail(LCC_ERR_DEVICE, "the no-allocation scratch was not set up on this device");
  return static_cast<unsigned char *>(na_ptr[device]);
}

__global__ void k_na_zero(int64_t *__restrict__ a, int64_t *__restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    a[i] = 0;
    b[i] = 0;
  }
}

// K[x] = sum of k and KK[x] = sum of kk (k^2 when absent) over C[v] = x.
__global__ void k_na_cluster_sums(const int32_t *__restrict__ C, const int64_t *__restrict__ k,
                                  const int64_t *__restrict__ kk, int64_t n, int64_t *__restrict__ K,
                                  int64_t *__restrict__ KK) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = C[v];
    const int64_t kv = k[v];
    if (kv) atomic_add_i64(&K[x], kv);
    const int64_t q = kk ? kk[v] : kv * kv;
    if (q) atomic_add_i64(&KK[x], q);
  }
}

// One block: the nb rows of `width` values (VAL_VROW: vertex pass, VAL_AROW:
// arc pass) combined into out.
__global__ __launch_bounds__(NA_NT) void k_na_combine_rows(const uint64_t *__restrict__ rows, int64_t nb, int width,
                                                           uint64_t *__restrict__ out) {
  __shared__ uint64_t acc[NA_NT][VAL_VROW];
  uint64_t a[VAL_VROW] = {0};
  for (int64_t b = threadIdx.x; b < nb; b += NA_NT) {
    if (width == VAL_VROW) combine_vertex_row(a, rows + b * VAL_VROW);
    else combine_arc_row(a, rows + b * VAL_AROW);
  }
  for (int j = 0; j < VAL_VROW; j++) acc[threadIdx.x][j] = a[j];
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t r[VAL_VROW] = {0};
    for (int i = 0; i < NA_NT; i++) {
      if (width == VAL_VROW) combine_vertex_row(r, acc[i]);
      else combine_arc_row(r, acc[i]);
    }
    for (int j = 0; j < width; j++) out[j] = r[j];
  }
}

// One block: the three groups of nb objective partials summed into out[0..2].
__global__ __launch_bounds__(NA_NT) void k_na_combine_objective(const u128 *__restrict__ part, int64_t nb,
                                                                u128 *__restrict__ out) {
  __shared__ i128 acc[3][NA_NT];
  i128 a0 = 0, a1 = 0, a2 = 0;
  for (int64_t b = threadIdx.x; b < nb; b += NA_NT) {
    a0 += (i128)part[b];
    a1 += (i128)part[nb + b];
    a2 += (i128)part[2 * nb + b];
  }
  acc[0][threadIdx.x] = a0;
  acc[1][threadIdx.x] = a1;
  acc[2][threadIdx.x] = a2;
  __syncthreads();
  if (threadIdx.x < 3) {
    i128 t = 0;
    for (int i = 0; i < NA_NT; i++) t += acc[threadIdx.x][i];
    out[threadIdx.x] = (u128)t;
  }
}

i128 objective_num_noalloc(Ctx &c, const lcc_graph &g, int64_t p, int64_t q, const int32_t *C) {
  const int64_t n = g.n;
  if (n > NA_MAX_N)
    fail(LCC_ERR_INVALID_ARG, "n = " + std::to_string(n) + " exceeds LCC_NOALLOC_MAX_N = " +
                                  std::to_string(NA_MAX_N) + " of the allocation-free objective");
  if (n == 0) return 0;
  unsigned char *base = na_base(c.device);
  int64_t *K = reinterpret_cast<int64_t *>(base + NA_K);
  int64_t *KK = reinterpret_cast<int64_t *>(base + NA_KK);
  uint64_t *vrows = reinterpret_cast<uint64_t *>(base + NA_VROWS);
  uint64_t *arows = reinterpret_cast<uint64_t *>(base + NA_AROWS);
  u128 *opart = reinterpret_cast<u128 *>(base + NA_OPART);
  uint64_t *totv = reinterpret_cast<uint64_t *>(base + NA_TOTV);
  uint64_t *tota = reinterpret_cast<uint64_t *>(base + NA_TOTA);
  u128 *toto = reinterpret_cast<u128 *>(base + NA_TOTO);
  const int64_t nb = std::min<int64_t>(cdiv(n, NA_NT), NA_BLOCKS);

  // validation as in lcc_objective: vertex pass, then (offsets usable) arcs
  GraphSummary s;
  launch_validate_vertices(c.stream, g, C, nb, vrows);
  hipLaunchKernelGGL(k_na_combine_rows, dim3(1), dim3(NA_NT), 0, c.stream, (const uint64_t *)vrows, nb,
                     (int)VAL_VROW, totv);
  LAUNCHCHECK();
  uint64_t rv[VAL_VROW] = {0};
  d2h(c, rv, totv, sizeof(rv));
  if (!summary_from_vertex_row(rv, s)) fail(LCC_ERR_INVALID_ARG, s.why);
  if (g.arcs > 0) {
    launch_validate_arcs(c.stream, g, true, nb, arows);
    hipLaunchKernelGGL(k_na_combine_rows, dim3(1), dim3(NA_NT), 0, c.stream, (const uint64_t *)arows, nb,
                       (int)VAL_AROW, tota);
    LAUNCHCHECK();
    uint64_t ra[VAL_AROW] = {0};
    d2h(c, ra, tota, sizeof(ra));
    summary_from_arc_row(ra, true, s);
    if (!s.ok) fail(LCC_ERR_INVALID_ARG, s.why);
  }
  std::string why;
  if (overflow_bounds(s, p, q, &why) != LCC_OK) fail(LCC_ERR_OVERFLOW, why);

  const unsigned grid = (unsigned)std::min<int64_t>(cdiv(n, NA_NT), NA_BLOCKS);
  hipLaunchKernelGGL(k_na_zero, dim3(grid), dim3(NA_NT), 0, c.stream, K, KK, n);
  LAUNCHCHECK();
  hipLaunchKernelGGL(k_na_cluster_sums, dim3(grid), dim3(NA_NT), 0, c.stream, C, g.k, g.kk, n, K, KK);
  LAUNCHCHECK();
  launch_objective_partials(c.stream, g, C, K, KK, nb, opart);
  hipLaunchKernelGGL(k_na_combine_objective, dim3(1), dim3(NA_NT), 0, c.stream, (const u128 *)opart, nb, toto);
  LAUNCHCHECK();
  u128 t[3];
  d2h(c, t, toto, sizeof(t));
  return objective_from_sums(p, q, (i128)t[0], (i128)t[1], (i128)t[2]);
}

}  // namespace lcc
