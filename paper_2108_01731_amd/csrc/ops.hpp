// ops.hpp -- host-side entry points of the kernels, shared between the
// translation units of liblcc (best-move, compress, objective, driver).
#pragma once

#include "common.hpp"

namespace lcc {

// Result of the device validation pass over a graph (and optionally a
// clustering).  Sums saturate at UINT64_MAX.
struct GraphSummary {
  bool ok = true;
  std::string why;
  uint64_t wabs2 = 0;  // sum over arcs of |w|
  uint64_t sabs = 0;   // sum of |s|
  uint64_t ktot = 0;   // sum of k
  uint64_t kksum = 0;  // sum of kk (or k^2)
  bool negative = false;
  int64_t maxdeg = 0;
  bool sorted_rows = false;  // every row strictly ascending (so no repeated neighbor)
};

// Validation pass (read-only): offsets, column range, self-loops, k >= 0,
// kk >= 0, optional cluster ids in [0, n).  Also returns the sums the
// overflow bounds need.
GraphSummary summarize_graph(Ctx &c, const lcc_graph &g, const int32_t *C, bool check_structure);

// The validation pass in pieces, for callers that bring their own scratch:
// the vertex pass writes one row of VAL_VROW values per block {error bits,
// sum k, sum kk, sum |s|, negative s, largest degree, 0, 0}, the arc pass one
// row of VAL_AROW values {error bits, sum |w|, negative w}; rows combine with
// combine_*_row (sums saturate at 2^64 - 1) and the combined rows fill a
// summary.  summary_from_vertex_row returns false when the offsets, k, kk or
// ids are unusable (the arc pass must then not run).
constexpr int VAL_VROW = 8;
constexpr int VAL_AROW = 3;

__host__ __device__ inline uint64_t sat_add(uint64_t a, uint64_t b) {
  const uint64_t s = a + b;
  return s < a ? ~0ull : s;
}
__host__ __device__ inline void combine_vertex_row(uint64_t *acc, const uint64_t *r) {
  acc[0] |= r[0];
  acc[1] = sat_add(acc[1], r[1]);
  acc[2] = sat_add(acc[2], r[2]);
  acc[3] = sat_add(acc[3], r[3]);
  acc[4] |= r[4];
  acc[5] = r[5] > acc[5] ? r[5] : acc[5];
}
__host__ __device__ inline void combine_arc_row(uint64_t *acc, const uint64_t *r) {
  acc[0] |= r[0];
  acc[1] = sat_add(acc[1], r[1]);
  acc[2] |= r[2];
}
int64_t validation_blocks(const Ctx &c, int64_t n);
void launch_validate_vertices(hipStream_t stream, const lcc_graph &g, const int32_t *C, int64_t nb, uint64_t *part);
void launch_validate_arcs(hipStream_t stream, const lcc_graph &g, bool check, int64_t nb, uint64_t *part);
bool summary_from_vertex_row(const uint64_t *r, GraphSummary &s);
void summary_from_arc_row(const uint64_t *r, bool check, GraphSummary &s);

// Checks the int64 bounds; returns LCC_OK or LCC_ERR_OVERFLOW.
lcc_status overflow_bounds(const GraphSummary &s, int64_t p, int64_t q, std::string *why);

// Per-cluster totals of a clustering with ids in [0, n): K[x] = sum of k,
// cnt[x] = members.  Deterministic, contention-free (sort + prefix sums).
void cluster_totals(Ctx &c, int64_t n, const int32_t *C, const int64_t *k, int64_t *K, int32_t *cnt);

// What Best-Moves may assume about its input (never changes a result).
struct BMShape {
  int64_t maxdeg;   // largest row length
  bool acc32;       // every row's sum of |w| is below 2^31 (32-bit accumulators)
  bool identity;    // C[v] = v on entry
  bool simple;      // no row repeats a neighbor
  int64_t mindeg = 0;  // a lower bound of the shortest row length
};

// Jobs of a batched run at one level: the graph holds the jobs' vertices
// block-diagonally in job order; jobs absent from the level have empty
// ranges.
struct BatchLevel {
  int64_t jobs = 0;
  const int32_t *jid = nullptr;    // device, job of every vertex
  const int64_t *jbase = nullptr;  // device, jobs + 1 prefix of per-job vertex counts
  const int64_t *jp = nullptr;     // device, per-job lambda
  const int64_t *jq = nullptr;
  const uint8_t *active = nullptr; // host, per job: takes part in this Best-Moves call
  int32_t *iters = nullptr;        // host out, per job: iterations started
  uint8_t *moved_any = nullptr;    // host out, per job
  // > 0: the jobs are identical copies of one graph of shared_n vertices (job
  // j owns [j * shared_n, (j + 1) * shared_n), rows shifted by j * shared_n),
  // so rows of low degree are read once for all jobs (at most 16 jobs)
  int64_t shared_n = 0;
};

// Best-Moves on graph g from clustering C (device, updated in place).  On
// return K (device, owned by the context as "bm.K") holds the cluster totals
// of C.  With `bl`, every job runs its own Best-Moves (own lambda, own
// termination) in the same launches.
void best_moves(Ctx &c, const lcc_graph &g, int64_t p, int64_t q, const lcc_params &prm, int32_t level,
                int32_t phase, int32_t *C, const BMShape &shape, lcc_bm_stats &st,
                const BatchLevel *bl = nullptr);

// Batched compress: only vertices of jobs with jcont[job] = 1 are kept
// (the others get map = -1); the jobs of the contracted vertices and the next
// level's job bases (jobs + 1 entries) are written out.
struct CompressJobs {
  int64_t jobs = 0;
  const int32_t *jid = nullptr;   // device, per vertex
  const uint8_t *jcont = nullptr; // device, per job
  int32_t *jid_next = nullptr;    // device out, per contracted vertex
  int64_t *jbase_next = nullptr;  // device out, jobs + 1
};

// Compress g by C into `out` (library-owned arrays); map (device int32[n]).
// `wide` selects int64 output weights (else int32).  maxdeg_out / mindeg_out
// (nullable) receive the longest and shortest row of the output (the
// shortest may be reported as 0 when it is not computed).
void compress_graph(Ctx &c, const lcc_graph &g, const int32_t *C, OwnedGraph &out, int32_t *map, bool wide,
                    int64_t *maxdeg_out, const CompressJobs *cj = nullptr, int64_t *mindeg_out = nullptr);

// Exact objective numerator of clustering C (ids in [0, n)).
i128 objective_num(Ctx &c, const lcc_graph &g, int64_t p, int64_t q, const int32_t *C);

// Its sums: over clusters of K^2 - KK, over intra-cluster arcs of w, of s.
struct ObjectiveParts {
  i128 pairs2 = 0, win2 = 0, ssum = 0;
};
ObjectiveParts objective_parts(Ctx &c, const lcc_graph &g, const int32_t *C);

// The objective of clustering F of g from the sums of a clustering P of the
// same graph, or of any graph P contracts to (contraction keeps s + win2 / 2
// per clustering): F's volume term is computed, and its intra-cluster
// weight is P's plus the change over the arcs of the vertices whose cluster
// differs between P and F (P and F: ids in [0, n)).
i128 objective_after_refine(Ctx &c, const lcc_graph &g, int64_t p, int64_t q, const int32_t *P, const int32_t *F,
                            const ObjectiveParts &before);

// The objective from caller-given per-cluster sums K, KK (ids in [0, n)):
// 3 * nb block partials in `part` (sum over clusters of K^2 - KK, then the
// intra-cluster arc weight, then sum s), combined by objective_from_sums.
void launch_objective_partials(hipStream_t stream, const lcc_graph &g, const int32_t *C, const int64_t *K,
                               const int64_t *KK, int64_t nb, u128 *part);
i128 objective_from_sums(int64_t p, int64_t q, i128 pairs2, i128 win2, i128 ssum);

// The allocation-free objective (lcc_objective_noalloc): every scratch array
// lives in a static device array of the library; noalloc_setup records its
// address on the current device (called once per device by lcc_ctx_create).
void noalloc_setup(int device);
i128 objective_num_noalloc(Ctx &c, const lcc_graph &g, int64_t p, int64_t q, const int32_t *C);

// labels[v] = rank of C[v]'s cluster in the order of smallest members.
// Returns the number of clusters.
int64_t canonical_labels(Ctx &c, int64_t n, const int32_t *C, int32_t *labels);

// Per-cluster sums of k and kk (kk = k^2 when absent) for ids in [0, n).
void cluster_sums_k_kk(Ctx &c, const lcc_graph &g, const int32_t *C, int64_t *K, int64_t *KK);

// Number of distinct cluster ids of C (ids in [0, n)): per job when jbase
// (device, J + 1 job bases, a job's ids inside its own range) is given, else
// one count (J = 1).
std::vector<int64_t> job_cluster_counts(Ctx &c, int64_t n, const int32_t *C, int64_t J, const int64_t *jbase);

// Largest row length of a CSR offset array (and, min_out, the smallest).
int64_t max_degree(Ctx &c, const int64_t *off, int64_t n, int64_t *min_out = nullptr);

// C[v] = Cnext[map[v]] for v < n with map[v] >= 0.
void flatten(Ctx &c, int64_t n, const int32_t *map, const int32_t *Cnext, int32_t *C);

// C[v] = v.
void iota_i32(Ctx &c, int32_t *C, int64_t n);

// ---- batched runs (jobs packed block-diagonally, job j owns [start_j, start_j+1))

// Largest vertex range handled by one block of the per-job sums; chunks are
// (job, first vertex, end vertex) triples that never span two jobs.
constexpr int64_t BATCH_CHUNK = 2048;

// jid[v] = job owning v (jstart: device, jobs + 1 entries).
void batch_fill_jid(Ctx &c, const int64_t *jstart, int64_t jobs, int64_t n, int32_t *jid);

// Per chunk: {sum |w| over arcs, sum k, sum kk (k^2 when absent), sum |s|,
// negative flag, arc-leaves-job flag}, saturating at 2^64 - 1.  Arcs are read
// when check_arcs is set or weights are stored; else sum |w| is the arc count.
std::vector<uint64_t> batch_vertex_sums(Ctx &c, const lcc_graph &g, const int64_t *jstart,
                                        const std::vector<int64_t> &chunks, bool check_arcs);

// Batched flatten: C[v] = Cnext[map[v]] - jbase_next[job] + jbase[job] for
// map[v] >= 0 (a job's ids move from its coarser range to its range here).
void batch_flatten(Ctx &c, int64_t n, const int32_t *map, const int32_t *Cnext, const int32_t *jid,
                   const int64_t *jbase, const int64_t *jbase_next, int32_t *C);

// J copies of g1 packed block-diagonally into `out` (job j: vertices
// shifted by j * g1.n, arcs by j * g1.arcs); returns the packed graph's view.
lcc_graph batch_replicate(Ctx &c, const lcc_graph &g1, int64_t J, OwnedGraph &out);

// labels[v] = glab[v] - glab[first vertex of v's job].
void batch_local_labels(Ctx &c, const int32_t *glab, const int32_t *jid, const int64_t *jstart, int64_t n,
                        int32_t *labels);

// glab of every job's first vertex (-1 for empty jobs).
std::vector<int32_t> batch_first_labels(Ctx &c, const int32_t *glab, const int64_t *jstart, int64_t jobs);

// Objective pieces per chunk: intra-cluster arc weight and sum s over vertex
// chunks of C, sum (K^2 - KK) over cluster-id chunks.
void batch_objective_parts(Ctx &c, const lcc_graph &g, const int32_t *C, const std::vector<int64_t> &vchunks,
                           const int64_t *K, const int64_t *KK, const std::vector<int64_t> &cchunks,
                           std::vector<i128> &intra, std::vector<i128> &self, std::vector<i128> &pairs);

}  // namespace lcc
