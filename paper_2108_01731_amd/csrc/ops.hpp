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
};

// Best-Moves on graph g from clustering C (device, updated in place).  On
// return K (device, owned by the context as "bm.K") holds the cluster totals
// of C.
void best_moves(Ctx &c, const lcc_graph &g, int64_t p, int64_t q, const lcc_params &prm, int32_t level,
                int32_t phase, int32_t *C, const BMShape &shape, lcc_bm_stats &st);

// Compress g by C into `out` (library-owned arrays); map (device int32[n]).
// `wide` selects int64 output weights (else int32).
void compress_graph(Ctx &c, const lcc_graph &g, const int32_t *C, OwnedGraph &out, int32_t *map, bool wide,
                    int64_t *maxdeg_out);

// Exact objective numerator of clustering C (ids in [0, n)).
i128 objective_num(Ctx &c, const lcc_graph &g, int64_t p, int64_t q, const int32_t *C);

// labels[v] = rank of C[v]'s cluster in the order of smallest members.
// Returns the number of clusters.
int64_t canonical_labels(Ctx &c, int64_t n, const int32_t *C, int32_t *labels);

// Per-cluster sums of k and kk (kk = k^2 when absent) for ids in [0, n).
void cluster_sums_k_kk(Ctx &c, const lcc_graph &g, const int32_t *C, int64_t *K, int64_t *KK);

// Largest row length of a CSR offset array.
int64_t max_degree(Ctx &c, const int64_t *off, int64_t n);

// C[v] = Cnext[map[v]] for v < n.
void flatten(Ctx &c, int64_t n, const int32_t *map, const int32_t *Cnext, int32_t *C);

// C[v] = v.
void iota_i32(Ctx &c, int32_t *C, int64_t n);

}  // namespace lcc
