/*
 * lcc.h -- C ABI of liblcc, a HIP (gfx950) implementation of the LambdaCC
 * parallel best-move local search and graph compression of Shi, Dhulipala,
 * Eisenstat, Lacki and Mirrokni, "Scalable Community Detection via Parallel
 * Correlation Clustering" (arXiv 2108.01731).
 *
 * Problem (paper Sec. 2): an undirected graph G = (V, E, w), non-negative
 * vertex weights k and a resolution lambda.  The rescaled weight of a pair is
 * w'_uv = w_uv - lambda*k_u*k_v on an edge and -lambda*k_u*k_v otherwise; the
 * goal is to maximize the sum of w'_uv over pairs placed in the same cluster.
 * Modularity is the case k_v = degree(v), lambda = gamma/(2m).
 *
 * All arithmetic is exact integer arithmetic.  lambda = p/q with p >= 0 and
 * q >= 1 (int64); edge weights are integers (unit, int16, int32 or int64);
 * vertex weights are int64.  Gains are compared as int64 "scores" (see
 * lcc_best_move), the objective is returned as an exact 128-bit numerator over
 * q.  The move schedule is deterministic, so every call returns bit-identical
 * results for identical inputs.
 *
 * Memory: every array argument named "device" is a pointer into the memory of
 * the GPU the context was created for (for instance the data pointer of a
 * torch.cuda tensor).  Structs passed by pointer (graph, params, stats,
 * objective) live in host memory.  The caller owns every input and every
 * fixed-size output buffer; the library owns only the graphs it returns from
 * lcc_compress (released with lcc_graph_owned_free) and its internal scratch
 * (released by lcc_ctx_destroy).  The library never frees caller memory.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 * stream).  The library enqueues its kernels on that stream and synchronizes
 * it before returning (every entry point reads small counters back to the
 * host to drive its loops), so outputs are ready when a call returns OK.
 *
 * Errors: every entry point returns an lcc_status.  LCC_ERR_INVALID_ARG and
 * LCC_ERR_OVERFLOW are detected before any output is written (argument
 * checks on the host, then one read-only validation pass on the device) and
 * leave every output untouched.  After LCC_ERR_DEVICE or
 * LCC_ERR_OUT_OF_MEMORY outputs are unspecified.  lcc_last_error() returns a
 * thread-local message describing the last failure of the calling thread.
 * No C++ exception crosses this interface.  A context may be used by one
 * host thread at a time; calls on one context must not overlap.
 */
#ifndef LCC_H
#define LCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lcc_status;
enum {
  LCC_OK = 0,
  LCC_ERR_INVALID_ARG = 1, /* bad sizes, offsets, ids, p < 0, q < 1, ... */
  LCC_ERR_OVERFLOW = 2,    /* the exact int64 bounds below do not hold */
  LCC_ERR_OUT_OF_MEMORY = 3,
  LCC_ERR_DEVICE = 4,      /* a HIP runtime call failed */
  LCC_ERR_UNSUPPORTED = 5
};

/* Edge weight storage. */
enum {
  LCC_WT_UNIT = 0, /* no weight array: every arc weighs 1 */
  LCC_WT_I16 = 1,  /* int16 per arc (e.g. Q1.15 fixed point; lambda in the same units) */
  LCC_WT_I32 = 2,  /* int32 per arc */
  LCC_WT_I64 = 3   /* int64 per arc */
};

/* Frontier rule between iterations of Best-Moves (paper Sec. 3.2.2, the two
 * ways of shrinking the set of vertices considered). */
enum {
  LCC_FRONTIER_ALL = 0,     /* every vertex is considered in every iteration */
  LCC_FRONTIER_NBR = 1,     /* neighbors of the vertices that moved in the last iteration */
  LCC_FRONTIER_CLUSTERS = 2 /* neighbors of every vertex that, at the end of the last iteration, is in a
                               cluster some vertex moved out of during it (a cluster left empty adds
                               nothing; ids are those before fresh ids are renamed) */
};

/* Why a Best-Moves call stopped. */
enum { LCC_TERM_NO_MOVES = 0, LCC_TERM_NUM_ITER = 1, LCC_TERM_STOPPED = 2 };

#define LCC_MAX_ITER_STATS 64
#define LCC_MAX_LEVELS 64

/* A graph in CSR form (paper Sec. 2), all arrays in device memory.
 *   n          vertices, 0 <= n < 2^30
 *   arcs       stored arcs = 2 x undirected edges
 *   off        int64[n+1], off[0] = 0, non-decreasing, off[n] = arcs
 *   col        int32[arcs], neighbor ids in [0, n), no self-loops; rows need
 *              not be sorted; the arc multiset must be symmetric with equal
 *              weights both ways (not checked: results on asymmetric input
 *              are deterministic but meaningless)
 *   wt         per-arc weights of type wt_kind; NULL for LCC_WT_UNIT (and
 *              allowed to be NULL for any kind when arcs == 0)
 *   k          int64[n] vertex weights, >= 0
 *   s          int64[n] self weight of each vertex (weight of the edges that a
 *              contraction folded inside it), NULL = all 0
 *   kk         int64[n] sum of k^2 over the original vertices folded into each
 *              vertex, NULL = k_v^2
 * s and kk keep the objective exact on contracted graphs; for an input graph
 * leave both NULL. */
typedef struct lcc_graph {
  int64_t n;
  int64_t arcs;
  const int64_t *off;
  const int32_t *col;
  const void *wt;
  int32_t wt_kind;
  int32_t reserved0;
  const int64_t *k;
  const int64_t *s;
  const int64_t *kk;
} lcc_graph;

/* lambda = p / q. */
typedef struct lcc_lambda {
  int64_t p;
  int64_t q;
} lcc_lambda;

/* Default and largest lcc_params.hub_limit: 7/10 of the 12288 slots of a hub
 * partition's LDS table (a partition stops claiming slots at 10240, so a
 * larger limit could let it drop clusters unnoticed). */
#define LCC_HUB_LIMIT_MAX 8601

/* Parameters.  The "semantic" fields define the result (two runs with equal
 * semantic fields and inputs return identical results); the "tuning" fields
 * never change a result. */
typedef struct lcc_params {
  /* semantic */
  int32_t S;                    /* sub-rounds per iteration, >= 1 (1 = the paper's synchronous setting) */
  int32_t num_iter;             /* iterations per Best-Moves call (the paper's num_iter, default 10) */
  uint64_t seed;                /* seeds the sub-round assignment */
  int32_t frontier;             /* LCC_FRONTIER_* */
  int32_t refine;               /* 1 = multi-level refinement (Sec. 3.2.3) */
  int32_t allow_isolate;        /* 1 = a vertex may leave for a fresh empty cluster */
  int32_t max_levels;           /* cap on the number of graphs in the hierarchy, 1..64 */
  int64_t stop_after_subrounds; /* > 0: lcc_best_move stops after this many sub-rounds */
  /* tuning */
  int32_t validate; /* 1 = run the device validation pass on input graphs (default).  0 skips its
                       per-arc checks (column range, self-loops, row order; offsets, k, kk and
                       the overflow bounds are always checked): the caller then guarantees a
                       valid graph, and a column id outside [0, n) is undefined behaviour
                       (an out-of-bounds device read) */
  int32_t timing;   /* 1 = time every kernel launch with HIP events (see lcc_ctx_kernel_stats) */
  int32_t hub_limit; /* 0 = default (LCC_HUB_LIMIT_MAX); 1 .. LCC_HUB_LIMIT_MAX: distinct clusters a
                        hash partition of a row beyond the LDS tables may hold before the call is
                        redone with global tables (lowering it forces that path, for tests); larger
                        values are rejected with LCC_ERR_INVALID_ARG */
  int32_t queue_ahead; /* 0 = automatic; k > 0: Best-Moves queues k iterations on the device between
                          two reads of its counters (an iteration queued after the one that ends the
                          call changes nothing: every vertex stays, or the frontier is empty) */
  int32_t small_level; /* 0 = default (LCC_SMALL_LEVEL_MAX); 1 .. LCC_SMALL_LEVEL_MAX: levels of at most
                          this many vertices run their iterations through the single-block partition
                          and iteration-end kernels (larger values are rejected) */
  int32_t low_merge;   /* 0 = default (32768); k > 0: a level with at most k rows of degree < 256 takes
                          them in one launch instead of one per degree bin */
  int32_t hub_row_limit; /* rows beyond the LDS tables are first aggregated one block per row, in one
                            pass, when they meet at most this many distinct clusters (the others take the
                            hash partitions): 0 = automatic (three quarters of the block's table, the
                            largest value used; larger values are lowered to it), -1 = never (every such
                            row takes the partitions); values below -1 are rejected */
  int32_t score_pruning; /* skip the cluster-total read of every candidate whose arc weight alone cannot
                            reach the score of the vertex's heaviest candidate (such a candidate can
                            neither win nor tie): 0 = automatic (on levels of at least 2^23 vertices,
                            in the kernels where it pays; in lcc_cluster_batch and lcc_sweep only when
                            a job has that many), 1 = on every level, -1 = never; other values are
                            rejected */
  /* mode (changes results) */
  int32_t async_moves; /* 1 = the paper's asynchronous setting (Sec. 3.2.1): a vertex's move is applied
                          the moment it is decided, so the other decisions of its sub-round see it or
                          not as the hardware happens to order them.  The result is a valid clustering
                          with its exact objective, but it is not deterministic and is not the oracle's
                          (the deterministic schedule above is the default, 0) */
  int32_t no_graph_replay; /* 0 = default: a small level's chunk of iterations that repeats exactly (a
                              repeated call on the same buffers) runs as one cached HIP graph; 1 = every
                              launch goes out on its own */
} lcc_params;

/* Largest lcc_params.small_level (one block of 1024 threads partitions a
 * level this size). */
#define LCC_SMALL_LEVEL_MAX 8192

/* Fills the defaults: S = 4, num_iter = 10, seed = 1, frontier = NBR,
 * refine = 1, allow_isolate = 1, max_levels = 64, stop_after_subrounds = 0,
 * validate = 1, timing = 0, and 0 (automatic) for the other tuning fields. */
void lcc_params_default(lcc_params *prm);

typedef struct lcc_bm_stats {
  int32_t iterations;         /* iterations started */
  int32_t subrounds;          /* sub-rounds executed */
  int32_t moved_any;          /* 1 if any vertex changed cluster */
  int32_t term;               /* LCC_TERM_* */
  int64_t moves;              /* vertex moves, isolations included */
  int64_t arcs_scanned;       /* sum of degrees of the vertices whose best move was computed */
  int64_t vertices_processed; /* number of best-move computations */
  int64_t candidates;         /* distinct neighbor clusters examined (own cluster included) */
  int64_t active_per_iter[LCC_MAX_ITER_STATS];
  int64_t moves_per_iter[LCC_MAX_ITER_STATS];
} lcc_bm_stats;

typedef struct lcc_objective_out {
  int64_t num_hi; /* exact numerator N = num_hi * 2^64 + num_lo (two's complement) */
  uint64_t num_lo;
  int64_t den;    /* = q; the objective is N / q */
  double value;   /* N / q rounded to double */
} lcc_objective_out;

typedef struct lcc_cluster_stats {
  int32_t levels;    /* graphs in the hierarchy */
  int32_t top_moved; /* 1 if the last level still moved (stopped by max_levels) */
  int64_t n_level[LCC_MAX_LEVELS];
  int64_t arcs_level[LCC_MAX_LEVELS];
  int32_t iters_coarsen[LCC_MAX_LEVELS];
  int32_t iters_refine[LCC_MAX_LEVELS];
  int64_t moves_total;
  int64_t arcs_scanned_total; /* best-move arcs over every level and phase */
  int64_t clusters;
  double ms_best_move; /* host wall time inside Best-Moves calls */
  double ms_compress;  /* host wall time inside compress calls */
  double ms_total;
} lcc_cluster_stats;

typedef struct lcc_ctx lcc_ctx;
typedef struct lcc_graph_owned lcc_graph_owned;

/* Device memory supplied by the caller (for instance a caching allocator such
 * as torch's) for a context's scratch and for the graphs it returns, so that
 * growing a buffer never calls hipFree, which waits for the whole device.
 *   alloc(user, bytes, stream): at least `bytes` bytes of memory of the
 *     context's device, 256-byte aligned, for work queued on `stream` (the
 *     stream of the call that needs it); NULL means out of memory
 *     (LCC_ERR_OUT_OF_MEMORY)
 *   free(user, ptr, bytes, stream): returns a block with the size and stream
 *     it was allocated for.  Before returning a block during a call, the
 *     library drains the call's stream, so nothing queued still reads it.
 * Both are called on the thread that called into the library.  A context
 * that uses one stream for all its calls suits a stream-ordered allocator
 * (blocks are reused on the stream they were allocated for). */
typedef struct lcc_allocator {
  void *(*alloc)(void *user, size_t bytes, void *stream);
  void (*free)(void *user, void *ptr, size_t bytes, void *stream);
  void *user;
} lcc_allocator;

/* Creates a context bound to HIP device `device`.  Scratch memory is
 * allocated lazily, grows to the largest graph seen, and is kept until
 * lcc_ctx_destroy.  alloc (host, nullable, copied) supplies the device
 * memory; NULL = hipMalloc / hipFree.  Graphs returned by lcc_compress are
 * freed with lcc_graph_owned_free before the context is destroyed.
 * Errors: INVALID_ARG (NULL out, alloc with a NULL callback), DEVICE. */
lcc_status lcc_ctx_create(int32_t device, const lcc_allocator *alloc, lcc_ctx **out);
lcc_status lcc_ctx_destroy(lcc_ctx *ctx);

/* Thread-local message for the last failed call on this thread ("" if none). */
const char *lcc_last_error(void);

/* Best-Moves (paper Algorithm 1, top; Sec. 3.2.1-3.2.2), from the clustering
 * in C_inout (device int32[n], cluster ids in [0, n)), at hierarchy level
 * `level` >= 0 and phase 0 (coarsening) or 1 (refinement); level and phase
 * only select the seeded sub-round assignment.
 *
 * Each iteration (at most num_iter) runs S sub-rounds.  Sub-round s holds the
 * active vertices v with mix(h ^ v) mod S == s, where mix is the SplitMix64
 * output function and h = mix(seed ^ mix(level << 33 | phase << 32 | it)).
 * Every vertex of a sub-round decides against the same snapshot of C, the
 * cluster totals K_X (sum of k) and sizes; then all its moves apply at once.
 * The decision of v in cluster c (Appendix A): with w(v,X) the weight from v
 * to cluster X,
 *   score(X)   = q*w(v,X) - p*k_v*K_X           for a neighbor cluster X != c
 *   score(c)   = q*w(v,c) - p*k_v*(K_c - k_v)   (staying)
 *   score(iso) = 0                              (a fresh empty cluster; only
 *                                               with allow_isolate and |c| >= 2)
 * q times the objective change of a move is score(target) - score(c).  The
 * best target is the highest score, ties to the lowest cluster id, iso after
 * every id; v moves only if it is strictly better than staying.  A vertex v
 * that isolates moves to the fresh cluster n + v (v is in one sub-round per
 * iteration, so that id is unused within the iteration; later sub-rounds may
 * join it); at the end of the iteration the non-empty fresh clusters, in
 * ascending id order, are renamed to the ascending ids in [0, n) that are
 * empty, so C holds ids in [0, n) between iterations and on return.  The
 * first iteration considers every vertex;
 * later ones follow params->frontier.  Stops after an iteration with no move,
 * after num_iter iterations, or after stop_after_subrounds sub-rounds.
 *
 * stats (host, nullable) receives counters.  Errors: INVALID_ARG (graph or
 * ids invalid, p < 0, q < 1, S < 1, num_iter < 0, level < 0, phase not 0/1),
 * OVERFLOW (the int64 bounds: Wabs = sum|w| over edges + sum|s|, Ktot = sum k,
 * require q*Wabs, p*Ktot, p*floor(Ktot^2/4), sum kk <= 2^63-1, and with a
 * negative weight q*Wabs + p*floor(Ktot^2/4) <= 2^63-1), DEVICE, OUT_OF_MEMORY. */
lcc_status lcc_best_move(lcc_ctx *ctx, const lcc_graph *g, lcc_lambda lam, const lcc_params *prm,
                         int32_t level, int32_t phase, int32_t *C_inout, lcc_bm_stats *stats,
                         void *stream);

/* Compress (paper Sec. 3.1 and Appendix B): one vertex per non-empty cluster
 * of C (device int32[n], ids in [0, n)), numbered by the rank of the cluster
 * id among non-empty ids; map_out (device int32[n]) receives that number for
 * every vertex.  The contracted graph has k' = sum of k, kk' = sum of kk,
 * s' = sum of s plus the weight of the edges inside the cluster, and one edge
 * per pair of adjacent clusters carrying the summed weight (kept when the sum
 * is 0); rows are sorted by neighbor id.  Its weights are int32 when the
 * input's Wabs < 2^31, else int64.  *out receives a library-owned graph
 * (read it with lcc_graph_owned_view, release it with lcc_graph_owned_free).
 * Errors: INVALID_ARG, OVERFLOW (sum bounds as above with p = 0, q = 1),
 * DEVICE, OUT_OF_MEMORY. */
lcc_status lcc_compress(lcc_ctx *ctx, const lcc_graph *g, const int32_t *C, lcc_graph_owned **out,
                        int32_t *map_out, void *stream);

/* A read-only view of an owned graph (pointers stay valid until it is freed). */
lcc_status lcc_graph_owned_view(const lcc_graph_owned *h, lcc_graph *view);
lcc_status lcc_graph_owned_free(lcc_ctx *ctx, lcc_graph_owned *h);

/* Objective (paper Sec. 2) of clustering C (device int32[n], ids in [0, n)),
 * summed over unordered pairs (the paper's V x V sum counts each pair twice
 * and equals 2*N/q):
 *   N = q*(sum_v s_v + W_in) - p * sum_X (K_X^2 - sum_{v in X} kk_v) / 2,
 * W_in = weight of the edges inside clusters.  Errors as lcc_best_move. */
lcc_status lcc_objective(lcc_ctx *ctx, const lcc_graph *g, lcc_lambda lam, const int32_t *C,
                         lcc_objective_out *out, void *stream);

/* Largest graph (vertices) that lcc_objective_noalloc accepts. */
#define LCC_NOALLOC_MAX_N 1048576

/* lcc_objective for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, checks, errors and result as lcc_objective, for graphs of
 * at most LCC_NOALLOC_MAX_N vertices; it calls no hipMalloc, hipFree or other
 * allocating routine.  Its scratch (per-cluster int64 sums for
 * LCC_NOALLOC_MAX_N ids plus block partials, 16.9 MB) is one static device
 * array of the library, which every device the library runs on holds until
 * the process ends; lcc_ctx_create looks up its address on the context's
 * device.  All calls on one device share that array, so calls that overlap
 * on one device race: the caller serializes them (one stream, or a lock).
 * Like lcc_objective it reads a few values back and synchronizes the stream.
 * Errors: as lcc_objective, plus INVALID_ARG for n > LCC_NOALLOC_MAX_N
 * (raised before any launch). */
lcc_status lcc_objective_noalloc(lcc_ctx *ctx, const lcc_graph *g, lcc_lambda lam, const int32_t *C,
                                 lcc_objective_out *out, void *stream);

/* Parallel-CC (paper Algorithm 1, bottom, with Sec. 3.2.3 refinement):
 * Best-Moves from singletons at level 0; while it moved anything and fewer
 * than max_levels graphs exist, compress and repeat on the contracted graph;
 * then walk back down, flattening each level's clustering through its map
 * (C[v] <- C'[map[v]]) and, with refine, running Best-Moves (phase 1) on it.
 * labels_out (device int32[n]) receives canonical labels: clusters numbered
 * 0, 1, ... in the order of their smallest vertex.  obj and stats (host) are
 * nullable.  Errors as lcc_best_move (plus INVALID_ARG for max_levels outside
 * 1..64). */
lcc_status lcc_cluster(lcc_ctx *ctx, const lcc_graph *g, lcc_lambda lam, const lcc_params *prm,
                       int32_t *labels_out, lcc_objective_out *obj, lcc_cluster_stats *stats,
                       void *stream);

/* Per-job result of a batched run. */
typedef struct lcc_job_out {
  lcc_objective_out obj; /* objective of the job's labels under the job's lambda */
  int64_t clusters;      /* number of clusters of the job */
  int32_t levels;        /* graphs in the job's hierarchy (as lcc_cluster_stats.levels) */
  int32_t top_moved;     /* as lcc_cluster_stats.top_moved */
} lcc_job_out;

/* Batch statistics (summed over jobs; wall times cover the whole batch). */
typedef struct lcc_batch_stats {
  int32_t levels; /* batch levels (the largest job hierarchy) */
  int32_t reserved0;
  int64_t n_level[LCC_MAX_LEVELS];    /* vertices of the packed graph at each level */
  int64_t arcs_level[LCC_MAX_LEVELS]; /* arcs of the packed graph at each level */
  int64_t moves_total;
  int64_t arcs_scanned_total;
  double ms_best_move;
  double ms_compress;
  double ms_total;
} lcc_batch_stats;

/* Parallel-CC (as lcc_cluster) on many independent jobs in shared launches.
 * g packs the jobs block-diagonally: job j owns the vertices
 * [job_start[j], job_start[j+1]) and every arc of those rows stays inside that
 * range.  job_start (host int64[jobs + 1]) is non-decreasing from 0 to g->n;
 * empty jobs are allowed.  lambdas (host, jobs entries) gives each job its
 * own resolution; prm is shared (stop_after_subrounds must be 0).
 *
 * Each job's result is the one lcc_cluster gives on that job's graph alone
 * (vertex v of job j being vertex v - job_start[j] there) with the same
 * params: the sub-round assignment hashes job-local vertex ids, a job stops
 * iterating and stops coarsening on its own conditions, isolating vertices
 * take the job's own empty ids, and compression keeps only the jobs still
 * coarsening.  labels_out (device int32[g->n]) receives each job's canonical
 * labels (0, 1, ... within the job, in the order of its smallest vertex).
 * jobs_out (host, jobs entries) and stats (host) are nullable.
 *
 * Errors: as lcc_cluster, plus INVALID_ARG (jobs < 0, job_start not a
 * partition of [0, n), an arc leaving its job, NULL job_start or lambdas,
 * stop_after_subrounds != 0) and OVERFLOW (the bounds of lcc_best_move
 * checked per job with that job's lambda). */
lcc_status lcc_cluster_batch(lcc_ctx *ctx, const lcc_graph *g, int64_t jobs, const int64_t *job_start,
                             const lcc_lambda *lambdas, const lcc_params *prm, int32_t *labels_out,
                             lcc_job_out *jobs_out, lcc_batch_stats *stats, void *stream);

/* Most resolutions one lcc_sweep call takes. */
#define LCC_SWEEP_MAX 16

/* Parallel-CC (as lcc_cluster) of ONE graph under several resolutions at
 * once: the quality experiments of Section 4.3 cluster each graph over a
 * grid of lambda values, and every value is a separate run of Algorithm 1
 * with the objective of Section 2.  Result j is exactly the result of
 * lcc_cluster(g, lambdas[j], prm) run alone.
 *
 * count (0..LCC_SWEEP_MAX) resolutions; lambdas (host, count entries); prm is
 * shared (stop_after_subrounds must be 0).  labels_out (device int32,
 * count * g->n entries) receives at offset j * g->n the canonical labels of
 * resolution j; jobs_out (host, count entries) and stats (host) are nullable.
 * The library packs count copies of g into its own device buffers (count
 * times the graph's arrays, kept until the context is destroyed or the next
 * sweep) and runs them as one batch in which the level-0 rows of degree
 * below 256 are read once for all resolutions, with the cluster ids of each
 * vertex under all resolutions held in one 64-byte line.
 *
 * Errors: as lcc_cluster_batch, plus INVALID_ARG for count outside
 * [0, LCC_SWEEP_MAX] or count * n >= 2^30; OVERFLOW names the first
 * resolution whose bounds fail. */
lcc_status lcc_sweep(lcc_ctx *ctx, const lcc_graph *g, int64_t count, const lcc_lambda *lambdas,
                     const lcc_params *prm, int32_t *labels_out, lcc_job_out *jobs_out, lcc_batch_stats *stats,
                     void *stream);

/* Per-kernel timing collected while params.timing was set (HIP events around
 * every launch, on the launch stream).  bytes is the algorithmic HBM traffic
 * the launches must move (inputs read once, outputs written once), computed
 * from counters, not measured. */
typedef struct lcc_kernel_stat {
  char name[64];
  int64_t launches;
  double total_ms;
  double bytes;
  double items; /* arcs for best-move kernels, elements for others */
} lcc_kernel_stat;

/* Copies up to max entries into out (host) and stores the number of kernel
 * classes in *count.  Errors: INVALID_ARG. */
lcc_status lcc_ctx_kernel_stats(lcc_ctx *ctx, lcc_kernel_stat *out, int32_t max, int32_t *count);
lcc_status lcc_ctx_reset_kernel_stats(lcc_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LCC_H */
