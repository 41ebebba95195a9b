/*
 * lcc_oracle.c -- plain, slow CPU reference for the LambdaCC best-move local
 * search, graph compression, objective and the multi-level driver (Shi,
 * Dhulipala, Eisenstat, Lacki, Mirrokni, "Scalable Community Detection via
 * Parallel Correlation Clustering", arXiv 2108.01731).
 *
 * It is single-threaded C.  Built with -fopenmp, the one parallel loop is the
 * per-vertex decisions of a sub-round (each thread with its own scratch):
 * those decisions read one fixed snapshot and write only their own slot, so
 * the build returns exactly what the single-threaded build returns.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity oracle: only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load it.
 * The product library never links, loads or calls it, and it shares no code,
 * header, table or helper with the GPU path.
 *
 * Everything is integer arithmetic: int64 weights, vertex weights, cluster
 * totals and gains; __int128 only for the final objective numerator.  The
 * resolution is a rational lambda = p/q (p >= 0, q >= 1), so every comparison
 * the method makes is exact.
 *
 * Paper passages this follows (cited by section / equation / algorithm):
 *   - Sec. 2 (Preliminaries): the rescaled weights w'_uv and the objective
 *     CC(x) = sum over V x V of w'_ij (1 - x_ij); modularity as the special
 *     case k_v = d_v, lambda = gamma / 2m.
 *   - Appendix A: the change in objective when v moves from c to c'.
 *   - Algorithm 1 (Best-Moves, Parallel-CC) and Sec. 3.2.1 (synchronous move
 *     application), Sec. 3.2.2 (neighbors-of-moved-vertices frontier),
 *     Sec. 3.2.3 (multi-level refinement).
 *   - Sec. 3.1 and Appendix B (compress: one vertex per cluster, k'(c) = K_c,
 *     parallel edges summed; flatten: C[v] <- C'[id(C[v])]).
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - The move schedule is synchronous over seeded subsets: in iteration `it`
 *     of a Best-Moves call at level `l`, phase `ph` (0 = coarsening, 1 =
 *     refinement), vertex v belongs to sub-round color(v) = mix(h ^ v) mod S
 *     with h = mix(seed ^ mix(l << 33 | ph << 32 | it)); mix is SplitMix64.
 *     Each sub-round decides all its vertices against one snapshot, then
 *     applies the moves together.  S = 1 is the paper's synchronous setting.
 *   - Candidates for v in cluster c: every cluster holding a neighbor of v
 *     (any arc, whatever its weight), plus "isolate" (a fresh empty cluster)
 *     when allow_isolate is set and |c| >= 2.  Best target: highest gain,
 *     ties to the lowest cluster id, isolate ranks after every id.  v moves
 *     only on a strict improvement over staying.
 *   - A vertex v that isolates moves to the fresh cluster n + v (each vertex
 *     belongs to one sub-round per iteration, so that id is unused within the
 *     iteration; other vertices may join it in later sub-rounds).  At the end
 *     of every iteration the non-empty fresh clusters, in ascending id order,
 *     are renamed to the ascending ids in [0, n) that are empty at that point,
 *     so every clustering seen between iterations uses ids in [0, n).
 *   - Frontier "neighbors of moved vertices": the union of N(v) over every v
 *     that moved in any sub-round of the iteration (v itself is not added).
 *   - Frontier "neighbors of clusters" (Sec. 3.2.2, the clusters the movers
 *     left): the union of N(u) over every u that, at the end of the
 *     iteration, belongs to a cluster some vertex moved out of during the
 *     iteration (moves in any sub-round; a cluster left empty adds nothing).
 *   - Parallel-CC recurses when the coarsening Best-Moves call changed the
 *     partition: a call that only exchanged the ids of singletons (every
 *     vertex still alone) counts as a call without moves.
 *   - Compress numbers clusters by the rank of their id among non-empty ids;
 *     self-loops of the contracted graph are kept out of the adjacency, in a
 *     per-vertex self weight s, and kk (sum of k^2 over original members) is
 *     carried so the objective stays exact at every level.
 *   - The objective reported is the unordered-pair sum (half of the V x V sum
 *     in Sec. 2), as an exact numerator over q.
 *   - Final labels: dense rank of each cluster's smallest member.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;

#define ORC_OK 0
#define ORC_INVALID 1
#define ORC_OVERFLOW 2
#define ORC_NOMEM 3

#define ORC_FRONTIER_ALL 0
#define ORC_FRONTIER_NBR 1
#define ORC_FRONTIER_CLUSTERS 2

#define ORC_TERM_NO_MOVES 0
#define ORC_TERM_NUM_ITER 1
#define ORC_TERM_STOPPED 2

#define ORC_ISO (-1)
#define ORC_MAX_ITER_STATS 64
#define ORC_MAX_LEVELS 64
#define ORC_MAX_N ((int64_t)1 << 30) /* cluster ids, fresh ones included, stay below 2^31 */

static const i128 I64LIM = (i128)INT64_MAX;

/* A graph at some level.  Rows are sorted or not; no self-loops; symmetric.
 * wt == NULL means every arc weighs 1.  s == NULL means all self weights 0;
 * kk == NULL means kk_v = k_v^2 (an uncontracted graph). */
typedef struct {
  int64_t n;
  int64_t arcs;
  const int64_t *off;
  const int32_t *col;
  const int64_t *wt;
  const int64_t *k;
  const int64_t *s;
  const int64_t *kk;
} orc_graph;

typedef struct {
  int32_t S;
  int32_t num_iter;
  uint64_t seed;
  int32_t frontier;
  int32_t refine;
  int32_t allow_isolate;
  int32_t max_levels;
  int64_t stop_after_subrounds; /* 0 = no limit */
} orc_params;

typedef struct {
  int32_t iterations;
  int32_t subrounds;
  int32_t moved_any;
  int32_t term;
  int64_t moves;
  int64_t arcs_scanned;
  int64_t vertices_processed;
  int64_t active_per_iter[ORC_MAX_ITER_STATS];
  int64_t moves_per_iter[ORC_MAX_ITER_STATS];
} orc_bm_stats;

/* A graph the oracle allocated (compress output). */
typedef struct {
  int64_t n;
  int64_t arcs;
  int64_t *off;
  int32_t *col;
  int64_t *wt;
  int64_t *k;
  int64_t *s;
  int64_t *kk;
} orc_graph_out;

typedef struct {
  int32_t levels;          /* number of graphs in the hierarchy (>= 1) */
  int32_t top_moved;       /* 1 if the top level stopped because of max_levels */
  int64_t n_level[ORC_MAX_LEVELS];
  int64_t arcs_level[ORC_MAX_LEVELS];
  int32_t iters_coarsen[ORC_MAX_LEVELS];
  int32_t iters_refine[ORC_MAX_LEVELS];
  int64_t moves_total;
  int64_t arcs_scanned_total;
  int64_t clusters;
} orc_cluster_stats;

/* ---------------------------------------------------------------- hashing */

/* SplitMix64 output function (Steele, Lea, Flood 2014; Vigna's public-domain
 * splitmix64): the state is advanced by the golden-ratio increment and then
 * scrambled by two xor-shift-multiply steps and a final xor-shift. */
uint64_t orc_mix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t orc_round_hash(uint64_t seed, int32_t level, int32_t phase, int32_t it) {
  uint64_t ctr = ((uint64_t)(uint32_t)level << 33) | ((uint64_t)(uint32_t)(phase & 1) << 32) |
                 (uint64_t)(uint32_t)it;
  return orc_mix64(seed ^ orc_mix64(ctr));
}

int32_t orc_color(uint64_t h, int64_t v, int32_t S) {
  return (int32_t)(orc_mix64(h ^ (uint64_t)v) % (uint64_t)S);
}

/* --------------------------------------------------------- graph accessors */

static int64_t W(const orc_graph *g, int64_t e) { return g->wt ? g->wt[e] : 1; }
static int64_t S_of(const orc_graph *g, int64_t v) { return g->s ? g->s[v] : 0; }
static i128 KK_of(const orc_graph *g, int64_t v) {
  return g->kk ? (i128)g->kk[v] : (i128)g->k[v] * (i128)g->k[v];
}

/* ------------------------------------------------------ validation checks */

/* Structural checks on a graph: sizes, offsets, column range, no self-loops,
 * non-negative vertex weights.  Symmetry is a precondition checked separately
 * (orc_check_symmetric) because it costs a sort. */
int orc_validate(const orc_graph *g) {
  if (!g || g->n < 0 || g->n >= ORC_MAX_N || g->arcs < 0) return ORC_INVALID;
  if (g->n > 0 && (!g->off || !g->k)) return ORC_INVALID;
  if (g->arcs > 0 && !g->col) return ORC_INVALID;
  if (g->n == 0) return g->arcs == 0 ? ORC_OK : ORC_INVALID;
  if (g->off[0] != 0 || g->off[g->n] != g->arcs) return ORC_INVALID;
  for (int64_t v = 0; v < g->n; v++) {
    if (g->off[v + 1] < g->off[v]) return ORC_INVALID;
    if (g->k[v] < 0) return ORC_INVALID;
    if (g->kk && g->kk[v] < 0) return ORC_INVALID;
    for (int64_t e = g->off[v]; e < g->off[v + 1]; e++) {
      int32_t u = g->col[e];
      if (u < 0 || (int64_t)u >= g->n || (int64_t)u == v) return ORC_INVALID;
    }
  }
  return ORC_OK;
}

/* Overflow bounds under which every gain the method forms fits in int64:
 *   Wabs = (sum over arcs |w|) / 2 + sum |s|,  Ktot = sum k,  KK = sum kk;
 *   Ktot, Wabs, KK, q*Wabs, p*Ktot, p*floor(Ktot^2/4) <= 2^63-1, and with any
 *   negative weight also q*Wabs + p*floor(Ktot^2/4) <= 2^63-1.
 * For v outside X, k_v + K_X <= Ktot so k_v*K_X <= Ktot^2/4; a row's weight
 * sum is at most Wabs.  Contraction never increases Wabs, Ktot or KK, so the
 * check made on the input graph covers every level. */
int orc_precheck(const orc_graph *g, int64_t p, int64_t q) {
  if (p < 0 || q < 1) return ORC_INVALID;
  int rc = orc_validate(g);
  if (rc) return rc;
  i128 wabs2 = 0, ktot = 0, kksum = 0, sabs = 0;
  int neg = 0;
  for (int64_t e = 0; e < g->arcs; e++) {
    int64_t w = W(g, e);
    if (w < 0) { neg = 1; wabs2 -= w; } else wabs2 += w;
    if (wabs2 > 2 * I64LIM + 2) return ORC_OVERFLOW;
  }
  for (int64_t v = 0; v < g->n; v++) {
    int64_t sv = S_of(g, v);
    if (sv < 0) { neg = 1; sabs -= sv; } else sabs += sv;
    ktot += g->k[v];
    kksum += KK_of(g, v);
    if (sabs > I64LIM || ktot > I64LIM || kksum > I64LIM) return ORC_OVERFLOW;
  }
  i128 wabs = wabs2 / 2 + sabs;
  if (wabs > I64LIM) return ORC_OVERFLOW;
  i128 kq = (ktot * ktot) / 4;
  if ((i128)q * wabs > I64LIM) return ORC_OVERFLOW;
  if ((i128)p * ktot > I64LIM) return ORC_OVERFLOW;
  if ((i128)p * kq > I64LIM) return ORC_OVERFLOW;
  if (neg && (i128)q * wabs + (i128)p * kq > I64LIM) return ORC_OVERFLOW;
  return ORC_OK;
}

static int cmp_triple(const void *a, const void *b) {
  const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
  for (int i = 0; i < 3; i++) {
    if (x[i] < y[i]) return -1;
    if (x[i] > y[i]) return 1;
  }
  return 0;
}

/* 1 if the arc multiset equals its reverse (same weights both ways). */
int orc_check_symmetric(const orc_graph *g) {
  int64_t m = g->arcs;
  if (m == 0) return 1;
  int64_t *a = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)m);
  int64_t *b = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)m);
  if (!a || !b) { free(a); free(b); return -1; }
  for (int64_t v = 0; v < g->n; v++)
    for (int64_t e = g->off[v]; e < g->off[v + 1]; e++) {
      a[3 * e] = v; a[3 * e + 1] = g->col[e]; a[3 * e + 2] = W(g, e);
      b[3 * e] = g->col[e]; b[3 * e + 1] = v; b[3 * e + 2] = W(g, e);
    }
  qsort(a, (size_t)m, 3 * sizeof(int64_t), cmp_triple);
  qsort(b, (size_t)m, 3 * sizeof(int64_t), cmp_triple);
  int ok = memcmp(a, b, sizeof(int64_t) * 3 * (size_t)m) == 0;
  free(a); free(b);
  return ok;
}

/* ------------------------------------------------------ cluster bookkeeping */

/* K_X = sum of k_v over v in X, cnt_X = |X|, for cluster ids in [0, n); the
 * fresh ids [n, 2n) start empty. */
static int cluster_totals(const orc_graph *g, const int32_t *C, int64_t *K, int32_t *cnt) {
  for (int64_t x = 0; x < 2 * g->n; x++) { K[x] = 0; cnt[x] = 0; }
  for (int64_t v = 0; v < g->n; v++) {
    int32_t c = C[v];
    if (c < 0 || (int64_t)c >= g->n) return ORC_INVALID;
    K[c] += g->k[v];
    cnt[c] += 1;
  }
  return ORC_OK;
}

/* Scratch for one vertex decision: a dense accumulator indexed by cluster id
 * plus the list of ids it touched, so a reset costs only the touched ids. */
typedef struct {
  int64_t *acc;
  uint8_t *seen;
  int32_t *list;
} decide_scratch;

static int scratch_init(decide_scratch *d, int64_t n) {
  size_t m = (size_t)(n > 0 ? 2 * n : 1); /* ids in [0, 2n) */
  d->acc = (int64_t *)calloc(m, sizeof(int64_t));
  d->seen = (uint8_t *)calloc(m, 1);
  d->list = (int32_t *)malloc(m * sizeof(int32_t));
  return (d->acc && d->seen && d->list) ? ORC_OK : ORC_NOMEM;
}
static void scratch_free(decide_scratch *d) { free(d->acc); free(d->seen); free(d->list); }

/* One scratch per thread of the decision loop (one without OpenMP). */
#ifdef _OPENMP
static int orc_threads(void) { return omp_get_max_threads(); }
static int orc_thread(void) { return omp_get_thread_num(); }
#else
static int orc_threads(void) { return 1; }
static int orc_thread(void) { return 0; }
#endif

static decide_scratch *scratch_init_all(int64_t n, int *count) {
  int t = orc_threads();
  decide_scratch *d = (decide_scratch *)calloc((size_t)t, sizeof(decide_scratch));
  if (!d) return NULL;
  for (int i = 0; i < t; i++) {
    if (scratch_init(&d[i], n)) {
      for (int j = 0; j <= i; j++) scratch_free(&d[j]);
      free(d);
      return NULL;
    }
  }
  *count = t;
  return d;
}

static void scratch_free_all(decide_scratch *d, int count) {
  if (!d) return;
  for (int i = 0; i < count; i++) scratch_free(&d[i]);
  free(d);
}

/* Number of oracle threads the decision loop uses (1 in the plain build). */
int orc_num_threads(void) { return orc_threads(); }

/* The best move of v against a fixed snapshot (C, K, cnt), Algorithm 1's
 * per-vertex step with the Appendix A change in objective.  The change for
 * moving v from c to X != c, scaled by q, is
 *     [q*w(v,X) - p*k_v*K_X] - [q*w(v,c) - p*k_v*(K_c - k_v)],
 * and moving v to a fresh empty cluster has first bracket 0.  The bracketed
 * terms are the "scores"; comparing scores compares the changes exactly.
 * Returns the target id, ORC_ISO, or c to stay. */
static int32_t decide(const orc_graph *g, int64_t p, int64_t q, int allow_iso, const int32_t *C,
                      const int64_t *K, const int32_t *cnt, int64_t v, decide_scratch *d) {
  int32_t c = C[v];
  int64_t kv = g->k[v];
  int64_t nl = 0;
  for (int64_t e = g->off[v]; e < g->off[v + 1]; e++) {
    int32_t X = C[g->col[e]];
    if (!d->seen[X]) { d->seen[X] = 1; d->acc[X] = 0; d->list[nl++] = X; }
    d->acc[X] += W(g, e);
  }
  int64_t w_c = d->seen[c] ? d->acc[c] : 0;
  int64_t stay = q * w_c - (p * kv) * (K[c] - kv);
  int have = 0;
  int64_t best = 0;
  int32_t best_id = 0;
  for (int64_t i = 0; i < nl; i++) {
    int32_t X = d->list[i];
    if (X == c) continue;
    int64_t sc = q * d->acc[X] - (p * kv) * K[X];
    if (!have || sc > best || (sc == best && X < best_id)) { have = 1; best = sc; best_id = X; }
  }
  if (allow_iso && cnt[c] >= 2) {
    /* isolate scores 0 and loses every tie against a real cluster id */
    if (!have || 0 > best) { have = 1; best = 0; best_id = ORC_ISO; }
  }
  for (int64_t i = 0; i < nl; i++) d->seen[d->list[i]] = 0;
  if (have && best > stay) return best_id;
  return c;
}

/* Applies the decisions D of the vertices in U together (Sec. 3.2.1,
 * synchronous setting); a vertex that isolates moves to the fresh cluster
 * n + v.  Returns the number of vertices whose decision differed from their
 * cluster. */
static int64_t apply_moves(const orc_graph *g, int32_t *C, int64_t *K, int32_t *cnt,
                           const int32_t *U, int64_t nu, const int32_t *D) {
  int64_t moved = 0;
  for (int64_t i = 0; i < nu; i++) {
    int32_t v = U[i];
    int32_t c = C[v], d = D[i];
    if (d == c) continue;
    moved++;
    K[c] -= g->k[v];
    cnt[c] -= 1;
    if (d == ORC_ISO) d = (int32_t)(g->n + v);
    K[d] += g->k[v];
    cnt[d] += 1;
    C[v] = d;
  }
  return moved;
}

/* End of an iteration: the non-empty fresh clusters (ids in [n, 2n)), in
 * ascending id order, take the ascending ids in [0, n) that are empty.  There
 * are enough: with T non-empty fresh clusters at most n - T regular ids are
 * in use. */
static void rename_fresh(const orc_graph *g, int32_t *C, int64_t *K, int32_t *cnt, int32_t *newid) {
  int64_t n = g->n, x = 0, any = 0;
  for (int64_t t = 0; t < n; t++) {
    newid[t] = -1;
    if (cnt[n + t] == 0) continue;
    while (cnt[x] != 0) x++;
    newid[t] = (int32_t)x;
    K[x] = K[n + t];
    cnt[x] = cnt[n + t];
    K[n + t] = 0;
    cnt[n + t] = 0;
    x++;
    any = 1;
  }
  if (!any) return;
  for (int64_t v = 0; v < n; v++)
    if (C[v] >= n) C[v] = newid[C[v] - n];
}

/* One synchronous sub-round over an explicit vertex list U (a test hook for
 * the sub-round semantics; Best-Moves itself builds U from the hash colors).
 * C is updated in place; D_out (length nu, may be NULL) receives the decisions
 * (ORC_ISO for isolate).  Returns the number of movers, or -1 on error. */
int64_t orc_subround(const orc_graph *g, int64_t p, int64_t q, int32_t allow_iso, int32_t *C,
                     const int32_t *U, int64_t nu, int32_t *D_out) {
  int64_t n = g->n;
  size_t n2 = (size_t)(n ? 2 * n : 1);
  int64_t *K = (int64_t *)malloc(sizeof(int64_t) * n2);
  int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * n2);
  int32_t *D = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nu ? nu : 1));
  int32_t *newid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
  decide_scratch sc;
  int64_t moved = -1;
  if (!K || !cnt || !D || !newid || scratch_init(&sc, n)) goto out;
  if (cluster_totals(g, C, K, cnt)) { scratch_free(&sc); goto out; }
  for (int64_t i = 0; i < nu; i++) D[i] = decide(g, p, q, allow_iso, C, K, cnt, U[i], &sc);
  if (D_out) memcpy(D_out, D, sizeof(int32_t) * (size_t)nu);
  moved = apply_moves(g, C, K, cnt, U, nu, D);
  rename_fresh(g, C, K, cnt, newid);
  scratch_free(&sc);
out:
  free(K); free(cnt); free(D); free(newid);
  return moved;
}

/* Decisions of the listed vertices against the clustering C, without moving
 * anything (used to check sampled vertices of very large graphs). */
int orc_decide_many(const orc_graph *g, int64_t p, int64_t q, int32_t allow_iso, const int32_t *C,
                    const int32_t *U, int64_t nu, int32_t *D_out) {
  int64_t n = g->n;
  int64_t *K = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n ? 2 * n : 1));
  int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? 2 * n : 1));
  int nsc = 0;
  decide_scratch *sc = NULL;
  int rc = ORC_NOMEM;
  if (!K || !cnt || !(sc = scratch_init_all(n, &nsc))) goto out;
  rc = cluster_totals(g, C, K, cnt);
  if (!rc) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nu; i++) D_out[i] = decide(g, p, q, allow_iso, C, K, cnt, U[i], &sc[orc_thread()]);
  }
out:
  scratch_free_all(sc, nsc);
  free(K); free(cnt);
  return rc;
}

/* Frontier "neighbors of moved vertices" (Algorithm 1, Sec. 3.2.2):
 * flags[u] = 1 for every neighbor u of a listed mover. */
void orc_frontier_nbr(const orc_graph *g, const int32_t *movers, int64_t nm, uint8_t *flags) {
  for (int64_t i = 0; i < nm; i++) {
    int32_t v = movers[i];
    for (int64_t e = g->off[v]; e < g->off[v + 1]; e++) flags[g->col[e]] = 1;
  }
}

/* -------------------------------------------------------------- Best-Moves */

/* Best-Moves (Algorithm 1, top) from the clustering in C, at hierarchy level
 * `level` and phase 0 (coarsening) or 1 (refinement).  At most num_iter
 * iterations; each iteration runs S sub-rounds over the active vertices;
 * stops after an iteration with no move. */
static int best_move_impl(const orc_graph *g, int64_t p, int64_t q, const orc_params *prm,
                          int32_t level, int32_t phase, int32_t *C, orc_bm_stats *st) {
  int64_t n = g->n;
  orc_bm_stats local;
  if (!st) st = &local;
  memset(st, 0, sizeof(*st));
  if (prm->S < 1 || prm->num_iter < 0) return ORC_INVALID;
  if (prm->frontier < ORC_FRONTIER_ALL || prm->frontier > ORC_FRONTIER_CLUSTERS) return ORC_INVALID;
  size_t nn = (size_t)(n ? n : 1);
  int64_t *K = (int64_t *)malloc(sizeof(int64_t) * 2 * nn);
  int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * 2 * nn);
  uint8_t *active = (uint8_t *)malloc(nn);
  uint8_t *next = (uint8_t *)calloc(nn, 1);
  int32_t *newid = (int32_t *)malloc(sizeof(int32_t) * nn);
  int32_t *U = (int32_t *)malloc(sizeof(int32_t) * nn);
  int32_t *D = (int32_t *)malloc(sizeof(int32_t) * nn);
  /* clusters (ids in [0, 2n)) that a vertex moved out of in this iteration */
  uint8_t *left = (uint8_t *)calloc(2 * nn, 1);
  int nsc = 0;
  decide_scratch *sc = NULL;
  int rc = ORC_NOMEM;
  if (!K || !cnt || !active || !next || !newid || !U || !D || !left || !(sc = scratch_init_all(n, &nsc))) goto out;
  rc = cluster_totals(g, C, K, cnt);
  if (rc) goto out;
  memset(active, 1, nn);
  st->term = ORC_TERM_NUM_ITER;
  for (int32_t it = 0; it < prm->num_iter; it++) {
    uint64_t h = orc_round_hash(prm->seed, level, phase, it);
    int64_t moved_it = 0, active_it = 0;
    for (int64_t v = 0; v < n; v++) active_it += active[v];
    st->iterations++;
    for (int32_t s = 0; s < prm->S; s++) {
      if (prm->stop_after_subrounds > 0 && st->subrounds >= prm->stop_after_subrounds) {
        st->term = ORC_TERM_STOPPED;
        if (it < ORC_MAX_ITER_STATS) { st->active_per_iter[it] = active_it; st->moves_per_iter[it] = moved_it; }
        goto done;
      }
      int64_t nu = 0;
      for (int64_t v = 0; v < n; v++)
        if (active[v] && orc_color(h, v, prm->S) == s) U[nu++] = (int32_t)v;
      /* every decision of the sub-round reads the same snapshot */
      int64_t arcs = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : arcs)
      for (int64_t i = 0; i < nu; i++) {
        D[i] = decide(g, p, q, prm->allow_isolate, C, K, cnt, U[i], &sc[orc_thread()]);
        arcs += g->off[U[i] + 1] - g->off[U[i]];
      }
      st->arcs_scanned += arcs;
      st->vertices_processed += nu;
      for (int64_t i = 0; i < nu; i++) {
        if (D[i] == C[U[i]]) continue;
        if (prm->frontier == ORC_FRONTIER_NBR) orc_frontier_nbr(g, &U[i], 1, next);
        left[C[U[i]]] = 1;
      }
      int64_t mv = apply_moves(g, C, K, cnt, U, nu, D);
      moved_it += mv;
      st->subrounds++;
    }
    if (prm->frontier == ORC_FRONTIER_CLUSTERS) {
      /* neighbors of every vertex now in a cluster that someone left (ids
       * are those of this iteration, before the fresh ones are renamed) */
      for (int64_t u = 0; u < n; u++)
        if (left[C[u]])
          for (int64_t e = g->off[u]; e < g->off[u + 1]; e++) next[g->col[e]] = 1;
    }
    memset(left, 0, 2 * nn);
    rename_fresh(g, C, K, cnt, newid);
    if (it < ORC_MAX_ITER_STATS) { st->active_per_iter[it] = active_it; st->moves_per_iter[it] = moved_it; }
    st->moves += moved_it;
    /* progress for long runs (ORC_PROGRESS set): one line per iteration */
    if (getenv("ORC_PROGRESS"))
      fprintf(stderr, "[oracle] level %d phase %d iteration %d: %lld active, %lld moved\n", (int)level, (int)phase,
              (int)it, (long long)active_it, (long long)moved_it);
    if (moved_it == 0) { st->term = ORC_TERM_NO_MOVES; break; }
    st->moved_any = 1;
    if (prm->frontier == ORC_FRONTIER_ALL) {
      memset(active, 1, nn);
    } else {
      memcpy(active, next, nn);
    }
    memset(next, 0, nn);
  }
done:
  /* moves of a partial (stopped) iteration also count */
  if (st->term == ORC_TERM_STOPPED) {
    rename_fresh(g, C, K, cnt, newid);
    int32_t it = st->iterations - 1;
    int64_t mv = (it >= 0 && it < ORC_MAX_ITER_STATS) ? st->moves_per_iter[it] : 0;
    st->moves += mv;
    if (mv) st->moved_any = 1;
  }
  rc = ORC_OK;
out:
  scratch_free_all(sc, nsc);
  free(K); free(cnt); free(active); free(next); free(newid); free(U); free(D); free(left);
  return rc;
}

int orc_best_move(const orc_graph *g, int64_t p, int64_t q, const orc_params *prm, int32_t level,
                  int32_t phase, int32_t *C, orc_bm_stats *st) {
  int rc = orc_precheck(g, p, q);
  if (rc) return rc;
  return best_move_impl(g, p, q, prm, level, phase, C, st);
}

/* ---------------------------------------------------------------- compress */

void orc_graph_free(orc_graph_out *o) {
  if (!o) return;
  free(o->off); free(o->col); free(o->wt); free(o->k); free(o->s); free(o->kk);
  memset(o, 0, sizeof(*o));
}

/* Compress (Sec. 3.1, Appendix B): one vertex per non-empty cluster, numbered
 * by the rank of the cluster id among non-empty ids (map[v] = rank of C[v]);
 * k'(c) = K_c; kk'(c) = sum of kk over members; s'(c) = sum of members' s plus
 * the weight of the edges inside c; the edges between two clusters are
 * combined into one edge carrying the summed weight (kept even when the sum
 * is 0).  Rows of the output are sorted by neighbor id.
 *
 * The row of coarse vertex c is formed from c's members (the vertices with
 * map[v] = c): every arc to another cluster adds its weight to a dense
 * accumulator indexed by the neighbor's number; the numbers it touched,
 * sorted, with their sums, are the row.  A first pass over the rows only
 * counts their lengths (so the output is allocated once), a second fills
 * them.  Built with OpenMP, rows are formed in parallel, each thread with
 * its own accumulator; a row is computed the same way by any thread. */
typedef struct {
  int64_t *acc;   /* weight sum per neighbor number, valid where stamp == row */
  int64_t *stamp; /* row that last touched the number */
  int32_t *list;  /* numbers touched by the current row */
} row_scratch;

static int row_scratch_init(row_scratch *r, int64_t n2) {
  size_t m = (size_t)(n2 ? n2 : 1);
  r->acc = (int64_t *)malloc(m * sizeof(int64_t));
  r->stamp = (int64_t *)malloc(m * sizeof(int64_t));
  r->list = (int32_t *)malloc(m * sizeof(int32_t));
  if (!r->acc || !r->stamp || !r->list) return ORC_NOMEM;
  for (size_t x = 0; x < m; x++) r->stamp[x] = -1;
  return ORC_OK;
}
static void row_scratch_free(row_scratch *r) { free(r->acc); free(r->stamp); free(r->list); }

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Sums the arcs of c's members into r by neighbor number (arcs inside c
 * skipped); returns the number of distinct neighbor numbers, listed in r. */
static int64_t coarse_row(const orc_graph *g, const int32_t *map, const int64_t *mstart, const int32_t *members,
                          int64_t c, row_scratch *r) {
  int64_t cnt = 0;
  for (int64_t i = mstart[c]; i < mstart[c + 1]; i++) {
    int32_t v = members[i];
    for (int64_t e = g->off[v]; e < g->off[v + 1]; e++) {
      int32_t x = map[g->col[e]];
      if ((int64_t)x == c) continue;
      if (r->stamp[x] != c) {
        r->stamp[x] = c;
        r->acc[x] = 0;
        r->list[cnt++] = x;
      }
      r->acc[x] += W(g, e);
    }
  }
  return cnt;
}

int orc_compress(const orc_graph *g, const int32_t *C, orc_graph_out *out, int32_t *map) {
  int64_t n = g->n;
  memset(out, 0, sizeof(*out));
  if (orc_validate(g)) return ORC_INVALID;
  size_t nn = (size_t)(n ? n : 1);
  int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * nn);
  uint8_t *present = (uint8_t *)calloc(nn, 1);
  int64_t *mstart = NULL, *len = NULL;
  int32_t *members = NULL;
  i128 *intra = NULL;
  int rc = ORC_NOMEM, failed = 0;
  if (!rank || !present) goto fail;
  for (int64_t v = 0; v < n; v++) {
    if (C[v] < 0 || (int64_t)C[v] >= n) { rc = ORC_INVALID; goto fail; }
    present[C[v]] = 1;
  }
  int64_t n2 = 0;
  for (int64_t x = 0; x < n; x++) rank[x] = present[x] ? (int32_t)n2++ : -1;
  for (int64_t v = 0; v < n; v++) map[v] = rank[C[v]];
  out->n = n2;
  size_t n2s = (size_t)(n2 ? n2 : 1);
  out->k = (int64_t *)calloc(n2s, sizeof(int64_t));
  out->s = (int64_t *)calloc(n2s, sizeof(int64_t));
  out->kk = (int64_t *)calloc(n2s, sizeof(int64_t));
  out->off = (int64_t *)calloc(n2s + 1, sizeof(int64_t));
  intra = (i128 *)calloc(n2s, sizeof(i128));
  mstart = (int64_t *)calloc(n2s + 1, sizeof(int64_t));
  len = (int64_t *)calloc(n2s, sizeof(int64_t));
  members = (int32_t *)malloc(sizeof(int32_t) * nn);
  if (!out->k || !out->s || !out->kk || !out->off || !intra || !mstart || !len || !members) goto fail;
  for (int64_t v = 0; v < n; v++) {
    int32_t cv = map[v];
    out->k[cv] += g->k[v];
    out->kk[cv] += (int64_t)KK_of(g, v);
    intra[cv] += 2 * (i128)S_of(g, v);
    for (int64_t e = g->off[v]; e < g->off[v + 1]; e++)
      if (map[g->col[e]] == cv) intra[cv] += W(g, e);
  }
  /* each intra edge was seen from both endpoints, each self weight doubled */
  for (int64_t c = 0; c < n2; c++) out->s[c] = (int64_t)(intra[c] / 2);
  /* the members of every coarse vertex, in vertex order */
  for (int64_t v = 0; v < n; v++) mstart[map[v] + 1]++;
  for (int64_t c = 0; c < n2; c++) mstart[c + 1] += mstart[c];
  for (int64_t c = 0; c < n2; c++) len[c] = mstart[c];
  for (int64_t v = 0; v < n; v++) members[len[map[v]]++] = (int32_t)v;
  /* row lengths */
#pragma omp parallel
  {
    row_scratch r;
    int ok = row_scratch_init(&r, n2) == ORC_OK;
    if (!ok) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(dynamic, 64)
    for (int64_t c = 0; c < n2; c++)
      if (ok) len[c] = coarse_row(g, map, mstart, members, c, &r);
    row_scratch_free(&r);
  }
  if (failed) goto fail;
  for (int64_t c = 0; c < n2; c++) out->off[c + 1] = out->off[c] + len[c];
  int64_t m2 = out->off[n2];
  out->arcs = m2;
  out->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m2 ? m2 : 1));
  out->wt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m2 ? m2 : 1));
  if (!out->col || !out->wt) goto fail;
  /* rows: sorted neighbor numbers with their summed weights */
#pragma omp parallel
  {
    row_scratch r;
    int ok = row_scratch_init(&r, n2) == ORC_OK;
    if (!ok) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(dynamic, 64)
    for (int64_t c = 0; c < n2; c++) {
      if (!ok) continue;
      int64_t cnt = coarse_row(g, map, mstart, members, c, &r);
      qsort(r.list, (size_t)cnt, sizeof(int32_t), cmp_i32);
      for (int64_t i = 0; i < cnt; i++) {
        out->col[out->off[c] + i] = r.list[i];
        out->wt[out->off[c] + i] = r.acc[r.list[i]];
      }
    }
    row_scratch_free(&r);
  }
  if (failed) goto fail;
  free(rank); free(present); free(intra); free(mstart); free(len); free(members);
  return ORC_OK;
fail:
  free(rank); free(present); free(intra); free(mstart); free(len); free(members);
  orc_graph_free(out);
  return rc;
}

/* --------------------------------------------------------------- objective */

/* The objective of Sec. 2 over unordered pairs: the sum over pairs {i, j} in
 * the same cluster of w'_ij, where w'_ij = w_ij - lambda*k_i*k_j on edges and
 * -lambda*k_i*k_j on non-edges.  With lambda = p/q the value is N/q with
 *   N = q*(sum_v s_v + W_in) - p * sum_X (K_X^2 - sum_{v in X} kk_v) / 2,
 * W_in the weight of edges inside clusters (each edge once).  (The V x V sum
 * of Sec. 2 counts every pair twice and equals 2N/q.)  Returns N split in two
 * 64-bit halves. */
int orc_objective(const orc_graph *g, int64_t p, int64_t q, const int32_t *C, int64_t *num_hi,
                  uint64_t *num_lo) {
  int rc = orc_precheck(g, p, q);
  if (rc) return rc;
  int64_t n = g->n;
  size_t nn = (size_t)(n ? n : 1);
  i128 *K = (i128 *)calloc(nn, sizeof(i128));
  i128 *KK = (i128 *)calloc(nn, sizeof(i128));
  if (!K || !KK) { free(K); free(KK); return ORC_NOMEM; }
  i128 win2 = 0, ssum = 0;
  for (int64_t v = 0; v < n; v++) {
    if (C[v] < 0 || (int64_t)C[v] >= n) { free(K); free(KK); return ORC_INVALID; }
    K[C[v]] += g->k[v];
    KK[C[v]] += KK_of(g, v);
    ssum += S_of(g, v);
    for (int64_t e = g->off[v]; e < g->off[v + 1]; e++)
      if (C[g->col[e]] == C[v]) win2 += W(g, e);
  }
  i128 pairs2 = 0;
  for (int64_t x = 0; x < n; x++) pairs2 += K[x] * K[x] - KK[x];
  i128 N = (i128)q * (ssum + win2 / 2) - (i128)p * (pairs2 / 2);
  *num_hi = (int64_t)(N >> 64);
  *num_lo = (uint64_t)N;
  free(K); free(KK);
  return ORC_OK;
}

/* -------------------------------------------------------- labels / cluster */

/* Canonical labels: clusters numbered 0, 1, ... in the order of their
 * smallest member. */
int orc_canonical_labels(int64_t n, const int32_t *C, int32_t *labels) {
  size_t nn = (size_t)(n ? n : 1);
  int32_t *minv = (int32_t *)malloc(sizeof(int32_t) * nn);
  int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * nn);
  if (!minv || !lab) { free(minv); free(lab); return ORC_NOMEM; }
  for (int64_t x = 0; x < n; x++) minv[x] = INT32_MAX;
  for (int64_t v = 0; v < n; v++) {
    if (C[v] < 0 || (int64_t)C[v] >= n) { free(minv); free(lab); return ORC_INVALID; }
    if ((int32_t)v < minv[C[v]]) minv[C[v]] = (int32_t)v;
  }
  int32_t next = 0;
  for (int64_t v = 0; v < n; v++)
    if (minv[C[v]] == (int32_t)v) lab[C[v]] = next++;
  for (int64_t v = 0; v < n; v++) labels[v] = lab[C[v]];
  free(minv); free(lab);
  return ORC_OK;
}

/* Parallel-CC (Algorithm 1, bottom) with multi-level refinement (Sec. 3.2.3):
 * Best-Moves from singletons; while it moved something (and the level cap is
 * not reached) compress and recurse; on the way back flatten each level's
 * clustering through its map and, with refinement, run Best-Moves again on
 * that level.  Writes canonical labels and the objective numerator. */
/* Number of distinct cluster ids in C (ids in [0, n)). */
static int64_t count_clusters(const int32_t *C, int64_t n) {
  uint8_t *seen = (uint8_t *)calloc((size_t)(n ? n : 1), 1);
  if (!seen) return -1;
  int64_t k = 0;
  for (int64_t v = 0; v < n; v++)
    if (!seen[C[v]]) { seen[C[v]] = 1; k++; }
  free(seen);
  return k;
}

int orc_cluster(const orc_graph *g0, int64_t p, int64_t q, const orc_params *prm, int32_t *labels,
                int64_t *num_hi, uint64_t *num_lo, orc_cluster_stats *cs) {
  int rc = orc_precheck(g0, p, q);
  if (rc) return rc;
  if (prm->max_levels < 1 || prm->max_levels > ORC_MAX_LEVELS || prm->S < 1) return ORC_INVALID;
  orc_cluster_stats local;
  if (!cs) cs = &local;
  memset(cs, 0, sizeof(*cs));
  orc_graph G[ORC_MAX_LEVELS];
  orc_graph_out owned[ORC_MAX_LEVELS];
  int32_t *Cl[ORC_MAX_LEVELS];
  int32_t *map[ORC_MAX_LEVELS];
  memset(owned, 0, sizeof(owned));
  memset(Cl, 0, sizeof(Cl));
  memset(map, 0, sizeof(map));
  G[0] = *g0;
  int32_t top = 0;
  rc = ORC_OK;
  for (int32_t l = 0;; l++) {
    int64_t n = G[l].n;
    cs->n_level[l] = n;
    cs->arcs_level[l] = G[l].arcs;
    cs->levels = l + 1;
    Cl[l] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    if (!Cl[l]) { rc = ORC_NOMEM; goto out; }
    for (int64_t v = 0; v < n; v++) Cl[l][v] = (int32_t)v;
    orc_bm_stats st;
    rc = best_move_impl(&G[l], p, q, prm, l, 0, Cl[l], &st);
    if (rc) goto out;
    cs->iters_coarsen[l] = st.iterations;
    cs->moves_total += st.moves;
    cs->arcs_scanned_total += st.arcs_scanned;
    /* Algorithm 1 recurses only when Best-Moves made a move.  This call
     * started from singletons; if every vertex ends alone in its cluster, the
     * moves only exchanged the ids of singletons (the synchronous sub-rounds
     * allow such swaps, the paper's immediate moves do not) and the partition
     * is the one the call started from: no move changed it, and its
     * contraction would be the same graph renumbered.  The recursion ends
     * there as it does after a call without moves. */
    int64_t ncl = st.moved_any ? count_clusters(Cl[l], n) : n;
    if (ncl < 0) { rc = ORC_NOMEM; goto out; }
    int changed = st.moved_any && ncl < n;
    if (!changed || l + 1 == prm->max_levels) {
      top = l;
      cs->top_moved = changed;
      break;
    }
    map[l] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    if (!map[l]) { rc = ORC_NOMEM; goto out; }
    if (getenv("ORC_PROGRESS")) fprintf(stderr, "[oracle] level %d: contracting\n", (int)l);
    rc = orc_compress(&G[l], Cl[l], &owned[l + 1], map[l]);
    if (rc) goto out;
    orc_graph_out *o = &owned[l + 1];
    G[l + 1].n = o->n; G[l + 1].arcs = o->arcs; G[l + 1].off = o->off; G[l + 1].col = o->col;
    G[l + 1].wt = o->wt; G[l + 1].k = o->k; G[l + 1].s = o->s; G[l + 1].kk = o->kk;
  }
  for (int32_t l = top - 1; l >= 0; l--) {
    for (int64_t v = 0; v < G[l].n; v++) Cl[l][v] = Cl[l + 1][map[l][v]];
    if (prm->refine) {
      orc_bm_stats st;
      rc = best_move_impl(&G[l], p, q, prm, l, 1, Cl[l], &st);
      if (rc) goto out;
      cs->iters_refine[l] = st.iterations;
      cs->moves_total += st.moves;
      cs->arcs_scanned_total += st.arcs_scanned;
    }
  }
  rc = orc_canonical_labels(g0->n, Cl[0], labels);
  if (rc) goto out;
  {
    int32_t mx = -1;
    for (int64_t v = 0; v < g0->n; v++) if (labels[v] > mx) mx = labels[v];
    cs->clusters = (int64_t)mx + 1;
  }
  rc = orc_objective(g0, p, q, labels, num_hi, num_lo);
out:
  for (int32_t l = 0; l < ORC_MAX_LEVELS; l++) {
    free(Cl[l]);
    free(map[l]);
    orc_graph_free(&owned[l]);
  }
  return rc;
}
