"""Plants plausible mistakes in a copy of the oracle source (CPU only) and
checks that the pins in test_oracle_pins.py catch every one of them.  This
shows the pins constrain each part of the oracle: the gain terms, the tie
rules, the isolate rule, the objective, compress, the frontier, synchronous
application, flattening, refinement and the final labels.

Each variant is loaded into this process, so a mutation must keep the oracle
memory-safe (one that, say, stops clusters from ever emptying would send the
fresh-id renaming past its arrays)."""
import os

import pytest

import oracle as O
from tests import test_oracle_pins as P

MUTATIONS = {
    "stay_drops_self_term": ("(p * kv) * (K[c] - kv)", "(p * kv) * K[c]"),
    "tie_to_highest_id": ("(sc == best && X < best_id)", "(sc == best && X > best_id)"),
    "move_on_equal_gain": ("if (have && best > stay) return best_id;",
                           "if (have && best >= stay) return best_id;"),
    "isolate_from_singleton": ("if (allow_iso && cnt[c] >= 2)", "if (allow_iso && cnt[c] >= 1)"),
    "target_counts_self": ("int64_t sc = q * d->acc[X] - (p * kv) * K[X];",
                           "int64_t sc = q * d->acc[X] - (p * kv) * (K[X] + kv);"),
    "objective_sign": ("- (i128)p * (pairs2 / 2);", "+ (i128)p * (pairs2 / 2);"),
    "objective_ordered_pairs": ("(ssum + win2 / 2)", "(ssum + win2)"),
    "compress_intra_not_halved": ("out->s[c] = (int64_t)(intra[c] / 2);",
                                  "out->s[c] = (int64_t)(intra[c]);"),
    "compress_kk_overwritten": ("out->kk[cv] += (int64_t)KK_of(g, v);",
                                "out->kk[cv] = (int64_t)KK_of(g, v);"),
    "compress_rows_unsorted": ("qsort(r.list, (size_t)cnt, sizeof(int32_t), cmp_i32);",
                               "qsort(r.list, (size_t)cnt / 2, sizeof(int32_t), cmp_i32);"),
    "frontier_adds_mover": ("for (int64_t e = g->off[v]; e < g->off[v + 1]; e++) flags[g->col[e]] = 1;",
                            "flags[v] = 1; for (int64_t e = g->off[v]; e < g->off[v + 1]; e++) flags[g->col[e]] = 1;"),
    "fresh_ids_skip_first_empty": ("    while (cnt[x] != 0) x++;\n    newid[t] = (int32_t)x;",
                                   "    x += (x == 0);\n    while (cnt[x] != 0) x++;\n    newid[t] = (int32_t)x;"),
    "fresh_cluster_not_renamed": ("    if (C[v] >= n) C[v] = newid[C[v] - n];", "    if (0) C[v] = newid[C[v] - n];"),
    "isolate_score_positive": ("if (!have || 0 > best) { have = 1; best = 0; best_id = ORC_ISO; }",
                               "if (!have || 1 > best) { have = 1; best = 0; best_id = ORC_ISO; }"),
    "mix_wrong_constant": ("z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;",
                           "z = (z ^ (z >> 27)) * 0x94D049BB133111EDULL;"),
    "refine_skipped": ("    if (prm->refine) {\n      orc_bm_stats st;",
                       "    if (0 && prm->refine) {\n      orc_bm_stats st;"),
    "frontier_from_stayers": ("        if (D[i] == C[U[i]]) continue;\n        if (prm->frontier == ORC_FRONTIER_NBR)",
                              "        if (D[i] != C[U[i]]) continue;\n        if (prm->frontier == ORC_FRONTIER_NBR)"),
    "clusters_frontier_from_targets": ("        left[C[U[i]]] = 1;",
                                       "        left[D[i] == ORC_ISO ? g->n + U[i] : D[i]] = 1;"),
    "clusters_frontier_marks_members": ("          for (int64_t e = g->off[u]; e < g->off[u + 1]; e++) next[g->col[e]] = 1;",
                                        "          next[u] = 1;"),
    "apply_source_volume_kept": ("    K[c] -= g->k[v];\n    cnt[c] -= 1;", "    K[c] -= 0;\n    cnt[c] -= 1;"),
    "compress_self_weight_dropped": ("    intra[cv] += 2 * (i128)S_of(g, v);", "    intra[cv] += 0 * (i128)S_of(g, v);"),
    "labels_by_largest_member": ("    if ((int32_t)v < minv[C[v]]) minv[C[v]] = (int32_t)v;",
                                 "    if ((int32_t)v > minv[C[v]] || minv[C[v]] == INT32_MAX) minv[C[v]] = (int32_t)v;"),
    "moves_applied_at_once": (
        "        arcs += g->off[U[i] + 1] - g->off[U[i]];\n",
        "        arcs += g->off[U[i] + 1] - g->off[U[i]];\n"
        "        if (D[i] != C[U[i]]) { orc_frontier_nbr(g, &U[i], 1, next);"
        " moved_it += apply_moves(g, C, K, cnt, &U[i], 1, &D[i]); D[i] = C[U[i]]; }\n"),
    "recursion_on_id_swaps": ("    int changed = st.moved_any && ncl < n;", "    int changed = st.moved_any;"),
    "flatten_drops_coarse_clustering": ("    for (int64_t v = 0; v < G[l].n; v++) Cl[l][v] = Cl[l + 1][map[l][v]];",
                                        "    for (int64_t v = 0; v < G[l].n; v++) Cl[l][v] = map[l][v];"),
}

# a mutation that leaves behavior unchanged is excluded (kept to document it)
# ("isolate_from_singleton": a singleton's staying score is exactly 0, the
# isolate score, so the |c| >= 2 guard never changes a decision.)
EQUIVALENT = {"isolate_from_singleton"}


def _pins():
    checks = []
    checks.append(P.test_splitmix64_published_vectors)
    for s in range(4):
        checks.append(lambda s=s: P.test_P1_objective_matches_pair_definition(s))
    for s in range(6):
        checks.append(lambda s=s: P.test_P2_decision_matches_brute_force_every_partition(s))
    for s in range(5):
        checks.append(lambda s=s: P.test_P5_compress_contraction_invariant(s))
    checks += [P.test_P7_figure1_simultaneous_moves_lower_objective, P.test_P8_star_frontier_footnote,
               P.test_P9_symmetric_pair_swaps_or_merges, P.test_second_iteration_uses_neighbors_of_movers,
               P.test_isolation_takes_smallest_empty_ids, P.test_P3_refinement_ends_in_single_move_local_optimum,
               P.test_P5_two_level_compress_invariant, P.test_canonical_labels_order_by_min_member,
               P.test_clusters_frontier_reconsiders_neighbors_of_the_left_cluster,
               P.test_clusters_frontier_second_iteration_matches_definition,
               P.test_recursion_ends_when_only_singleton_ids_were_exchanged]
    for s in range(2):
        checks.append(lambda s=s: P.test_P4_decisions_are_best_modularity_moves(s))
    return checks


@pytest.mark.parametrize("name", sorted(set(MUTATIONS) - EQUIVALENT))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = O.source_text()
    assert src.count(old) == 1, f"mutation anchor not found exactly once: {old}"
    lib = O.build_variant(src.replace(old, new), os.path.join(str(tmp_path), f"mut_{name}.so"))
    prev = O.use_library(lib)
    caught = []
    try:
        for chk in _pins():
            try:
                chk()
            except (AssertionError, O.OracleError) as e:
                caught.append(repr(e)[:80])
                break
    finally:
        O.use_library(prev)
    assert caught, f"no pin caught the planted mistake {name}"
