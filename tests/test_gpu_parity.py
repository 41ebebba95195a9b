"""GPU parity: the HIP path through the C ABI against the CPU oracle, element
by element, on seeded inputs.  Everything is integer, so the bar is
bit-exact equality of clusterings, contracted graphs, objectives and the
schedule counters."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2108_01731_amd import graphgen as G
from paper_2108_01731_amd import lcc as L
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return L.context(0)


def dev(h):
    return L.DeviceGraph.from_host(h, "cuda")


def oparams(**kw):
    return O.Params(**kw)


def dparams(**kw):
    return L.Params(**kw)


def run_pair_best_move(ctx, h, p, q, C0=None, level=0, phase=0, **kw):
    g_o = H.to_oracle(h)
    g_d = dev(h)
    n = g_o.n
    C0 = np.arange(n, dtype=np.int32) if C0 is None else np.asarray(C0, np.int32)
    Co, so = O.best_move(g_o, p, q, oparams(**kw), C0, level, phase)
    Cd = torch.from_numpy(C0.copy()).cuda()
    sd = L.lcc_best_move(ctx, g_d, p, q, dparams(**kw), Cd, level, phase)
    return Co, so, Cd.cpu().numpy(), sd


def assert_same_bm(Co, so, Cd, sd):
    assert np.array_equal(Co, Cd)
    for key in ("iterations", "subrounds", "moved_any", "term", "moves", "arcs_scanned", "vertices_processed",
                "active_per_iter", "moves_per_iter"):
        assert so[key] == sd[key], (key, so[key], sd[key])


def graphs():
    """(name, HostGraph, p, q) cases spanning weight kinds, degree bins and
    lambda regimes."""
    c1 = G.c1_sbm(1)
    cl = G.chung_lu_planted(30000, 400000, 2.1, 0.3, seed=2)
    out = [
        ("sbm_c1", c1, 1, 100),
        ("sbm_c1_i16", H.with_weights(c1, "i16", 1, -3, 40), 1, 10),
        ("sbm_c1_i64", H.with_weights(c1, "i64", 2, -2, 7), 3, 7),
        ("chung_lu_mod", cl, 1, int(cl.arcs)),
        ("hubs_i32", H.hub_graph(), 1, 40),
        ("hubs_unit", H.hub_graph(weighted=False), 1, 500),
        ("random_signed", G.random_signed(3000, 9000, 3, wmin=-4, wmax=6, kmax=3), 1, 9),
        # rows beyond the LDS tables (flat aggregation into global tables)
        ("wide_hubs", H.hub_graph(n=40000, m=60000, hubs=(16000, 25000, 31000, 14500), seed=21), 1, 60),
    ]
    return out


GRAPHS = None


def cases():
    global GRAPHS
    if GRAPHS is None:
        GRAPHS = graphs()
    return GRAPHS


@pytest.mark.parametrize("idx", range(8))
def test_subround_by_subround_parity(ctx, idx):
    """C and the schedule counters after every one of the first sub-rounds."""
    name, h, p, q = cases()[idx]
    S = 3
    for stop in range(1, 2 * S + 2):
        Co, so, Cd, sd = run_pair_best_move(ctx, h, p, q, S=S, seed=7, stop_after_subrounds=stop)
        assert_same_bm(Co, so, Cd, sd)
    # the neighbors-of-clusters frontier, from a clustering with multi-vertex
    # clusters, into the third iteration
    C0 = np.random.default_rng(idx).integers(0, max(1, h.n // 20), size=h.n).astype(np.int32)
    for stop in (S + 1, 2 * S + 1):
        Co, so, Cd, sd = run_pair_best_move(ctx, h, p, q, C0=C0, S=S, seed=3, frontier=2,
                                            stop_after_subrounds=stop)
        assert_same_bm(Co, so, Cd, sd)


@pytest.mark.parametrize("idx", range(8))
@pytest.mark.parametrize("cfg", [dict(S=4), dict(S=1, num_iter=4), dict(S=2, frontier=0), dict(S=8, allow_isolate=0),
                                 dict(S=4, seed=12345, num_iter=25), dict(S=4, frontier=2),
                                 dict(S=3, frontier=2, seed=99, num_iter=25)])
def test_best_move_parity(ctx, idx, cfg):
    name, h, p, q = cases()[idx]
    Co, so, Cd, sd = run_pair_best_move(ctx, h, p, q, **cfg)
    assert_same_bm(Co, so, Cd, sd)


@pytest.mark.parametrize("idx", range(8))
def test_pruned_scoring_parity(ctx, idx):
    """Scoring that skips the cluster totals of candidates whose arc weight
    alone cannot reach the heaviest candidate's score (on every level here,
    not only on the large ones where it is automatic) and scoring without it
    both equal the oracle: from singletons, from a given clustering with a
    large lambda (isolations), and over a whole clustering."""
    name, h, p, q = cases()[idx]
    g_o, g_d = H.to_oracle(h), dev(h)
    C0 = np.random.default_rng(idx + 40).integers(0, max(1, h.n // 30), size=h.n).astype(np.int32)
    for start, (pp, qq), cfg in [(None, (p, q), dict(S=4)), (C0, (p * 50, q), dict(S=3, frontier=2)),
                                 (C0, (p, q), dict(S=2, frontier=0))]:
        Cs = np.arange(h.n, dtype=np.int32) if start is None else start
        Co, so = O.best_move(g_o, pp, qq, oparams(**cfg), Cs, 1, 0)
        for sp in (1, -1):
            Cd = torch.from_numpy(Cs.copy()).cuda()
            sd = L.lcc_best_move(ctx, g_d, pp, qq, dparams(score_pruning=sp, **cfg), Cd, 1, 0)
            assert_same_bm(Co, so, Cd.cpu().numpy(), sd)
    lo, No, _ = O.cluster(g_o, p, q, oparams())
    for sp in (1, -1):
        ld, Nd, _ = L.lcc_cluster(ctx, g_d, p, q, dparams(score_pruning=sp))
        assert np.array_equal(lo, ld.cpu().numpy()) and No == Nd, sp


@pytest.mark.parametrize("idx", range(8))
def test_best_move_from_given_clustering(ctx, idx):
    """Refinement-style start: an arbitrary clustering, level 3, phase 1, and a
    large lambda so isolation happens."""
    name, h, p, q = cases()[idx]
    n = h.n
    rng = np.random.default_rng(idx)
    C0 = rng.integers(0, max(1, n // 50), size=n).astype(np.int32)
    for pp, qq in [(p, q), (p * 50, q)]:
        Co, so, Cd, sd = run_pair_best_move(ctx, h, pp, qq, C0=C0, level=3, phase=1, S=4)
        assert_same_bm(Co, so, Cd, sd)


@pytest.mark.parametrize("idx", range(8))
def test_compress_parity(ctx, idx):
    name, h, p, q = cases()[idx]
    n = h.n
    rng = np.random.default_rng(100 + idx)
    for C0 in [rng.integers(0, max(1, n // 30), size=n), rng.integers(0, n, size=n), np.zeros(n)]:
        C0 = C0.astype(np.int32)
        go, mo = O.compress(H.to_oracle(h), C0)
        gd, md = L.lcc_compress(ctx, dev(h), torch.from_numpy(C0).cuda())
        assert np.array_equal(mo, md.cpu().numpy())
        assert np.array_equal(go.off, gd.off.cpu().numpy())
        assert np.array_equal(go.col, gd.col.cpu().numpy())
        assert np.array_equal(go.wt, gd.wt.cpu().numpy().astype(np.int64))
        assert np.array_equal(go.k, gd.k.cpu().numpy())
        assert np.array_equal(go.s, gd.s.cpu().numpy())
        assert np.array_equal(go.kk, gd.kk.cpu().numpy())
        # second level on the device's own output
        C1 = rng.integers(0, max(1, go.n // 3), size=go.n).astype(np.int32)
        go2, _ = O.compress(go, C1)
        gd2, _ = L.lcc_compress(ctx, gd, torch.from_numpy(C1).cuda())
        assert np.array_equal(go2.col, gd2.col.cpu().numpy())
        assert np.array_equal(go2.wt, gd2.wt.cpu().numpy().astype(np.int64))
        assert np.array_equal(go2.s, gd2.s.cpu().numpy())


def assert_same_graph(go, gd):
    assert gd.n == go.n and gd.arcs == len(go.col)
    assert np.array_equal(go.off, gd.off.cpu().numpy())
    assert np.array_equal(go.col, gd.col.cpu().numpy())
    assert np.array_equal(go.wt, gd.wt.cpu().numpy().astype(np.int64))
    assert np.array_equal(go.k, gd.k.cpu().numpy())
    assert np.array_equal(go.s, gd.s.cpu().numpy())
    assert np.array_equal(go.kk, gd.kk.cpu().numpy())


@pytest.mark.parametrize("kind", ["unit", "i16", "i32", "i64"])
def test_compress_parity_small_graphs(ctx, kind):
    """Graphs of at most 2048 vertices contract through the dense path; every
    output array equals the oracle's, zero-sum coarse edges included (weights
    in [-3, 3] cancel), and so does a second level on the device's output
    (self weights and kk present)."""
    rng = np.random.default_rng(7)
    for n, m, seed in [(2, 1, 2), (37, 60, 3), (300, 2000, 4), (1500, 40000, 5), (2048, 9000, 6)]:
        h = G.random_signed(n, m, seed, wmin=-3, wmax=3, kmax=4, unit=kind == "unit")
        if kind != "unit":
            h = H.with_weights(h, kind, seed=seed, lo=-3, hi=3)
        for C0 in [np.zeros(n), np.arange(n), rng.integers(0, max(1, n // 7), size=n), rng.integers(0, n, size=n)]:
            C0 = C0.astype(np.int32)
            go, mo = O.compress(H.to_oracle(h), C0)
            gd, md = L.lcc_compress(ctx, dev(h), torch.from_numpy(C0).cuda())
            assert np.array_equal(mo, md.cpu().numpy()), (n, kind)
            assert_same_graph(go, gd)
            C1 = rng.integers(0, max(1, go.n // 3), size=go.n).astype(np.int32)
            go2, mo2 = O.compress(go, C1)
            gd2, md2 = L.lcc_compress(ctx, gd, torch.from_numpy(C1).cuda())
            assert np.array_equal(mo2, md2.cpu().numpy())
            assert_same_graph(go2, gd2)


@pytest.mark.parametrize("n,ncl", [(5000, 700), (70000, 0)])
def test_compress_parity_64_bit_coarse_weights(ctx, n, ncl):
    """The sorting path (more than 2048 vertices) when the coarse weights need
    64 bits (sum |w| >= 2^31): with 32-bit sort keys (700 clusters, 2b <= 32)
    and with 64-bit ones (identity clustering of 70000 vertices); every output
    array equals the oracle's, and so does a second level."""
    h = G.random_signed(n, 6 * n, seed=n, wmin=-3, wmax=3, kmax=4)
    h = H.with_weights(h, "i32", seed=1, lo=-(1 << 26), hi=1 << 26)
    rng = np.random.default_rng(n)
    C0 = (rng.integers(0, ncl, size=n) if ncl else np.arange(n)).astype(np.int32)
    go, mo = O.compress(H.to_oracle(h), C0)
    gd, md = L.lcc_compress(ctx, dev(h), torch.from_numpy(C0).cuda())
    assert gd.wt.dtype == torch.int64
    assert np.array_equal(mo, md.cpu().numpy())
    assert_same_graph(go, gd)
    C1 = rng.integers(0, max(1, go.n // 5), size=go.n).astype(np.int32)
    go2, mo2 = O.compress(go, C1)
    gd2, md2 = L.lcc_compress(ctx, gd, torch.from_numpy(C1).cuda())
    assert np.array_equal(mo2, md2.cpu().numpy())
    assert_same_graph(go2, gd2)


@pytest.mark.parametrize("idx", range(8))
def test_objective_parity(ctx, idx):
    name, h, p, q = cases()[idx]
    n = h.n
    rng = np.random.default_rng(200 + idx)
    g_o = H.to_oracle(h)
    g_d = dev(h)
    for C0 in [np.arange(n), rng.integers(0, max(1, n // 40), size=n), np.zeros(n)]:
        C0 = C0.astype(np.int32)
        assert O.objective(g_o, p, q, C0) == L.lcc_objective(ctx, g_d, p, q, torch.from_numpy(C0).cuda())


@pytest.mark.parametrize("idx", range(8))
@pytest.mark.parametrize("cfg", [dict(), dict(S=2, refine=0), dict(S=8, frontier=0, num_iter=20), dict(frontier=2)])
def test_cluster_parity(ctx, idx, cfg):
    name, h, p, q = cases()[idx]
    lo, No, so = O.cluster(H.to_oracle(h), p, q, oparams(**cfg))
    ld, Nd, sd = L.lcc_cluster(ctx, dev(h), p, q, dparams(**cfg))
    assert np.array_equal(lo, ld.cpu().numpy())
    assert No == Nd
    for key in ("levels", "top_moved", "n_level", "arcs_level", "iters_coarsen", "iters_refine", "moves_total",
                "arcs_scanned_total", "clusters"):
        assert so[key] == sd[key], (key, so[key], sd[key])


def test_cluster_parity_synchronous_pathology(ctx):
    """S = 1 (the paper's synchronous setting) oscillates: at the fourth level
    every vertex ends alone (ids exchanged in pairs), so the recursion ends
    there, as the oracle's does; with a cap of two levels the cap ends it."""
    h = G.c1_sbm(1)
    for cfg, levels, top_moved in ((dict(S=1), 4, 0), (dict(S=1, max_levels=2), 2, 1)):
        lo, No, so = O.cluster(H.to_oracle(h), 1, 100, oparams(**cfg))
        ld, Nd, sd = L.lcc_cluster(ctx, dev(h), 1, 100, dparams(**cfg))
        assert np.array_equal(lo, ld.cpu().numpy()) and No == Nd
        assert so["levels"] == sd["levels"] == levels and so["top_moved"] == sd["top_moved"] == top_moved


def test_determinism_and_row_order_invariance(ctx):
    h = H.hub_graph(seed=9)
    runs = [L.lcc_cluster(ctx, dev(h), 1, 40, dparams()) for _ in range(3)]
    runs.append(L.lcc_cluster(ctx, dev(H.shuffle_rows(h, 3)), 1, 40, dparams()))
    for lab, N, _ in runs[1:]:
        assert torch.equal(lab, runs[0][0]) and N == runs[0][1]


def test_repeated_neighbors_equal_merged_arcs(ctx):
    """Parallel arcs (rows repeating a neighbor, so the validation pass must
    report them as not strictly ascending) cluster exactly like the merged
    graph, and like the oracle on the same arcs."""
    h = H.with_weights(G.random_signed(400, 2500, 11), "i64", seed=4, lo=-2, hi=6)
    hs = H.split_arcs(h)
    assert hs.arcs > h.arcs
    for cfg in [dict(), dict(S=2, refine=0)]:
        lo, No, _ = O.cluster(H.to_oracle(hs), 1, 30, oparams(**cfg))
        ls, Ns, _ = L.lcc_cluster(ctx, dev(hs), 1, 30, dparams(**cfg))
        lm, Nm, _ = L.lcc_cluster(ctx, dev(h), 1, 30, dparams(**cfg))
        assert np.array_equal(lo, ls.cpu().numpy()) and No == Ns
        assert torch.equal(ls, lm) and Ns == Nm


def test_hub_rows_with_64_bit_sums(ctx):
    """Hub rows (beyond the LDS tables) whose weight sums need 64 bits take
    the unpacked global tables; rows below 2^31 take the packed ones (the
    other hub cases)."""
    h = H.with_weights(H.hub_graph(n=40000, m=60000, hubs=(16000, 25000), seed=23, weighted=False), "i64", seed=5,
                       lo=1 << 27, hi=1 << 28)
    for cfg in [dict(), dict(S=2, refine=0)]:
        lo, No, _ = O.cluster(H.to_oracle(h), 1, 60, oparams(**cfg))
        ld, Nd, _ = L.lcc_cluster(ctx, dev(h), 1, 60, dparams(**cfg))
        assert np.array_equal(lo, ld.cpu().numpy()) and No == Nd


# (hub_limit, hub_row_limit): the default; every hub row through the hash
# partitions; partitions that overflow (the call is redone with the global
# tables); one-pass rows up to 64 clusters, the others through partitions
HUB_PATHS = [(0, 0), (0, -1), (64, -1), (0, 64)]


def test_hub_partition_overflow_redoes_the_call(ctx):
    """Rows beyond the LDS tables are aggregated one block per row in one
    pass when their clusters fit its table, else in hash partitions; a tiny
    hub_limit makes partitions overflow, so the call is redone from its saved
    clustering with the global tables.  Every way gives the oracle's result."""
    graphs = [H.hub_graph(n=40000, m=60000, hubs=(16000, 25000, 31000, 14500), seed=21),
              H.hub_graph(n=40000, m=60000, hubs=(16000, 25000), seed=22, weighted=False)]
    for h in graphs:
        lo, No, _ = O.cluster(H.to_oracle(h), 1, 60, oparams())
        for limit, row_limit in HUB_PATHS:
            ld, Nd, _ = L.lcc_cluster(ctx, dev(h), 1, 60, dparams(hub_limit=limit, hub_row_limit=row_limit))
            assert np.array_equal(lo, ld.cpu().numpy()) and No == Nd, (limit, row_limit)
    # a single call from a given clustering, device-driven and stopped inside
    # an iteration (host-driven)
    h = graphs[0]
    g_o, g_d = H.to_oracle(h), dev(h)
    C0 = np.random.default_rng(3).integers(0, 200, size=h.n).astype(np.int32)
    for cfg in [dict(S=3), dict(S=3, stop_after_subrounds=5)]:
        Co, so = O.best_move(g_o, 1, 60, oparams(**cfg), C0, 2, 1)
        for limit, row_limit in HUB_PATHS:
            Cd = torch.from_numpy(C0.copy()).cuda()
            sd = L.lcc_best_move(ctx, g_d, 1, 60, dparams(hub_limit=limit, hub_row_limit=row_limit, **cfg), Cd, 2, 1)
            assert_same_bm(Co, so, Cd.cpu().numpy(), sd)


def test_hub_rows_one_pass_and_partitions_in_one_launch(ctx):
    """Starting clusterings whose hub rows meet from a few dozen to over
    20,000 distinct clusters: with one-pass limits between those counts,
    some hub rows of a launch are decided in one pass and the others by the
    partitions (the launch after them skips the former); every mix equals
    the oracle, 32- and 64-bit sums alike."""
    hs = [H.hub_graph(n=60000, m=60000, hubs=(16000, 25000, 31000, 14500, 22000), seed=24),
          H.with_weights(H.hub_graph(n=60000, m=60000, hubs=(16000, 25000), seed=25, weighted=False), "i64",
                         seed=6, lo=1 << 27, hi=1 << 28)]
    rng = np.random.default_rng(8)
    for h in hs:
        g_o, g_d = H.to_oracle(h), dev(h)
        # hub i's neighbors fall in about min(deg, ncl) clusters
        for ncl in [50, 3000, 60000]:
            C0 = rng.integers(0, ncl, size=h.n).astype(np.int32)
            Co, so = O.best_move(g_o, 1, 60, oparams(S=2, num_iter=2), C0, 1, 0)
            for row_limit in [0, -1, 1000, 12000]:
                Cd = torch.from_numpy(C0.copy()).cuda()
                sd = L.lcc_best_move(ctx, g_d, 1, 60, dparams(S=2, num_iter=2, hub_row_limit=row_limit), Cd, 1, 0)
                assert_same_bm(Co, so, Cd.cpu().numpy(), sd)


def test_hub_rows_wider_than_65536(ctx):
    """Rows wider than 65536 make the level scatter each hub row's ids by
    partition before aggregating; with and without one-pass rows and a
    forced redo the result is the oracle's."""
    h = H.hub_graph(n=150000, m=200000, hubs=(70000, 90000, 20000), seed=31)
    lo, No, _ = O.cluster(H.to_oracle(h), 1, 80, oparams())
    for limit, row_limit in HUB_PATHS:
        ld, Nd, _ = L.lcc_cluster(ctx, dev(h), 1, 80, dparams(hub_limit=limit, hub_row_limit=row_limit))
        assert np.array_equal(lo, ld.cpu().numpy()) and No == Nd, (limit, row_limit)


def test_tiny_and_degenerate_graphs(ctx):
    cases_ = [
        G.HostGraph(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int64)),  # empty
        G.HostGraph(np.zeros(2, np.int64), np.zeros(0, np.int32), np.ones(1, np.int64)),  # one vertex
        G.HostGraph(np.zeros(6, np.int64), np.zeros(0, np.int32), np.ones(5, np.int64)),  # edgeless
        G.HostGraph(np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32), np.ones(2, np.int64)),  # one edge
        G.random_signed(50, 10, 4),  # mostly isolated vertices
        G.random_signed(40, 300, 5, wmin=0, wmax=0),  # all-zero weights
        G.random_signed(40, 300, 6, wmin=-5, wmax=-1),  # all negative
        H.with_k(G.random_signed(60, 200, 7, unit=True), np.zeros(60)),  # k = 0 everywhere
    ]
    for i, h in enumerate(cases_):
        for p, q in [(1, 2), (0, 1), (5, 3)]:
            lo, No, so = O.cluster(H.to_oracle(h), p, q, oparams())
            ld, Nd, sd = L.lcc_cluster(ctx, dev(h), p, q, dparams())
            assert np.array_equal(lo, ld.cpu().numpy()), (i, p, q)
            assert No == Nd, (i, p, q)


def test_lambda_zero_components_on_gpu(ctx):
    """lambda = 0 with non-negative weights: every positive edge ends inside a
    cluster (the objective is q times the total weight)."""
    h = G.random_signed(2000, 2500, 11, wmin=0, wmax=4)
    ld, Nd, sd = L.lcc_cluster(ctx, dev(h), 0, 3, dparams())
    assert sd["top_moved"] == 0
    assert Nd == 3 * int(np.asarray(h.numpy().wt).sum()) // 2


def test_invalid_inputs_are_rejected_before_any_output(ctx):
    h = G.random_signed(100, 300, 1)
    g = dev(h)
    C = torch.arange(100, dtype=torch.int32, device="cuda")
    bad = L.DeviceGraph(off=g.off, col=g.col.clone(), k=g.k, wt=g.wt)
    bad.col[0] = 1000
    with pytest.raises(L.LccError) as e:
        L.lcc_best_move(ctx, bad, 1, 2, dparams(), C)
    assert e.value.code == L.LCC_ERR_INVALID_ARG
    assert torch.equal(C, torch.arange(100, dtype=torch.int32, device="cuda"))
    self_loop = L.DeviceGraph(off=g.off, col=g.col.clone(), k=g.k, wt=g.wt)
    v = int(np.nonzero(np.diff(h.off))[0][0])
    self_loop.col[int(h.off[v])] = v
    with pytest.raises(L.LccError):
        L.lcc_cluster(ctx, self_loop, 1, 2, dparams())
    big = L.DeviceGraph(off=g.off, col=g.col, k=torch.full((100,), 2**40, dtype=torch.int64, device="cuda"), wt=g.wt)
    with pytest.raises(L.LccError) as e:
        L.lcc_cluster(ctx, big, 1, 1, dparams())
    assert e.value.code == L.LCC_ERR_OVERFLOW
    Cbad = C.clone()
    Cbad[5] = 100
    with pytest.raises(L.LccError) as e:
        L.lcc_objective(ctx, g, 1, 2, Cbad)
    assert e.value.code == L.LCC_ERR_INVALID_ARG
    with pytest.raises(L.LccError):
        L.lcc_best_move(ctx, g, -1, 2, dparams(), C)
    short = torch.zeros(10, dtype=torch.int32, device="cuda")
    with pytest.raises(L.LccError) as e:
        L.lcc_best_move(ctx, g, 1, 2, dparams(), short)
    assert e.value.code == L.LCC_ERR_INVALID_ARG
    host_c = torch.arange(100, dtype=torch.int32)
    with pytest.raises(L.LccError):
        L.lcc_best_move(ctx, g, 1, 2, dparams(), host_c)
    # a hub partition limit above the default could drop clusters unnoticed
    for bad_limit in (L.LCC_HUB_LIMIT_MAX + 1, -1):
        with pytest.raises(L.LccError) as e:
            L.lcc_cluster(ctx, g, 1, 2, dparams(hub_limit=bad_limit))
        assert e.value.code == L.LCC_ERR_INVALID_ARG
        with pytest.raises(L.LccError) as e:
            L.lcc_best_move(ctx, g, 1, 2, dparams(hub_limit=bad_limit), C)
        assert e.value.code == L.LCC_ERR_INVALID_ARG
    assert torch.equal(C, torch.arange(100, dtype=torch.int32, device="cuda"))
    lo, No, _ = O.cluster(H.to_oracle(h), 1, 2, oparams())
    ld, Nd, _ = L.lcc_cluster(ctx, g, 1, 2, dparams(hub_limit=L.LCC_HUB_LIMIT_MAX))
    assert np.array_equal(lo, ld.cpu().numpy()) and No == Nd


def test_validation_covers_every_arc(ctx):
    """The arc checks split a block's arcs into per-thread chunks: a bad
    column at the very last arc, a self-loop in the middle of a hub row and
    a repeated arc in the middle of a long row (rows are then not strictly
    ascending, so the singleton shortcut that assumes distinct neighbors
    must not be taken) are all seen."""
    h = H.hub_graph(n=20000, m=40000, hubs=(9000, 3000, 600), seed=41)
    g = dev(h)
    last = L.DeviceGraph(off=g.off, col=g.col.clone(), k=g.k, wt=g.wt)
    last.col[-1] = h.n + 5
    with pytest.raises(L.LccError) as e:
        L.lcc_cluster(ctx, last, 1, 40, dparams())
    assert e.value.code == L.LCC_ERR_INVALID_ARG
    loop = L.DeviceGraph(off=g.off, col=g.col.clone(), k=g.k, wt=g.wt)
    mid = int(h.off[0]) + 4500  # vertex 0 is the 9000-arc hub
    loop.col[mid] = 0
    with pytest.raises(L.LccError) as e:
        L.lcc_cluster(ctx, loop, 1, 40, dparams())
    assert e.value.code == L.LCC_ERR_INVALID_ARG
    # a repeated neighbor in the middle of the hub row (symmetric: the
    # neighbor gets the reverse arc twice as well), rows sorted otherwise
    hn = h.numpy()
    off, col = hn.off.astype(np.int64), hn.col.astype(np.int32)
    wt = None if hn.wt is None else hn.wt.copy()
    rows = [np.sort(col[off[v]:off[v + 1]]) for v in range(hn.n)]
    u = int(rows[0][4500])
    rows[0] = np.sort(np.append(rows[0], u))
    rows[u] = np.sort(np.append(rows[u], 0))
    deg = np.array([len(r) for r in rows], np.int64)
    off2 = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    col2 = np.concatenate(rows).astype(np.int32)
    rep = G.HostGraph(off2, col2, hn.k)
    lo, No, _ = O.cluster(H.to_oracle(rep), 1, 40, oparams())
    ld, Nd, _ = L.lcc_cluster(ctx, dev(rep), 1, 40, dparams())
    assert np.array_equal(lo, ld.cpu().numpy()) and No == Nd


def test_full_size_modularity_graph_sampled(ctx):
    """The 4M-vertex / 100M-edge Chung-Lu modularity workload, in the launch
    configuration the benchmark uses: sampled vertices of the first sub-round
    equal the oracle's one-by-one decision; the first full iteration of
    level-0 Best-Moves (every sub-round) equals the oracle's; three full
    clusterings (with and without event timing) equal the oracle's full
    clustering bit for bit."""
    h = G.chung_lu_planted(4_000_000, 100_000_000, 2.1, 0.3, seed=1, device="cuda")
    g_d = dev(h)
    m2 = h.arcs
    p, q = 1, m2
    S = 4
    C = torch.arange(h.n, dtype=torch.int32, device="cuda")
    L.lcc_best_move(ctx, g_d, p, q, dparams(S=S, stop_after_subrounds=1), C)
    Cd1 = C.cpu().numpy()
    hh = h.numpy()
    g_o = H.to_oracle(hh)
    hr = O.round_hash(1, 0, 0, 0)
    rng = np.random.default_rng(0)
    cand = rng.choice(h.n, size=20000, replace=False)
    U = np.array([v for v in cand if O.color(hr, int(v), S) == 0], dtype=np.int32)[:4000]
    D = O.decide_many(g_o, p, q, np.arange(h.n, dtype=np.int32), U)
    assert np.array_equal(D, Cd1[U])
    # one full iteration, all four sub-rounds, bit-exact
    C = torch.arange(h.n, dtype=torch.int32, device="cuda")
    sd = L.lcc_best_move(ctx, g_d, p, q, dparams(S=S, stop_after_subrounds=S), C)
    Co, so = O.best_move(g_o, p, q, oparams(S=S, stop_after_subrounds=S))
    assert np.array_equal(Co, C.cpu().numpy())
    assert so["moves"] == sd["moves"] and so["arcs_scanned"] == sd["arcs_scanned"]
    # full clustering, repeated with and without per-launch event timing:
    # every run equals the oracle's full clustering
    runs = [L.lcc_cluster(ctx, g_d, p, q, dparams(timing=t)) for t in (1, 0, 1)]
    lo, No, so = O.cluster(g_o, p, q, oparams())
    for lab, N, st in runs:
        assert np.array_equal(lab.cpu().numpy(), lo) and N == No
        assert st["arcs_scanned_total"] == so["arcs_scanned_total"]
    assert O.objective(g_o, p, q, lo) == No


def assert_same_graph_chunked(go, gd, chunk=1 << 27):
    """assert_same_graph for graphs of billions of arcs, compared in chunks."""
    assert gd.n == go.n and gd.arcs == len(go.col)
    for name in ("off", "k", "s", "kk"):
        assert np.array_equal(getattr(go, name), getattr(gd, name).cpu().numpy()), name
    for a in range(0, len(go.col), chunk):
        b = min(a + chunk, len(go.col))
        assert np.array_equal(go.col[a:b], gd.col[a:b].cpu().numpy()), ("col", a)
        assert np.array_equal(go.wt[a:b], gd.wt[a:b].cpu().numpy().astype(np.int64)), ("wt", a)


# The 65.6M-vertex / 1.8B-edge Chung-Lu workload (3.6B arcs, beyond 2^31)
# against the oracle element by element (its OpenMP build, whose results equal
# the single-threaded build's), in steps that share one generated graph: the
# whole first sub-round (host-driven launches), the whole first level-0
# iteration through the device-driven launches the benchmark uses, the
# level-0 contraction of that clustering (every array), and the full
# clustering (its objective evaluated by the oracle on the returned labels;
# with LCC_FULL_ORACLE=1 also labels and hierarchy against the oracle's own
# full clustering).

def progress(msg):
    print(f"[billion-edge] {msg}", flush=True)


@pytest.fixture(scope="module")
def c3():
    state = {}
    yield state
    state.clear()
    torch.cuda.empty_cache()


def c3_graph(state):
    if "g_d" not in state:
        progress("generating the graph")
        h = G.chung_lu_planted(65_608_366, 1_806_067_135, 2.2, 0.4, seed=1, device="cuda")
        state["g_d"] = dev(h)
        torch.cuda.empty_cache()
        state["p"], state["q"] = 1, h.arcs
        hh = h.numpy()
        del h
        state["g_o"] = H.to_oracle(hh)
        progress(f"n={state['g_o'].n} arcs={state['g_o'].arcs}")
    return state["g_d"], state["g_o"], state["p"], state["q"]


def test_billion_edge_first_subround(ctx, c3):
    g_d, g_o, p, q = c3_graph(c3)
    S = 4
    prev = O.use_openmp(True)
    try:
        C = torch.arange(g_o.n, dtype=torch.int32, device="cuda")
        sd = L.lcc_best_move(ctx, g_d, p, q, dparams(S=S, stop_after_subrounds=1), C)
        progress("oracle: first sub-round")
        Co, so = O.best_move(g_o, p, q, oparams(S=S, stop_after_subrounds=1))
        assert np.array_equal(Co, C.cpu().numpy())
        assert so["moves"] == sd["moves"] and so["arcs_scanned"] == sd["arcs_scanned"]
    finally:
        O.use_library(prev)


def test_billion_edge_first_iteration(ctx, c3):
    g_d, g_o, p, q = c3_graph(c3)
    S = 4
    prev = O.use_openmp(True)
    try:
        C = torch.arange(g_o.n, dtype=torch.int32, device="cuda")
        sd = L.lcc_best_move(ctx, g_d, p, q, dparams(S=S, num_iter=1), C)
        progress("oracle: first iteration")
        Co, so = O.best_move(g_o, p, q, oparams(S=S, num_iter=1))
        assert np.array_equal(Co, C.cpu().numpy())
        for key in ("iterations", "subrounds", "moves", "arcs_scanned", "vertices_processed", "term"):
            assert so[key] == sd[key], (key, so[key], sd[key])
        c3["C1"] = Co
    finally:
        O.use_library(prev)


def test_billion_edge_level0_contraction(ctx, c3):
    g_d, g_o, p, q = c3_graph(c3)
    if "C1" not in c3:
        pytest.skip("needs the first-iteration clustering of the previous step")
    C1 = c3.pop("C1")
    prev = O.use_openmp(True)
    try:
        g2d, map_d = L.lcc_compress(ctx, g_d, torch.from_numpy(C1).cuda())
        progress(f"contracted on the GPU: n={g2d.n} arcs={g2d.arcs}; oracle contraction")
        g2o, map_o = O.compress(g_o, C1)
        assert np.array_equal(map_o, map_d.cpu().numpy())
        del map_d, map_o
        progress("comparing the contracted graphs")
        assert_same_graph_chunked(g2o, g2d)
    finally:
        O.use_library(prev)
    del g2d, g2o
    torch.cuda.empty_cache()


def test_billion_edge_full_clustering(ctx, c3):
    import os

    g_d, g_o, p, q = c3_graph(c3)
    lab, N, st = L.lcc_cluster(ctx, g_d, p, q, dparams())
    labh = lab.cpu().numpy()
    assert labh.min() == 0 and labh.max() == st["clusters"] - 1
    progress("oracle: objective of the labels")
    assert O.objective(g_o, p, q, labh) == N
    if os.environ.get("LCC_FULL_ORACLE") == "1":
        prev = O.use_openmp(True)
        try:
            progress("oracle: full clustering")
            lo, No, so = O.cluster(g_o, p, q, oparams())
        finally:
            O.use_library(prev)
        assert np.array_equal(lo, labh) and No == N
        for key in ("levels", "top_moved", "n_level", "arcs_level", "iters_coarsen", "iters_refine",
                    "moves_total", "arcs_scanned_total", "clusters"):
            assert so[key] == st[key], (key, so[key], st[key])
    c3.clear()
    torch.cuda.empty_cache()
