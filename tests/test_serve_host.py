"""Host-side pieces of the serving loop (no GPU): the seeded trace and the
HBM estimate used for admission."""
import numpy as np

from paper_2108_01731_amd import graphgen as G
from paper_2108_01731_amd import serve as V


def test_trace_is_seeded_and_poisson():
    a = V.make_trace(30, qps=200.0, seed=3, mmin=500, mmax=5000)
    b = V.make_trace(30, qps=200.0, seed=3, mmin=500, mmax=5000)
    assert [r.arrival for r in a] == [r.arrival for r in b]
    assert all(np.array_equal(x.graph.col, y.graph.col) and (x.p, x.q) == (y.p, y.q) for x, y in zip(a, b))
    arr = np.array([r.arrival for r in a])
    assert np.all(np.diff(arr) > 0)
    assert {r.kind for r in a} == {"sbm", "chung_lu", "knn"}
    # a long exponential trace has mean gap 1/qps
    gaps = np.diff([r.arrival for r in V.retime(a * 100, 50.0, seed=1)])
    assert abs(gaps.mean() - 1 / 50.0) < 0.1 / 50.0


def test_request_graphs_are_valid_and_sized():
    for kind in ("sbm", "chung_lu", "knn"):
        for m in (800, 20000):
            g, (p, q) = V.request_graph(kind, m, seed=m)
            h = g.numpy()
            assert p >= 1 and q >= 1
            assert h.off[0] == 0 and h.off[-1] == len(h.col)
            src = np.repeat(np.arange(h.n), np.diff(h.off))
            assert np.all(src != h.col)
            assert 0.3 * m <= h.arcs // 2 <= 1.5 * m, (kind, m, h.arcs // 2)
            if kind == "knn":
                assert h.wt_kind == "i16"


def test_hbm_estimate_grows_with_the_graph():
    small = G.sbm_blocks(200, 100, 10, 0.2, seed=1).numpy()
    big = G.sbm_blocks(2000, 100, 10, 0.2, seed=1).numpy()
    es, eb = V.hbm_estimate(small), V.hbm_estimate(big)
    assert es < eb
    # at least two copies of the graph arrays
    assert eb >= 2 * (8 * (big.n + 1) + 4 * big.arcs + 8 * big.n)
