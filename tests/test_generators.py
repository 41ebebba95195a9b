"""Seeded generators: determinism, validity and the workload shapes."""
import numpy as np
import torch

import oracle as O
from paper_2108_01731_amd import graphgen as G


def _og(h):
    h = h.numpy()
    return O.Graph(off=h.off, col=h.col, k=h.k, wt=None if h.wt is None else h.wt.astype(np.int64))


def test_sbm_small_config_shape_and_determinism():
    a = G.c1_sbm(1)
    b = G.c1_sbm(1)
    assert torch.equal(a.off, b.off) and torch.equal(a.col, b.col)
    assert a.n == 10000
    m = a.arcs // 2
    # E[m] = 20 * C(500,2) * 0.02 + C(20,2) * 500^2 * 0.0005 = 49,900 + 23,750
    assert abs(m - 73650) < 4 * 300
    g = _og(a)
    assert O.validate(g) == O.OK and O.check_symmetric(g)
    c = G.c1_sbm(2)
    assert not torch.equal(a.col[:1000], c.col[:1000])


def test_chung_lu_small_shape():
    h = G.chung_lu_planted(20000, 200000, 2.1, 0.3, seed=3)
    g = _og(h)
    assert O.validate(g) == O.OK and O.check_symmetric(g)
    deg = np.diff(g.off)
    assert np.array_equal(g.k, deg)  # modularity setting: k = degree
    assert g.arcs // 2 == 200000
    assert deg.max() <= 1.3 * np.sqrt(2 * 200000) + 50
    h2 = G.chung_lu_planted(20000, 200000, 2.1, 0.3, seed=3)
    assert torch.equal(h.col, h2.col)


def test_knn_weights_are_q15_and_symmetric():
    h = G.knn_gaussian(2000, 20, 16, 10, 0.3, seed=4)
    assert h.wt.dtype == torch.int16
    g = _og(h)
    assert O.validate(g) == O.OK and O.check_symmetric(g)
    deg = np.diff(g.off)
    assert deg.min() >= 10


def test_random_signed_valid():
    for s in range(5):
        g = _og(G.random_signed(30, 80, s))
        assert O.validate(g) == O.OK and O.check_symmetric(g)


def test_range_built_csr_equals_sort_built():
    """The range-by-range relabelled CSR (for graphs beyond 2^31 arcs) equals
    the single-sort build followed by the relabel, for any range size."""
    gen = torch.Generator().manual_seed(3)
    n = 3000
    u = torch.randint(0, n, (30000,), generator=gen)
    v = torch.randint(0, n, (30000,), generator=gen)
    keep = u != v
    key = torch.unique(torch.minimum(u[keep], v[keep]) * n + torch.maximum(u[keep], v[keep]))
    a, b = key // n, key % n
    perm = torch.randperm(n, generator=gen)
    o1, c1, _ = G.csr_from_edges(n, a, b)
    o1, c1, _ = G.relabel(o1, c1, None, perm)
    for max_arcs in (1 << 30, 2000, 7):
        o2, c2 = G.csr_relabeled(n, a, b, perm, max_arcs=max_arcs)
        assert torch.equal(o1, o2) and torch.equal(c1.to(torch.int32), c2), max_arcs


def test_hash_order_is_a_seeded_permutation():
    p = G._hash_perm(5000, 7, "cpu")
    assert torch.equal(torch.sort(p).values, torch.arange(5000))
    assert torch.equal(p, G._hash_perm(5000, 7, "cpu"))
    assert not torch.equal(p, G._hash_perm(5000, 8, "cpu"))
    # the mixing reaches every bit: each of the 64 bits is set about half the time
    h = G._hash64(torch.arange(1 << 14), 1)
    bits = torch.stack([(h >> k) & 1 for k in range(64)]).float().mean(dim=1)
    assert bool(((bits > 0.45) & (bits < 0.55)).all())


def test_pack_and_slice_round_trip():
    gs = [G.sbm_blocks(n, 100, 8.0, 0.2, seed=i) for i, n in enumerate([0, 1, 60, 250])]
    gs.append(G.random_signed(80, 300, 5, wmin=-3, wmax=4, kmax=2, unit=True))
    P, start = G.pack(gs)
    assert list(np.diff(start)) == [g.n for g in gs]
    g = _og(P)
    assert O.validate(g) == O.OK and O.check_symmetric(g)
    for j, h in enumerate(gs):
        s = G.job_slice(P, start, j)
        hn = h.numpy()
        assert np.array_equal(s.off, hn.off) and np.array_equal(s.col, hn.col) and np.array_equal(s.k, hn.k)
    Pt, st = G.pack_torch([G.HostGraph(*(torch.as_tensor(x) if x is not None else None
                                         for x in (h.off, h.col, h.k, h.wt, h.s, h.kk)), h.wt_kind)
                           for h in (g_.numpy() for g_ in gs)], "cpu")
    assert np.array_equal(st, start) and np.array_equal(Pt.col.numpy(), P.col)


def test_sbm_blocks_degree_and_blocks():
    h = G.sbm_blocks(4000, 500, 20.0, 0.2, seed=5)
    g = _og(h)
    assert O.validate(g) == O.OK and O.check_symmetric(g)
    assert abs(g.arcs / g.n - 20.0) < 1.5
