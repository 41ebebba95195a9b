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
