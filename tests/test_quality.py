"""Average precision / recall against ground-truth communities (the paper's
quality measure, Sec. 4 setup): each community is matched to the cluster
sharing most of its vertices.  Hand-computed cases and limiting clusterings."""
import numpy as np
import pytest

from paper_2108_01731_amd import graphgen as G
from paper_2108_01731_amd import quality as Q


def test_hand_computed_example():
    # community 0 = {0,1,2}: meets cluster 5 in 2 vertices, cluster 7 in 1 ->
    # cluster 5 (size 2): P = 1, R = 2/3; community 1 = {3,4}: cluster 7
    # (size 4): P = 2/4, R = 1; vertex 5 is in no community
    comm = np.array([0, 0, 0, 1, 1, -1])
    lab = np.array([5, 5, 7, 7, 7, 7])
    p, r, k = Q.precision_recall(lab, comm)
    assert k == 2
    assert p == pytest.approx((1 + 0.5) / 2) and r == pytest.approx((2 / 3 + 1) / 2)


def test_ties_go_to_the_smallest_label():
    p, r, _ = Q.precision_recall(np.array([3, 1, 1, 3, 3]), np.array([0, 0, -1, -1, -1]))
    # community {0, 1} meets clusters 3 and 1 once each: cluster 1 (size 2)
    assert p == pytest.approx(0.5) and r == pytest.approx(0.5)


def test_limiting_clusterings():
    rng = np.random.default_rng(0)
    comm = rng.integers(0, 30, size=500)
    sizes = np.bincount(comm)
    assert Q.precision_recall(comm * 7 + 3, comm)[:2] == (1.0, 1.0)  # the communities themselves
    p, r, _ = Q.precision_recall(np.arange(500), comm)  # singletons
    assert p == 1.0 and r == pytest.approx(np.mean(1.0 / sizes[sizes > 0]))
    p, r, _ = Q.precision_recall(np.zeros(500, np.int64), comm)  # one cluster
    assert r == 1.0 and p == pytest.approx(np.mean(sizes[sizes > 0] / 500))


def test_top_communities_by_size():
    comm = np.array([0, 0, 0, 1, 1, 2, -1])
    lab = np.array([0, 0, 1, 1, 1, 2, 2])
    p, r, k = Q.precision_recall(lab, comm, top=2)
    assert k == 2  # communities 0 (3 vertices) and 1 (2 vertices)
    assert p == pytest.approx((1 + 2 / 3) / 2) and r == pytest.approx((2 / 3 + 1) / 2)


def test_planted_communities_of_the_generator():
    """The Chung-Lu generator's planted communities hold most edges (mixing
    0.3: about 70% of the draws stay inside a community) and score perfectly
    against themselves."""
    h, comm = G.chung_lu_planted(20000, 200000, 2.1, 0.3, seed=3, return_communities=True)
    off, col = h.off.numpy(), h.col.numpy()
    src = np.repeat(np.arange(h.n), np.diff(off))
    assert (comm[src] == comm[col]).mean() > 0.7
    sizes = np.bincount(comm)
    assert sizes.min() >= 20 and sizes.max() <= 5000
    assert Q.precision_recall(comm, comm)[:2] == (1.0, 1.0)
