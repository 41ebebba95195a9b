"""Resolution sweeps through lcc_sweep: one graph clustered under up to 16
lambdas at once.  Every resolution's labels, objective numerator, cluster
count, hierarchy depth and top-level move flag must equal those of
lcc_cluster on the same graph and lambda (and the CPU oracle's on a few),
bit for bit."""
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


def check(ctx, h, lams, cfg, oracle_js=()):
    d = dev(h)
    lab, jobs, st = L.lcc_sweep(ctx, d, lams, L.Params(**cfg))
    assert tuple(lab.shape) == (len(lams), h.n)
    lab = lab.cpu().numpy()
    for j, (p, q) in enumerate(lams):
        ld, Nd, sd = L.lcc_cluster(ctx, d, p, q, L.Params(**cfg))
        assert np.array_equal(lab[j], ld.cpu().numpy()), f"resolution {j} ({p}/{q}): labels differ from lcc_cluster"
        assert jobs[j]["N"] == Nd, (j, jobs[j]["N"], Nd)
        assert jobs[j]["clusters"] == sd["clusters"], j
        assert jobs[j]["levels"] == sd["levels"], (j, jobs[j]["levels"], sd["levels"])
        assert jobs[j]["top_moved"] == sd["top_moved"], j
        if j in oracle_js:
            lo, No, _ = O.cluster(H.to_oracle(h), p, q, O.Params(**cfg))
            assert np.array_equal(lab[j], lo), f"resolution {j}: labels differ from the oracle"
            assert jobs[j]["N"] == No, j
    return lab, jobs, st


def knn_lambdas(count):
    rs = np.geomspace(0.01, 0.85, count)
    return [(int(round(r * 1000)) * 32768, 1000) for r in rs]


@pytest.fixture(scope="module")
def knn():
    # 16 x 2500 packed vertices: above the small-level size, so level 0 takes
    # the shared-row launches
    return G.knn_gaussian(2500, 25, 16, 10, 0.4, seed=7).numpy()


CFGS = [dict(), dict(S=2, refine=0), dict(S=8, frontier=0, num_iter=20), dict(frontier=2), dict(allow_isolate=0),
        dict(max_levels=2), dict(S=1, num_iter=6), dict(num_iter=1)]


@pytest.mark.parametrize("cfg", CFGS)
def test_sweep_equals_each_resolution_alone(ctx, knn, cfg):
    check(ctx, knn, knn_lambdas(16), cfg, oracle_js={0, 15} if not cfg else ())


def test_sweep_fewer_resolutions_signed_weights(ctx):
    h = H.with_weights(G.random_signed(3000, 12000, seed=44, wmin=-4, wmax=6, kmax=3), "i64", seed=3, lo=-3, hi=9)
    lams = [(1, 9), (2, 11), (3, 13), (5, 7), (1, 40)]
    check(ctx, h, lams, dict(), oracle_js={1})
    check(ctx, h, lams, dict(S=3, frontier=0))


def test_sweep_rows_of_every_bin(ctx):
    # hub rows (wider than the shared launch takes) next to low-degree rows
    h = H.hub_graph(n=6000, m=20000, seed=5)
    check(ctx, h, [(1, 40), (1, 25), (3, 50), (1, 400)], dict())


def test_sweep_small_levels(ctx):
    # 16 x 400 vertices fit the small-level path from level 0 on
    h = G.knn_gaussian(400, 8, 8, 6, 0.5, seed=3).numpy()
    check(ctx, h, knn_lambdas(16), dict(), oracle_js={3})


def test_sweep_deterministic(ctx, knn):
    d = dev(knn)
    a, ja, _ = L.lcc_sweep(ctx, d, knn_lambdas(16), L.Params())
    b, jb, _ = L.lcc_sweep(ctx, d, knn_lambdas(16), L.Params())
    assert torch.equal(a, b) and [x["N"] for x in ja] == [x["N"] for x in jb]


def test_sweep_edge_cases(ctx, knn):
    d = dev(knn)
    # one resolution, and none
    lab, jobs, _ = L.lcc_sweep(ctx, d, [(3, 1000)], L.Params())
    ld, Nd, _ = L.lcc_cluster(ctx, d, 3, 1000, L.Params())
    assert torch.equal(lab[0], ld) and jobs[0]["N"] == Nd
    lab, jobs, _ = L.lcc_sweep(ctx, d, [], L.Params())
    assert lab.numel() == 0 and jobs == []
    # an empty graph
    E = G.HostGraph(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int64))
    lab, jobs, _ = L.lcc_sweep(ctx, dev(E), [(1, 2), (3, 4)], L.Params())
    assert lab.shape == (2, 0) and [x["N"] for x in jobs] == [0, 0]
    # too many resolutions, stopping inside an iteration, per-resolution overflow
    with pytest.raises(L.LccError) as e:
        L.lcc_sweep(ctx, d, knn_lambdas(17), L.Params())
    assert e.value.code == L.LCC_ERR_INVALID_ARG
    with pytest.raises(L.LccError) as e:
        L.lcc_sweep(ctx, d, knn_lambdas(4), L.Params(stop_after_subrounds=1))
    assert e.value.code == L.LCC_ERR_INVALID_ARG
    with pytest.raises(L.LccError) as e:
        L.lcc_sweep(ctx, d, [(1, 2), (3, 4), (2**62, 1)], L.Params())
    assert e.value.code == L.LCC_ERR_OVERFLOW and "lambda 2" in str(e.value)


def test_config_sweep_ends_equal_the_oracle(ctx):
    """The 16-value sweep on the 1M-point cosine kNN graph at its full shape
    (1000-center 64-d Gaussian mixture, k = 50, Q1.15 weights), in the one
    lcc_sweep call the benchmark times: the two ends of the lambda grid equal
    the oracle's clustering (its OpenMP build) of the graph at that lambda."""
    h = G.knn_gaussian(1_000_000, 1000, 64, 50, 1.0, seed=1, device="cuda")
    lams = knn_lambdas(16)
    lab, jobs, _ = L.lcc_sweep(ctx, dev(h), lams, L.Params())
    lab = lab.cpu().numpy()
    g_o = H.to_oracle(h)
    prev = O.use_openmp(True)
    try:
        for j in (0, len(lams) - 1):
            lo, No, so = O.cluster(g_o, *lams[j], O.Params())
            assert np.array_equal(lab[j], lo), f"resolution {j} differs from the oracle"
            assert jobs[j]["N"] == No and jobs[j]["clusters"] == so["clusters"], j
    finally:
        O.use_library(prev)
