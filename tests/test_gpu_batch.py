"""Batched runs: many jobs packed block-diagonally through lcc_cluster_batch.
Every job's labels, objective numerator, cluster count and hierarchy depth
must equal those of the same job run alone (lcc_cluster on the GPU, and the
CPU oracle), bit for bit."""
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


def run_batch(ctx, graphs, lambdas, cfg):
    P, start = G.pack(graphs)
    lab, jobs, st = L.lcc_cluster_batch(ctx, dev(P), start, lambdas, L.Params(**cfg))
    lab = lab.cpu().numpy()
    return [lab[start[j]:start[j + 1]] for j in range(len(graphs))], jobs, st


def check_against_alone(ctx, graphs, lambdas, cfg, oracle_jobs=None):
    labs, jobs, _ = run_batch(ctx, graphs, lambdas, cfg)
    for j, (h, (p, q)) in enumerate(zip(graphs, lambdas)):
        ld, Nd, sd = L.lcc_cluster(ctx, dev(h), p, q, L.Params(**cfg))
        ld = ld.cpu().numpy()
        assert np.array_equal(labs[j], ld), f"job {j} (n={h.n}) labels differ from the job alone"
        assert jobs[j]["N"] == Nd, (j, jobs[j]["N"], Nd)
        assert jobs[j]["clusters"] == sd["clusters"], j
        assert jobs[j]["levels"] == sd["levels"], (j, jobs[j]["levels"], sd["levels"])
        assert jobs[j]["top_moved"] == sd["top_moved"], j
        if oracle_jobs is None or j in oracle_jobs:
            ocfg = {k: v for k, v in cfg.items() if k != "hub_limit"}  # a tuning field: no oracle counterpart
            lo, No, so = O.cluster(H.to_oracle(h), p, q, O.Params(**ocfg))
            assert np.array_equal(labs[j], lo), f"job {j} labels differ from the oracle"
            assert jobs[j]["N"] == No, j
    return labs, jobs


def sbm_jobs(count, seed, nmax=1500):
    graphs, lams = [], []
    rng = np.random.default_rng(seed)
    for i in range(count):
        n = int(rng.integers(2, nmax))
        graphs.append(G.sbm_blocks(n, 120, float(rng.uniform(6, 20)), 0.2, seed=seed * 1000 + i))
        lams.append((int(rng.integers(1, 501)), 1000))
    return graphs, lams


CFGS = [dict(), dict(S=2, refine=0), dict(S=8, frontier=0, num_iter=20), dict(frontier=2), dict(allow_isolate=0),
        dict(max_levels=2), dict(S=1, num_iter=6, max_levels=4), dict(num_iter=1)]


@pytest.mark.parametrize("cfg", CFGS)
def test_batch_equals_each_job_alone(ctx, cfg):
    graphs, lams = sbm_jobs(9, seed=4)
    # degenerate jobs: empty, one vertex, two vertices joined by an edge
    graphs += [G.HostGraph(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int64)),
               G.HostGraph(np.zeros(2, np.int64), np.zeros(0, np.int32), np.ones(1, np.int64)),
               G.HostGraph(np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32), np.ones(2, np.int64))]
    lams += [(3, 7), (1, 2), (1, 4)]
    order = np.random.default_rng(1).permutation(len(graphs))
    graphs = [graphs[i] for i in order]
    lams = [lams[i] for i in order]
    check_against_alone(ctx, graphs, lams, cfg)


def test_batch_signed_weights_and_vertex_weights(ctx):
    graphs, lams = [], []
    for i in range(6):
        h = G.random_signed(300 + 150 * i, 1200 + 500 * i, seed=40 + i, wmin=-4, wmax=6, kmax=3)
        graphs.append(H.with_weights(h, "i64", seed=i, lo=-3, hi=9))
        lams.append((1 + i, 9 + 2 * i))
    check_against_alone(ctx, graphs, lams, dict())
    check_against_alone(ctx, graphs, lams, dict(S=3, frontier=0))


def test_lambda_sweep_on_one_knn_graph(ctx):
    """16 resolutions on one Q1.15-weighted kNN graph: lambda = r * 2^15 with
    r geometric in [0.01, 0.85] as p / 1000."""
    h = G.knn_gaussian(2500, 25, 16, 10, 0.4, seed=7).numpy()
    rs = np.geomspace(0.01, 0.85, 16)
    lams = [(int(round(r * 1000)) * 32768, 1000) for r in rs]
    labs, jobs = check_against_alone(ctx, [h] * 16, lams, dict(), oracle_jobs={0, 7, 15})
    # larger lambda never gives fewer clusters on this graph family
    assert jobs[0]["clusters"] <= jobs[-1]["clusters"]


def test_batch_hub_rows_every_bin(ctx):
    graphs = [H.hub_graph(), H.hub_graph(weighted=True, seed=9),
              H.hub_graph(n=40000, m=60000, hubs=(16000, 25000, 31000, 14500), seed=21)]
    lams = [(1, 40), (1, 25), (1, 60)]
    check_against_alone(ctx, graphs, lams, dict())


def test_batch_hub_partition_overflow_redo(ctx):
    """A tiny hub_limit makes the hub partitions overflow inside a batch: the
    batched call is redone with the global tables and every job still equals
    the job alone (and the oracle)."""
    graphs = [H.hub_graph(n=40000, m=60000, hubs=(16000, 25000, 31000, 14500), seed=21), H.hub_graph(seed=9)]
    lams = [(1, 60), (1, 40)]
    check_against_alone(ctx, graphs, lams, dict(hub_limit=64), oracle_jobs={0})


def test_many_small_jobs_deterministic(ctx):
    graphs, lams = sbm_jobs(200, seed=11, nmax=400)
    a = run_batch(ctx, graphs, lams, dict())
    b = run_batch(ctx, graphs, lams, dict())
    for j in range(len(graphs)):
        assert np.array_equal(a[0][j], b[0][j])
    assert [x["N"] for x in a[1]] == [x["N"] for x in b[1]]
    for j in range(0, len(graphs), 17):
        ld, Nd, sd = L.lcc_cluster(ctx, dev(graphs[j]), *lams[j], L.Params())
        assert np.array_equal(a[0][j], ld.cpu().numpy()), j
        assert a[1][j]["N"] == Nd


def test_batch_rejects_invalid_input(ctx):
    graphs, lams = sbm_jobs(3, seed=2, nmax=200)
    P, start = G.pack(graphs)
    d = dev(P)
    # job_start must partition [0, n)
    for bad in ([0, start[1], start[2], P.n - 1], [1, start[1], start[2], P.n], [0, start[2], start[1], P.n]):
        with pytest.raises(L.LccError) as e:
            L.lcc_cluster_batch(ctx, d, bad, lams, L.Params())
        assert e.value.code == L.LCC_ERR_INVALID_ARG
    with pytest.raises(L.LccError) as e:
        L.lcc_cluster_batch(ctx, d, start, lams, L.Params(stop_after_subrounds=1))
    assert e.value.code == L.LCC_ERR_INVALID_ARG
    # splitting a job in two leaves arcs across the split
    with pytest.raises(L.LccError) as e:
        split = [0, start[1] // 2, start[1], start[2], P.n]
        L.lcc_cluster_batch(ctx, d, split, lams[:1] + lams, L.Params())
    assert e.value.code == L.LCC_ERR_INVALID_ARG
    # the overflow bounds hold per job, under each job's own lambda
    with pytest.raises(L.LccError) as e:
        L.lcc_cluster_batch(ctx, d, start, [lams[0], (2**62, 1), lams[2]], L.Params())
    assert e.value.code == L.LCC_ERR_OVERFLOW
    assert "job 1" in str(e.value)
    # an empty batch is fine
    E = G.HostGraph(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int64))
    lab, jobs, st = L.lcc_cluster_batch(ctx, dev(E), [0], [], L.Params())
    assert lab.numel() == 0 and jobs == []


def test_config_batch_sampled_jobs_equal_the_oracle(ctx):
    """The 4096-job SBM batch at its full shape (n log-uniform in [100,
    50000], average degree in [8, 40], each job its own lambda), in the one
    lcc_cluster_batch call the benchmark times: a sample of jobs (the largest,
    the smallest and six seeded others) equals the oracle's clustering of the
    job alone, labels, numerator and cluster count."""
    graphs, lams = G.sbm_batch(4096, 0, device="cuda")
    P, start = G.pack_torch(graphs, "cuda")
    lab, jobs, _ = L.lcc_cluster_batch(ctx, dev(P), start, lams, L.Params())
    lab = lab.cpu().numpy()
    ns = [g.n for g in graphs]
    pick = {int(np.argmax(ns)), int(np.argmin(ns))}
    pick |= set(int(x) for x in np.random.default_rng(3).choice(len(graphs), 6, replace=False))
    for j in sorted(pick):
        lo, No, so = O.cluster(H.to_oracle(graphs[j]), *lams[j], O.Params())
        assert np.array_equal(lab[start[j]:start[j + 1]], lo), f"job {j} (n={ns[j]}) differs from the oracle"
        assert jobs[j]["N"] == No and jobs[j]["clusters"] == so["clusters"], j
