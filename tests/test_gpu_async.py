"""The asynchronous mode (the paper's setting of Sec. 3.2.1: a move is
applied the moment it is decided).  It is not deterministic, so it is not
compared with the oracle bit for bit; what must hold on every run:

* the labels are a canonical clustering and the returned numerator is the
  exact objective of those labels (checked by the oracle);
* an asynchronous Best-Moves call leaves ids in [0, n), from which the
  deterministic path continues exactly as the oracle does.
Its objective over seeds, against the deterministic schedule's, is recorded
by the benchmark's report (at full GPU concurrency most decisions of a
sub-round do not see each other's moves, so it is not the better setting it
is on the paper's CPUs)."""
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


def cases():
    cl = G.chung_lu_planted(60000, 900000, 2.1, 0.3, seed=8)
    return [("sbm_c1", G.c1_sbm(1), 1, 100), ("chung_lu", cl, 1, int(cl.arcs)),
            ("hubs", H.hub_graph(n=40000, m=60000, hubs=(16000, 25000, 31000, 14500), seed=21), 1, 60),
            ("signed", G.random_signed(5000, 30000, 3, wmin=-4, wmax=6, kmax=3), 1, 9)]


@pytest.mark.parametrize("idx", range(4))
def test_async_clusterings_are_valid_with_exact_objective(ctx, idx):
    name, h, p, q = cases()[idx]
    g = L.DeviceGraph.from_host(h, "cuda")
    g_o = H.to_oracle(h)
    for seed in range(3):
        for S in (1, 4):
            for fr in (0, 1, 2):
                lab, N, st = L.lcc_cluster(ctx, g, p, q, L.Params(S=S, seed=seed, frontier=fr, async_moves=1))
                labh = lab.cpu().numpy()
                assert np.array_equal(labh, O.canonical_labels(labh)), (name, seed, S, fr)
                assert O.objective(g_o, p, q, labh) == N, (name, seed, S, fr)
                assert st["clusters"] == labh.max() + 1


@pytest.mark.parametrize("idx", range(4))
def test_async_best_move_leaves_a_valid_clustering(ctx, idx):
    """One asynchronous Best-Moves call: cluster ids stay in [0, n) (fresh
    ids renamed), and the deterministic path continues from its clustering
    exactly as the oracle does (sub-round by sub-round)."""
    name, h, p, q = cases()[idx]
    g = L.DeviceGraph.from_host(h, "cuda")
    g_o = H.to_oracle(h)
    C = torch.arange(h.n, dtype=torch.int32, device="cuda")
    L.lcc_best_move(ctx, g, p, q, L.Params(S=4, num_iter=3, async_moves=1), C)
    Ch = C.cpu().numpy()
    assert Ch.min() >= 0 and Ch.max() < h.n
    Cd = C.clone()
    L.lcc_best_move(ctx, g, p, q, L.Params(S=4, stop_after_subrounds=5), Cd, level=1, phase=1)
    Co, _ = O.best_move(g_o, p, q, O.Params(S=4, stop_after_subrounds=5), Ch, level=1, phase=1)
    assert np.array_equal(Cd.cpu().numpy(), Co)


def test_async_rejects_bad_flag(ctx):
    g = L.DeviceGraph.from_host(G.c1_sbm(1), "cuda")
    with pytest.raises(L.LccError) as e:
        L.lcc_cluster(ctx, g, 1, 100, L.Params(async_moves=2))
    assert e.value.code == L.LCC_ERR_INVALID_ARG
