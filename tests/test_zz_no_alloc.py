"""The allocation-free objective (lcc_objective_noalloc) through the C ABI:
equal to lcc_objective on two calls in a row (the second on a smaller graph,
so stale sums of the first call in the shared static scratch would show),
on contracted graphs (self weights and kk), on signed weights of every
storage kind, and with the oracle.  Sizes above LCC_NOALLOC_MAX_N are refused
before any launch."""
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


def clustering(n, seed, clusters):
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.integers(0, max(1, clusters), size=n).astype(np.int32)).cuda()


def both(ctx, h, p, q, C):
    g = L.DeviceGraph.from_host(h, "cuda")
    a = L.lcc_objective(ctx, g, p, q, C)
    b = L.lcc_objective_noalloc(ctx, g, p, q, C)
    return a, b


def test_two_calls_in_a_row_second_smaller(ctx):
    big = G.chung_lu_planted(200000, 2000000, 2.1, 0.3, seed=7)
    small = G.c1_sbm(3)
    C_big = clustering(big.n, 1, 5000)
    C_small = clustering(small.n, 2, 40)
    a1, b1 = both(ctx, big, 1, int(big.arcs), C_big)
    a2, b2 = both(ctx, small, 1, 100, C_small)
    assert a1 == b1
    assert a2 == b2
    g_o = H.to_oracle(small)
    assert b2 == O.objective(g_o, 1, 100, C_small.cpu().numpy())
    # the same small call again, after the big one filled the scratch
    a3, b3 = both(ctx, big, 1, int(big.arcs), C_big)
    assert (a3, b3) == (a1, b1)


def test_labels_of_a_clustering_and_largest_size(ctx):
    h = G.c1_sbm(1)
    g = L.DeviceGraph.from_host(h, "cuda")
    lab, N, _ = L.lcc_cluster(ctx, g, 1, 100, L.Params())
    assert L.lcc_objective_noalloc(ctx, g, 1, 100, lab) == N
    # exactly LCC_NOALLOC_MAX_N vertices: a path graph
    n = L.LCC_NOALLOC_MAX_N
    u = torch.arange(n - 1)
    off, col, _ = G.csr_from_edges(n, u, u + 1, None)
    hp = G.HostGraph(off.numpy(), col.numpy(), np.ones(n, np.int64))
    C = (torch.arange(n, dtype=torch.int32, device="cuda") // 1000).contiguous()
    a, b = both(ctx, hp, 1, 1000, C)
    assert a == b


@pytest.mark.parametrize("kind", ["i16", "i32", "i64"])
def test_signed_weights(ctx, kind):
    h = H.with_weights(G.c1_sbm(2), kind, seed=4, lo=-6, hi=9)
    C = clustering(h.n, 5, 60)
    a, b = both(ctx, h, 2, 7, C)
    assert a == b == O.objective(H.to_oracle(h), 2, 7, C.cpu().numpy())


def test_contracted_graph_with_self_weights(ctx):
    h = H.with_weights(G.c1_sbm(1), "i32", seed=3, lo=-2, hi=7)
    g = L.DeviceGraph.from_host(h, "cuda")
    C0 = clustering(h.n, 8, 700)
    g2, _ = L.lcc_compress(ctx, g, C0)
    C2 = clustering(g2.n, 9, 50)
    a = L.lcc_objective(ctx, g2, 3, 11, C2)
    b = L.lcc_objective_noalloc(ctx, g2, 3, 11, C2)
    assert a == b


def test_refuses_graphs_beyond_the_limit_and_bad_input(ctx):
    n = L.LCC_NOALLOC_MAX_N + 1
    g = L.DeviceGraph(off=torch.zeros(n + 1, dtype=torch.int64, device="cuda"),
                      col=torch.zeros(0, dtype=torch.int32, device="cuda"),
                      k=torch.ones(n, dtype=torch.int64, device="cuda"))
    C = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(L.LccError) as e:
        L.lcc_objective_noalloc(ctx, g, 1, 2, C)
    assert e.value.code == L.LCC_ERR_INVALID_ARG and "LCC_NOALLOC_MAX_N" in str(e.value)
    # a cluster id out of range: the validation pass refuses it, as lcc_objective does
    h = G.c1_sbm(1)
    gd = L.DeviceGraph.from_host(h, "cuda")
    Cb = torch.zeros(h.n, dtype=torch.int32, device="cuda")
    Cb[17] = h.n
    for f in (L.lcc_objective, L.lcc_objective_noalloc):
        with pytest.raises(L.LccError) as e:
            f(ctx, gd, 1, 100, Cb)
        assert e.value.code == L.LCC_ERR_INVALID_ARG
    # the overflow bound, as lcc_objective
    with pytest.raises(L.LccError) as e:
        L.lcc_objective_noalloc(ctx, gd, 2**62, 1, Cb * 0)
    assert e.value.code == L.LCC_ERR_OVERFLOW


def test_empty_graph(ctx):
    g = L.DeviceGraph(off=torch.zeros(1, dtype=torch.int64, device="cuda"),
                      col=torch.zeros(0, dtype=torch.int32, device="cuda"),
                      k=torch.zeros(0, dtype=torch.int64, device="cuda"))
    C = torch.zeros(0, dtype=torch.int32, device="cuda")
    assert L.lcc_objective_noalloc(ctx, g, 1, 2, C) == L.lcc_objective(ctx, g, 1, 2, C) == 0
