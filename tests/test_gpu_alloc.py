"""Contexts whose device memory comes from the caller's allocator (here
torch's caching allocator through lcc_allocator callbacks): results equal a
default context's and the oracle's, the library's scratch and returned graphs
live in the caller's pool while held and go back to it when released, and
growing buffers (a larger graph after a smaller one) change no result."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2108_01731_amd import graphgen as G
from paper_2108_01731_amd import lcc as L
from tests import helpers as H

pytestmark = pytest.mark.gpu


def test_torch_pool_context_equals_default_and_oracle():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    alloc = L.TorchAllocator(0)
    ctx_t = L.Context(0, alloc)
    ctx_d = L.Context(0)
    try:
        cases = [(G.c1_sbm(1), 1, 100), (H.hub_graph(n=40000, m=60000, hubs=(16000, 25000, 31000, 14500), seed=21), 1, 60),
                 (G.c1_sbm(2), 1, 100)]  # small, larger (buffers grow), small again
        for h, p, q in cases:
            g = L.DeviceGraph.from_host(h, "cuda")
            lt, Nt, st = L.lcc_cluster(ctx_t, g, p, q, L.Params())
            ld, Nd, sd = L.lcc_cluster(ctx_d, g, p, q, L.Params())
            assert torch.equal(lt, ld) and Nt == Nd
            lo, No, _ = O.cluster(H.to_oracle(h), p, q, O.Params())
            assert np.array_equal(lt.cpu().numpy(), lo) and Nt == No
            assert alloc.live, "the library's scratch should come from the pool"
        held = sum(alloc.live.values())
        assert torch.cuda.memory_allocated(0) >= held
        # a returned graph comes from the pool and goes back when freed
        h = G.c1_sbm(1)
        g = L.DeviceGraph.from_host(h, "cuda")
        C = torch.from_numpy(np.random.default_rng(1).integers(0, 300, size=h.n).astype(np.int32)).cuda()
        before = dict(alloc.live)
        gc_t, mp_t = L.lcc_compress(ctx_t, g, C)
        gc_d, mp_d = L.lcc_compress(ctx_d, g, C)
        assert torch.equal(mp_t, mp_d) and torch.equal(gc_t.col, gc_d.col) and torch.equal(gc_t.wt, gc_d.wt)
        assert set(alloc.live) >= set(before)
    finally:
        ctx_t.close()
        ctx_d.close()
    assert not alloc.live, "every block goes back to the pool when the context is destroyed"


def test_allocator_returning_null_is_out_of_memory():
    """An allocator that refuses every request: the call fails with
    LCC_ERR_OUT_OF_MEMORY before any kernel runs on unallocated memory."""
    import ctypes

    fn_a = L._ALLOC_FN(lambda user, nbytes, stream: None)
    fn_f = L._FREE_FN(lambda user, ptr, nbytes, stream: None)

    class Refusing:
        def __init__(self):
            self._a, self._f = fn_a, fn_f
            self.c = L._Allocator(fn_a, fn_f, None)

    ctx = L.Context(0, Refusing())
    try:
        h = G.c1_sbm(1)
        with pytest.raises(L.LccError) as e:
            L.lcc_cluster(ctx, L.DeviceGraph.from_host(h, "cuda"), 1, 100, L.Params())
        assert e.value.code == L.LCC_ERR_OUT_OF_MEMORY
    finally:
        ctx.close()
