"""Serving loop: requests of mixed kinds arrive as a seeded Poisson stream and
are served by continuous batching; every request's labels and objective must
equal the same request run alone, and the CPU oracle's clustering of it."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2108_01731_amd import lcc as L
from paper_2108_01731_amd import serve as V
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trace():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return V.make_trace(36, qps=600.0, seed=5, mmin=500, mmax=60_000, device="cuda")


def alone(tr):
    ctx = L.Context(0)
    out = {}
    for r in tr:
        lab, N, st = L.lcc_cluster(ctx, L.DeviceGraph.from_host(r.graph, "cuda"), r.p, r.q, L.Params())
        out[r.rid] = (lab.cpu().numpy(), N, st["clusters"])
    ctx.close()
    return out


def oracle_ref(tr):
    out = {}
    for r in tr:
        lab, N, st = O.cluster(H.to_oracle(r.graph), r.p, r.q, O.Params())
        out[r.rid] = (lab, N, st["clusters"])
    return out


def check(stats, ref):
    assert len(stats.done) == len(ref)
    for d in stats.done:
        assert d.error is None, (d.rid, d.error)
        lab, N, ncl = ref[d.rid]
        assert np.array_equal(d.labels, lab), f"request {d.rid}: labels differ from the request alone"
        assert d.N == N and d.clusters == ncl, d.rid
        assert d.finished >= d.started >= d.admitted - 1e-6 and d.admitted >= d.arrival - 1e-3


def test_served_results_equal_each_request_alone(trace):
    ref = alone(trace)
    srv = V.Server(0, slots=2)
    try:
        st = srv.serve(trace)
    finally:
        srv.close()
    check(st, ref)
    # and every served request equals the oracle's clustering of it
    check(st, oracle_ref(trace))
    # requests were batched: fewer batches than requests
    assert st.batches < len(trace)
    assert max(d.batch_jobs for d in st.done) > 1


def test_hbm_budget_limits_admission(trace):
    ref = alone(trace)
    ests = sorted(V.hbm_estimate(r.graph) for r in trace)
    budget = ests[-1] + ests[-2]  # room for about two large requests at a time
    srv = V.Server(0, slots=2, hbm_budget=budget)
    try:
        st = srv.serve(trace)
    finally:
        srv.close()
    check(st, ref)
    assert st.peak_hbm_estimate <= budget


def test_over_budget_request_is_refused_others_served(trace):
    ref = alone(trace[:10])
    ests = [V.hbm_estimate(r.graph) for r in trace[:10]]
    big = int(np.argmax(ests))
    budget = max(e for i, e in enumerate(ests) if i != big)
    assert ests[big] > budget
    srv = V.Server(0, slots=2, hbm_budget=budget)
    try:
        st = srv.serve(trace[:10])
    finally:
        srv.close()
    for d in st.done:
        if d.rid == trace[big].rid:
            assert d.error is not None
        else:
            assert d.error is None and np.array_equal(d.labels, ref[d.rid][0])


def test_plain_path_equals_alone(trace):
    ref = alone(trace[:12])
    srv = V.Server(0, plain=True)
    try:
        st = srv.serve(trace[:12])
    finally:
        srv.close()
    check(st, ref)
    assert st.batches == 12
