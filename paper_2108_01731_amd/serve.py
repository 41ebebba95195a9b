"""Serving loop: clustering requests arrive over time and are served by
continuous batching on one GPU.

Pipeline (one condition variable guards the queues and the HBM ledger):

  arrival -> pending (FIFO) -> admitted: graph uploaded and resident in HBM
          -> ready -> a free worker takes every ready request that stores its
             weights like the oldest ready one (up to its caps), packs them
             block-diagonally on its own stream and runs one
             lcc_cluster_batch -> labels copied out, HBM released -> done

Admission: a request is admitted only while the sum of the HBM estimates of
the admitted, unfinished requests stays within the budget; requests are
admitted in arrival order (the head of the queue waits for room).  Workers
are slots: each owns a library context and a HIP stream, so batches formed
while another batch is on the GPU run concurrently with it.  Requests that
arrive during a batch join the next free slot.  Every job's result equals the
job run alone (lcc_cluster), which the tests check.

The plain path for comparison runs the same trace with one slot that takes
one request at a time through lcc_cluster.
"""
from __future__ import annotations

import math
import threading
import time
from collections import deque
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import graphgen as G
from . import lcc


@dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the trace
    graph: G.HostGraph  # host (numpy) arrays
    p: int
    q: int
    kind: str = ""


@dataclass
class Done:
    rid: int
    labels: np.ndarray
    N: int
    clusters: int
    arrival: float
    admitted: float
    started: float
    finished: float
    batch_jobs: int
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def hbm_estimate(g: G.HostGraph) -> int:
    """Bytes a request may occupy while in flight: its resident graph, the
    packed copy inside a batch, per-level clustering state (about 64 B per
    vertex over the hierarchy) and the compression sort buffers (about 40 B
    per arc)."""
    n, m = g.n, g.arcs
    wb = 0 if g.wt is None else g.wt.element_size() if isinstance(g.wt, torch.Tensor) else np.asarray(g.wt).itemsize
    resident = 8 * (n + 1) + (4 + wb) * m + 8 * n * (1 + (g.s is not None) + (g.kk is not None))
    return 2 * resident + 64 * n + 40 * m + 4096


# ----------------------------------------------------------------- traces


def request_graph(kind: str, m: int, seed: int, device="cpu"):
    """A request graph of about m undirected edges, and its lambda (p, q).

    sbm: blocks of ~500, average degree uniform in [8, 40], k = 1,
         lambda = p/1000 with p uniform in [1, 500];
    chung_lu: degree exponent 2.1, mixing 0.3, average degree uniform in
         [8, 40], k = degree, lambda = r/(2m) with r = p/100;
    knn: cosine 10-NN graph of a 16-d Gaussian mixture (one center per 1000
         points, sigma 1.0), Q1.15 weights, k = 1, lambda = (p/1000) * 2^15."""
    rng = np.random.default_rng([seed, 7])
    p = int(rng.integers(1, 501))
    if kind == "sbm":
        d = float(rng.uniform(8, 40))
        n = max(20, int(round(2 * m / d)))
        g = G.sbm_blocks(n, 500, d, 0.2, seed=seed, device=device)
        return g, (p, 1000)
    if kind == "chung_lu":
        d = float(rng.uniform(8, 40))
        n = max(20, int(round(2 * m / d)))
        g = G.chung_lu_planted(n, m, 2.1, 0.3, seed=seed, device=device, comm_max=min(5000, max(20, n // 2)))
        return g, (p, 100 * max(1, g.arcs))
    if kind == "knn":
        pts = max(20, m // 8)
        g = G.knn_gaussian(pts, max(2, pts // 1000), 16, 10, 1.0, seed=seed, device=device)
        return g, (p * 32768, 1000)
    raise ValueError(kind)


def pinned(g: G.HostGraph) -> G.HostGraph:
    """The graph's arrays as page-locked host tensors (fast uploads)."""
    def pin(a):
        if a is None:
            return None
        t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
        return t.cpu().pin_memory() if torch.cuda.is_available() else t.cpu()

    return G.HostGraph(pin(g.off), pin(g.col), pin(g.k), pin(g.wt), pin(g.s), pin(g.kk), g.wt_kind)


def make_trace(count: int, qps: float, seed: int = 0, mmin: int = 1000, mmax: int = 5_000_000,
               device="cpu", kinds=("sbm", "chung_lu", "knn")) -> List[Request]:
    """Seeded Poisson arrivals at rate qps; request type uniform over kinds,
    edge count log-uniform in [mmin, mmax].  Graphs are generated on
    `device` and kept in host memory (page-locked when a GPU is present)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / qps)) if qps > 0 else 0.0
        kind = kinds[int(rng.integers(0, len(kinds)))]
        m = int(round(math.exp(rng.uniform(math.log(mmin), math.log(mmax)))))
        g, (p, q) = request_graph(kind, m, seed * 1_000_003 + i, device=device)
        out.append(Request(i, t, pinned(g), p, q, kind))
    return out


def retime(trace: List[Request], qps: float, seed: int = 0) -> List[Request]:
    """The same requests with new Poisson arrival times at rate qps."""
    rng = np.random.default_rng([seed, 99])
    t = 0.0
    out = []
    for r in trace:
        t += float(rng.exponential(1.0 / qps)) if qps > 0 else 0.0
        out.append(Request(r.rid, t, r.graph, r.p, r.q, r.kind))
    return out


# ----------------------------------------------------------------- server


@dataclass
class _Resident:
    req: Request
    dev: lcc.DeviceGraph
    est: int
    admitted: float


@dataclass
class ServeStats:
    done: List[Done] = field(default_factory=list)
    makespan: float = 0.0
    batches: int = 0
    peak_hbm_estimate: int = 0

    def latencies(self) -> np.ndarray:
        return np.array([d.latency for d in self.done if d.error is None])

    def summary(self) -> dict:
        lat = self.latencies()
        ok = len(lat)
        return {"requests": len(self.done), "ok": ok, "makespan_s": self.makespan,
                "throughput_rps": ok / self.makespan if self.makespan > 0 else 0.0,
                "p50_ms": float(np.percentile(lat, 50) * 1e3) if ok else None,
                "p99_ms": float(np.percentile(lat, 99) * 1e3) if ok else None,
                "mean_ms": float(lat.mean() * 1e3) if ok else None,
                "batches": self.batches, "peak_hbm_estimate_bytes": self.peak_hbm_estimate}


class Server:
    """Continuous-batching server on one GPU.

    slots: concurrent batches (each a library context + HIP stream);
    torch_pool: the contexts take device memory from torch's caching allocator;
    hbm_budget: bytes of HBM estimates admitted requests may hold together;
    max_jobs / max_arcs: caps of one batch; plain: one request at a time
    through lcc_cluster on one slot (the comparison path)."""

    def __init__(self, device: int = 0, slots: int = 2, hbm_budget: int = 64 << 30, max_jobs: int = 4096,
                 max_arcs: int = 1_500_000_000, params: Optional[lcc.Params] = None, plain: bool = False,
                 torch_pool: bool = True):
        self.device = device
        self.plain = plain
        self.slots = 1 if plain else slots
        self.hbm_budget = hbm_budget
        self.max_jobs = 1 if plain else max_jobs
        self.max_arcs = max_arcs
        self.params = params or lcc.Params()
        # each slot's context takes its scratch from torch's caching allocator
        # (torch_pool): a buffer that grows goes back to the pool instead of
        # through hipFree, which would wait for every slot's work
        self.ctxs = [lcc.Context(device, lcc.TorchAllocator(device) if torch_pool else None)
                     for _ in range(self.slots)]
        self.streams = [torch.cuda.Stream(device=device) for _ in range(self.slots)]
        self.up_stream = torch.cuda.Stream(device=device)

    def close(self):
        for c in self.ctxs:
            c.close()

    def warmup(self, trace: List[Request]):
        """One pass over a few requests per slot so that scratch buffers exist."""
        for s in range(self.slots):
            rs = trace[: min(len(trace), 8)]
            with torch.cuda.stream(self.streams[s]):
                devs = [lcc.DeviceGraph.from_host(r.graph, f"cuda:{self.device}") for r in rs]
                if self.plain:
                    for r, d in zip(rs, devs):
                        self._run(s, [r], [d])
                else:
                    self._run(s, rs, devs)
            self.streams[s].synchronize()

    def _run(self, slot: int, reqs: List[Request], devs: List[lcc.DeviceGraph]):
        ctx, stream = self.ctxs[slot], self.streams[slot]
        if self.plain:
            assert len(reqs) == 1
            lab, N, st = lcc.lcc_cluster(ctx, devs[0], reqs[0].p, reqs[0].q, self.params, stream=stream)
            return [lab.cpu().numpy()], [N], [st["clusters"]]
        hg = [G.HostGraph(d.off, d.col, d.k, d.wt, d.s, d.kk,
                          {None: "none", torch.int16: "i16", torch.int32: "i32", torch.int64: "i64"}[
                              None if d.wt is None else d.wt.dtype]) for d in devs]
        # one weight storage per launch: promote unit-weight jobs to the widest
        # stored type present (weights 1), which leaves every result unchanged
        kinds = {h.wt_kind for h in hg}
        if len(kinds) > 1:
            widest = max((k for k in kinds if k != "none"), key=lambda k: {"i16": 2, "i32": 4, "i64": 8}[k])
            dt = {"i16": torch.int16, "i32": torch.int32, "i64": torch.int64}[widest]
            hg = [h if h.wt_kind == widest else
                  G.HostGraph(h.off, h.col, h.k, (h.wt if h.wt is not None else
                                                  torch.ones(h.arcs, dtype=dt, device=h.col.device)).to(dt),
                              h.s, h.kk, widest) for h in hg]
        P, start = G.pack_torch(hg, f"cuda:{self.device}")
        gp = lcc.DeviceGraph.from_host(P, f"cuda:{self.device}")
        lab, jobs, _ = lcc.lcc_cluster_batch(ctx, gp, start, [(r.p, r.q) for r in reqs], self.params, stream=stream)
        labh = lab.cpu().numpy()
        return ([labh[start[j]:start[j + 1]] for j in range(len(reqs))], [j["N"] for j in jobs],
                [j["clusters"] for j in jobs])

    def serve(self, trace: List[Request], time_scale: float = 1.0) -> ServeStats:
        """Replays the trace (arrival times scaled by time_scale) and returns
        per-request results and timings."""
        cv = threading.Condition()
        pending: deque = deque()
        ready: deque = deque()
        stats = ServeStats()
        state = {"arrived": 0, "admitted_bytes": 0, "finished": 0, "error": None}
        total = len(trace)
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0

        def feeder():
            for r in sorted(trace, key=lambda r: r.arrival):
                dt = r.arrival * time_scale - now()
                if dt > 0:
                    time.sleep(dt)
                with cv:
                    pending.append(r)
                    state["arrived"] += 1
                    cv.notify_all()

        def admitter():
            torch.cuda.set_device(self.device)
            admitted = 0
            while admitted < total:
                with cv:
                    while not pending and state["error"] is None:
                        cv.wait()
                    if state["error"] is not None:
                        return
                    r = pending[0]
                    est = hbm_estimate(r.graph)
                    if est > self.hbm_budget:
                        pending.popleft()
                        stats.done.append(Done(r.rid, np.zeros(0, np.int32), 0, 0, r.arrival, now(), now(), now(), 0,
                                               error="request exceeds the HBM budget"))
                        state["finished"] += 1
                        admitted += 1
                        cv.notify_all()
                        continue
                    while state["admitted_bytes"] + est > self.hbm_budget and state["error"] is None:
                        cv.wait()
                    if state["error"] is not None:
                        return
                    pending.popleft()
                    state["admitted_bytes"] += est
                    stats.peak_hbm_estimate = max(stats.peak_hbm_estimate, state["admitted_bytes"])
                # upload outside the lock; the graph stays resident until done
                with torch.cuda.stream(self.up_stream):
                    d = lcc.DeviceGraph.from_host(r.graph, f"cuda:{self.device}")
                self.up_stream.synchronize()
                with cv:
                    ready.append(_Resident(r, d, est, now()))
                    admitted += 1
                    cv.notify_all()

        def worker(slot):
            torch.cuda.set_device(self.device)
            while True:
                with cv:
                    while not ready and state["finished"] < total and state["error"] is None:
                        cv.wait()
                    if state["finished"] >= total or state["error"] is not None:
                        return
                    # the ready requests that store weights like the oldest one
                    # (one weight storage per launch), in arrival order
                    kind = ready[0].req.graph.wt_kind if ready[0].req.graph.wt is not None else "none"
                    take, rest, arcs = [], deque(), 0
                    while ready:
                        r = ready.popleft()
                        rk = r.req.graph.wt_kind if r.req.graph.wt is not None else "none"
                        if rk == kind and len(take) < self.max_jobs and (
                                not take or arcs + r.req.graph.arcs <= self.max_arcs):
                            take.append(r)
                            arcs += r.req.graph.arcs
                        else:
                            rest.append(r)
                    ready.extend(rest)
                    stats.batches += 1
                t_start = now()
                try:
                    with torch.cuda.stream(self.streams[slot]):
                        labs, Ns, ncl = self._run(slot, [x.req for x in take], [x.dev for x in take])
                    self.streams[slot].synchronize()
                except Exception as e:  # report, stop the loop
                    with cv:
                        state["error"] = repr(e)
                        cv.notify_all()
                    return
                t_end = now()
                with cv:
                    for x, lab, N, c in zip(take, labs, Ns, ncl):
                        stats.done.append(Done(x.req.rid, lab, N, c, x.req.arrival * time_scale, x.admitted, t_start,
                                               t_end, len(take)))
                        state["admitted_bytes"] -= x.est
                        state["finished"] += 1
                    take.clear()
                    cv.notify_all()

        threads = [threading.Thread(target=feeder, daemon=True), threading.Thread(target=admitter, daemon=True)]
        threads += [threading.Thread(target=worker, args=(s,), daemon=True) for s in range(self.slots)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if state["error"] is not None:
            raise RuntimeError(f"serving failed: {state['error']}")
        stats.makespan = max((d.finished for d in stats.done), default=0.0) - min(
            (d.arrival for d in stats.done), default=0.0)
        stats.done.sort(key=lambda d: d.rid)
        return stats
