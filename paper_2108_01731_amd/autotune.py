"""Autotuner over the tuning fields of lcc_params.

The tuning fields (queue_ahead, small_level, low_merge, hub_row_limit,
score_pruning) choose launch shapes
and schedules, never results: every choice must return the same labels and
objective.  The tuner times a workload under candidate settings, one field at
a time (coordinate descent from the defaults), keeps the fastest, and checks
that every setting it tried returned the identical result; a difference
raises, so a tuned setting can be used without re-checking.

`run(params)` is any callable that runs the workload once and returns a
hashable result key (for instance the bytes of the labels and the objective
numerators); the tuner times it with a device synchronization on both sides.
"""
from __future__ import annotations

import dataclasses
import hashlib
import time
from typing import Callable, Dict, List, Optional, Tuple

import torch

from . import lcc

# Candidate values per field (0 = the library's automatic choice).
SPACE: Dict[str, List[int]] = {
    "queue_ahead": [0, 1, 2, 4, 10],
    "small_level": [0, 1024, 4096],
    "low_merge": [0, 4096, 262144],
    "hub_row_limit": [0, -1],
    "score_pruning": [0, 1, -1],
}


class TuningChangedResult(RuntimeError):
    pass


def result_key(*tensors_or_ints) -> str:
    """A digest of labels (tensors) and numerators (ints)."""
    h = hashlib.sha1()
    for x in tensors_or_ints:
        if isinstance(x, torch.Tensor):
            h.update(x.detach().cpu().numpy().tobytes())
        else:
            h.update(repr(x).encode())
    return h.hexdigest()


def _time(run, prm, reps):
    key = None
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = run(prm)
        torch.cuda.synchronize()
        best = min(best, (time.perf_counter() - t0) * 1e3)
        if key is None:
            key = k
        elif k != key:
            raise TuningChangedResult(f"repeated runs with {prm} returned different results")
    return key, best


def tune(run: Callable[[lcc.Params], str], base: Optional[lcc.Params] = None, space=None, reps: int = 2,
         budget_s: float = 120.0) -> Tuple[lcc.Params, List[dict]]:
    """Coordinate descent over `space` from `base`.  Returns (fastest
    params, table of every setting tried with its time).  Raises
    TuningChangedResult if any setting changes the result."""
    base = base or lcc.Params()
    space = space or SPACE
    t_start = time.perf_counter()
    ref_key, ref_ms = _time(run, base, reps)
    best, best_ms = base, ref_ms
    table = [{"params": {f: getattr(base, f) for f in space}, "ms": ref_ms}]
    for field, values in space.items():
        for v in values:
            if v == getattr(best, field):
                continue
            if time.perf_counter() - t_start > budget_s:
                return best, table
            cand = dataclasses.replace(best, **{field: v})
            key, ms = _time(run, cand, reps)
            table.append({"params": {f: getattr(cand, f) for f in space}, "ms": ms})
            if key != ref_key:
                raise TuningChangedResult(f"{field}={v} changed the result")
            if ms < best_ms:
                best, best_ms = cand, ms
    return best, table


def cluster_runner(ctx, g, p, q):
    def run(prm):
        lab, N, _ = lcc.lcc_cluster(ctx, g, p, q, prm)
        return result_key(lab, N)
    return run


def batch_runner(ctx, g, start, lambdas):
    def run(prm):
        lab, jobs, _ = lcc.lcc_cluster_batch(ctx, g, start, lambdas, prm)
        return result_key(lab, [j["N"] for j in jobs])
    return run


def sweep_runner(ctx, g, lambdas):
    def run(prm):
        lab, jobs, _ = lcc.lcc_sweep(ctx, g, lambdas, prm)
        return result_key(lab, [j["N"] for j in jobs])
    return run
