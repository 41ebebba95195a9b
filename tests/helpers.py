"""Shared test helpers: moving graphs between the generators, the oracle and
the GPU binding, and a few extra graph shapes for edge cases."""
import numpy as np
import torch

import oracle as O
from paper_2108_01731_amd import graphgen as G


def to_oracle(h) -> O.Graph:
    h = h.numpy()
    return O.Graph(off=h.off, col=h.col, k=h.k, wt=None if h.wt is None else np.asarray(h.wt).astype(np.int64),
                   s=h.s, kk=h.kk)


def with_weights(h, kind: str, seed: int = 0, lo: int = -5, hi: int = 9):
    """Same graph with symmetric random integer weights of the given storage."""
    h = h.numpy()
    rng = np.random.default_rng(seed)
    n = len(h.off) - 1
    src = np.repeat(np.arange(n), np.diff(h.off))
    a = np.minimum(src, h.col)
    b = np.maximum(src, h.col)
    key = a.astype(np.int64) * n + b
    uk, inv = np.unique(key, return_inverse=True)
    w = rng.integers(lo, hi + 1, size=len(uk))[inv]
    dt = {"i16": np.int16, "i32": np.int32, "i64": np.int64}[kind]
    return G.HostGraph(h.off, h.col, h.k, wt=w.astype(dt), wt_kind=kind)


def with_k(h, k):
    h = h.numpy()
    return G.HostGraph(h.off, h.col, np.asarray(k, np.int64), wt=h.wt, s=h.s, kk=h.kk, wt_kind=h.wt_kind)


def hub_graph(n=6000, m=20000, hubs=(2500, 3100, 4700, 300, 1200), seed=5, weighted=True):
    """A sparse random graph plus a few hub vertices of chosen degrees, so
    every degree bin of the aggregation kernels is exercised."""
    rng = np.random.default_rng(seed)
    u = list(rng.integers(0, n, m))
    v = list(rng.integers(0, n, m))
    for i, d in enumerate(hubs):
        nb = rng.choice(n, size=d, replace=False)
        u += [i] * d
        v += list(nb)
    u = torch.tensor(u)
    v = torch.tensor(v)
    w = torch.from_numpy(rng.integers(-2, 6, size=len(u))) if weighted else None
    off, col, wt = G.csr_from_edges(n, u, v, w)
    k = rng.integers(0, 4, size=n).astype(np.int64)
    if weighted:
        return G.HostGraph(off.numpy(), col.numpy(), k, wt=wt.numpy().astype(np.int32), wt_kind="i32")
    return G.HostGraph(off.numpy(), col.numpy(), np.ones(n, np.int64))


def shuffle_rows(h, seed=0):
    h = h.numpy()
    rng = np.random.default_rng(seed)
    col = h.col.copy()
    wt = None if h.wt is None else h.wt.copy()
    for v in range(len(h.off) - 1):
        a, b = h.off[v], h.off[v + 1]
        p = rng.permutation(b - a) + a
        col[a:b] = col[p]
        if wt is not None:
            wt[a:b] = wt[p]
    return G.HostGraph(h.off, col, h.k, wt=wt, s=h.s, kk=h.kk, wt_kind=h.wt_kind)


def split_arcs(h, every: int = 3):
    """The same graph with every `every`-th edge stored as two parallel arcs
    in both rows (weights w1 and w - w1, w1 fixed by the vertex pair), so rows
    repeat a neighbor and are no longer strictly ascending."""
    h = h.numpy()
    n = len(h.off) - 1
    wt = np.ones(len(h.col), np.int64) if h.wt is None else np.asarray(h.wt).astype(np.int64)
    off, col, w = [0], [], []
    for v in range(n):
        for e in range(h.off[v], h.off[v + 1]):
            u = int(h.col[e])
            key = min(u, v) * n + max(u, v)
            if key % every == 0:
                w1 = key % 5 - 2
                col += [u, u]
                w += [w1, int(wt[e]) - w1]
            else:
                col.append(u)
                w.append(int(wt[e]))
        off.append(len(col))
    return G.HostGraph(np.array(off, np.int64), np.array(col, np.int32), h.k, wt=np.array(w, np.int64),
                       s=h.s, kk=h.kk, wt_kind="i64")
