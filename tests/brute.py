"""Brute-force checkers written straight from the paper's definitions, used to
pin the oracle.  Nothing here calls the oracle's arithmetic.

* ``objective_q``: q times the objective of Sec. 2 summed over unordered pairs,
  from a dense pair loop over the rescaled weights w'_ij.
* ``objective_vxv_q``: the same over ordered pairs of V x V (the paper's
  printed form), which counts every pair twice.
* ``best_single_move``: the best move of one vertex found by evaluating the
  objective after every candidate move (no gain formula).
* ``partitions``: every set partition of range(n) as restricted growth strings.
* ``components``: union-find connected components.
"""
from __future__ import annotations

import numpy as np


def dense(g):
    """Dense symmetric weight matrix and edge mask of a host CSR graph."""
    n = len(g.off) - 1
    W = np.zeros((n, n), dtype=object)
    E = np.zeros((n, n), dtype=bool)
    for v in range(n):
        for e in range(int(g.off[v]), int(g.off[v + 1])):
            u = int(g.col[e])
            w = 1 if g.wt is None else int(g.wt[e])
            W[v, u] += w
            E[v, u] = True
    return W, E


def objective_q(W, E, k, p, q, C):
    """q * sum over unordered pairs i < j in the same cluster of w'_ij with
    w'_ij = w_ij - lambda k_i k_j on edges and -lambda k_i k_j otherwise."""
    n = len(C)
    tot = 0
    for i in range(n):
        for j in range(i + 1, n):
            if C[i] != C[j]:
                continue
            wij = W[i, j] if E[i, j] else 0
            tot += q * wij - p * int(k[i]) * int(k[j])
    return tot


def objective_vxv_q(W, E, k, p, q, C):
    """q * sum over ordered pairs (i, j) in V x V of w'_ij (1 - x_ij), with
    w'_ii = 0."""
    n = len(C)
    tot = 0
    for i in range(n):
        for j in range(n):
            if i == j or C[i] != C[j]:
                continue
            wij = W[i, j] if E[i, j] else 0
            tot += q * wij - p * int(k[i]) * int(k[j])
    return tot


def partitions(n):
    """All set partitions of range(n) as restricted growth strings."""
    if n == 0:
        yield []
        return
    a = [0] * n

    def rec(i, mx):
        if i == n:
            yield list(a)
            return
        for c in range(mx + 2):
            a[i] = c
            yield from rec(i + 1, max(mx, c))

    a[0] = 0
    yield from rec(1, 0)


ISO = -1


def best_single_move(W, E, k, p, q, C, v, allow_iso=True):
    """The decision of vertex v under the method's rules, found by brute force:
    every candidate target (a cluster holding a neighbor of v, or a fresh empty
    cluster when v's cluster has another member) is tried and the objective is
    recomputed from scratch.  Highest increase wins, ties go to the lowest
    cluster id with the fresh cluster last; v moves only if the increase is
    positive.  Returns the target id, ISO, or C[v]."""
    n = len(C)
    c = C[v]
    base = objective_q(W, E, k, p, q, C)
    cands = sorted({C[u] for u in range(n) if E[v, u]} - {c})
    size_c = sum(1 for x in C if x == c)
    best, best_id = None, None
    for X in cands:
        C2 = list(C)
        C2[v] = X
        gain = objective_q(W, E, k, p, q, C2) - base
        if best is None or gain > best:
            best, best_id = gain, X
    if allow_iso and size_c >= 2:
        fresh = max(C) + 1
        C2 = list(C)
        C2[v] = fresh
        gain = objective_q(W, E, k, p, q, C2) - base
        if best is None or gain > best:
            best, best_id = gain, ISO
    if best is not None and best > 0:
        return best_id
    return c


def components(n, edges):
    """Connected components (union-find) of the graph on range(n) with the
    given undirected edges; returns a representative per vertex."""
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for a, b in edges:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    return [find(x) for x in range(n)]
