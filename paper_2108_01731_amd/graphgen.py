"""Seeded synthetic graph generators for the LambdaCC workloads.

This module holds no clustering arithmetic: it only produces inputs (a CSR
graph, vertex weights k, optional integer edge weights) that both the GPU path
and the CPU oracle consume.  Every generator is deterministic for a given seed
on a given torch device (torch's own per-device generators are used, so a CPU
graph and a GPU graph with the same seed differ; callers that compare two
implementations build the graph once and hand the same arrays to both).

Graph shapes stand in for the paper's inputs (its Table 1 SNAP graphs and the
k-NN graphs of its weighted experiments), which are not available here:
  * ``sbm``: stochastic block model, exact Bernoulli trials per vertex pair
    (geometric skipping inside each block pair's pair grid);
  * ``chung_lu_planted``: Chung-Lu expected-degree graph with a power-law degree
    sequence and planted communities with power-law sizes; a mixing fraction
    of the edges is drawn globally, the rest inside the first endpoint's
    community;
  * ``knn_gaussian``: cosine k-NN graph of a Gaussian mixture, symmetrized by
    union, weights round(cos * 2^15) clamped to int16 (Q1.15);
  * ``random_signed``: tiny random graphs with signed weights and random vertex
    weights, for exhaustive checks.
All generators apply a seeded random relabel of the vertex ids at the end, so
ids do not align with blocks or communities.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch


@dataclass
class HostGraph:
    """CSR arrays (numpy or torch, host or device).

    off: int64[n+1]; col: int32[arcs]; wt: None (unit) or int16/int32/int64[arcs];
    k: int64[n]; s / kk: None or int64[n].  Symmetric, no self-loops."""

    off: object
    col: object
    k: object
    wt: object = None
    s: object = None
    kk: object = None
    wt_kind: str = "none"  # none | i16 | i32 | i64

    @property
    def n(self) -> int:
        return int(self.off.shape[0]) - 1

    @property
    def arcs(self) -> int:
        return int(self.col.shape[0])

    def to(self, device) -> "HostGraph":
        def mv(a):
            if a is None:
                return None
            if isinstance(a, np.ndarray):
                a = torch.from_numpy(a)
            return a.to(device)

        return HostGraph(mv(self.off), mv(self.col), mv(self.k), mv(self.wt), mv(self.s),
                         mv(self.kk), self.wt_kind)

    def numpy(self) -> "HostGraph":
        def cv(a):
            if a is None:
                return None
            if isinstance(a, torch.Tensor):
                return a.cpu().numpy()
            return a

        return HostGraph(cv(self.off), cv(self.col), cv(self.k), cv(self.wt), cv(self.s),
                         cv(self.kk), self.wt_kind)


def _hash64(x: torch.Tensor, salt: int) -> torch.Tensor:
    """A seeded 64-bit mixing of int64 values (SplitMix64's finalizer with
    logical shifts), used as random sort keys: unlike torch.randperm it gives
    the same order on every run and every device at any size."""
    def srl(t, k):
        return (t >> k) & ((1 << (64 - k)) - 1)

    def s64(c):
        return c - (1 << 64) if c >= (1 << 63) else c

    z = x + s64((0x9E3779B97F4A7C15 * (salt + 1)) % (1 << 64))
    z = (z ^ srl(z, 30)) * s64(0xBF58476D1CE4E5B9)
    z = (z ^ srl(z, 27)) * s64(0x94D049BB133111EB)
    return z ^ srl(z, 31)


def _hash_perm(n: int, salt: int, device) -> torch.Tensor:
    """A seeded permutation of [0, n): indices sorted by their hash (stable)."""
    return torch.sort(_hash64(torch.arange(n, device=device, dtype=torch.int64), salt), stable=True).indices


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) & (2**63 - 1))
    return g


def csr_from_edges(n: int, u: torch.Tensor, v: torch.Tensor, w: Optional[torch.Tensor] = None,
                   device=None) -> tuple:
    """Undirected edge list -> symmetric CSR without self-loops or duplicate
    edges.  Duplicate undirected edges keep the weight of their first
    occurrence in (min, max, weight) order.  Returns (off, col, wt)."""
    device = device or u.device
    u = u.to(device=device, dtype=torch.int64)
    v = v.to(device=device, dtype=torch.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    if w is not None:
        w = w.to(device)[keep]
    a = torch.minimum(u, v)
    b = torch.maximum(u, v)
    key = a * n + b
    if w is None:
        key = torch.unique(key)
        ww = None
    else:
        key, order = torch.sort(key, stable=True)
        w = w[order]
        first = torch.ones_like(key, dtype=torch.bool)
        first[1:] = key[1:] != key[:-1]
        key, ww = key[first], w[first]
    a = key // n
    b = key % n
    src = torch.cat([a, b])
    dst = torch.cat([b, a])
    akey = src * n + dst
    akey, order = torch.sort(akey)
    col = (akey % n).to(torch.int32)
    srcs = akey // n
    cnt = torch.bincount(srcs, minlength=n)
    off = torch.zeros(n + 1, dtype=torch.int64, device=device)
    off[1:] = torch.cumsum(cnt, 0)
    wt = None
    if ww is not None:
        wt = torch.cat([ww, ww])[order]
    return off, col, wt


def csr_relabeled(n: int, a: torch.Tensor, b: torch.Tensor, perm: torch.Tensor, max_arcs: int = 1 << 30):
    """Symmetric CSR of the distinct undirected edges (a, b), a != b, after
    the vertex relabel old -> perm[old], rows ascending; the same result as
    relabel(csr_from_edges(...)).  Rows are built range by range (at most
    max_arcs arcs sorted at a time), so graphs beyond 2^31 arcs fit."""
    device = a.device
    a = perm[a]
    b = perm[b]
    deg = torch.zeros(n, dtype=torch.int64, device=device)
    step = 1 << 28
    for s0 in range(0, a.numel(), step):
        deg += torch.bincount(a[s0:s0 + step], minlength=n)
        deg += torch.bincount(b[s0:s0 + step], minlength=n)
    off = torch.zeros(n + 1, dtype=torch.int64, device=device)
    off[1:] = torch.cumsum(deg, 0)
    arcs = int(off[-1])
    col = torch.empty(arcs, dtype=torch.int32, device=device)
    r0 = 0
    while r0 < n:
        # rows [r0, r1) hold at most max_arcs arcs (a single wider row alone)
        r1 = int(torch.searchsorted(off, off[r0] + max_arcs, right=True)) - 1
        r1 = min(max(r1, r0 + 1), n)
        parts = []
        for s0 in range(0, a.numel(), step):
            x, y = a[s0:s0 + step], b[s0:s0 + step]
            m1 = (x >= r0) & (x < r1)
            m2 = (y >= r0) & (y < r1)
            parts.append((x[m1] - r0) * n + y[m1])
            parts.append((y[m2] - r0) * n + x[m2])
        key = torch.sort(torch.cat(parts)).values
        del parts
        col[int(off[r0]):int(off[r1])] = (key % n).to(torch.int32)
        del key
        r0 = r1
    return off, col


def relabel(off: torch.Tensor, col: torch.Tensor, wt, perm: torch.Tensor):
    """Apply the vertex relabel old -> perm[old]; rows keep ascending columns."""
    n = off.shape[0] - 1
    device = off.device
    deg = off[1:] - off[:-1]
    src = torch.repeat_interleave(torch.arange(n, device=device), deg)
    ns = perm[src]
    nd = perm[col.to(torch.int64)]
    key = ns * n + nd
    key, order = torch.sort(key)
    ncol = (key % n).to(torch.int32)
    cnt = torch.bincount(key // n, minlength=n)
    noff = torch.zeros(n + 1, dtype=torch.int64, device=device)
    noff[1:] = torch.cumsum(cnt, 0)
    nwt = None if wt is None else wt[order]
    return noff, ncol, nwt


# --------------------------------------------------------------------- SBM


def sbm(block_sizes, p_in: float, p_out: float, seed: int, device="cpu") -> HostGraph:
    """Stochastic block model: every vertex pair is an independent Bernoulli
    trial, p_in inside a block and p_out across blocks.  Unit weights, k = 1."""
    device = torch.device(device)
    gen = _gen(seed, device)
    sizes = [int(s) for s in block_sizes]
    n = sum(sizes)
    base = np.concatenate([[0], np.cumsum(sizes)])
    us, vs = [], []
    for a in range(len(sizes)):
        for b in range(a, len(sizes)):
            p = p_in if a == b else p_out
            if p <= 0:
                continue
            rows, cols = sizes[a], sizes[b]
            N = rows * cols  # pair grid; for a == b only cells above the diagonal count
            idx = _bernoulli_positions(N, p, gen, device)
            i = idx // cols
            j = idx % cols
            if a == b:
                keep = i < j
                i, j = i[keep], j[keep]
            us.append(i + int(base[a]))
            vs.append(j + int(base[b]))
    u = torch.cat(us) if us else torch.zeros(0, dtype=torch.int64, device=device)
    v = torch.cat(vs) if vs else torch.zeros(0, dtype=torch.int64, device=device)
    off, col, _ = csr_from_edges(n, u, v, device=device)
    perm = torch.randperm(n, generator=gen, device=device)
    off, col, _ = relabel(off, col, None, perm)
    k = torch.ones(n, dtype=torch.int64, device=device)
    return HostGraph(off, col, k)


def _bernoulli_positions(N: int, p: float, gen, device) -> torch.Tensor:
    """Sorted positions in [0, N) of successes of N Bernoulli(p) trials, by
    geometric skipping."""
    if p >= 1.0:
        return torch.arange(N, device=device)
    out = []
    pos = -1
    lq = math.log1p(-p)
    chunk = max(1024, int(N * p * 1.2) + 64)
    while True:
        u = torch.rand(chunk, generator=gen, device=device, dtype=torch.float64)
        u = torch.clamp(u, min=1e-300)
        gaps = torch.floor(torch.log(u) / lq).to(torch.int64) + 1
        posv = pos + torch.cumsum(gaps, 0)
        keep = posv < N
        out.append(posv[keep])
        if not bool(keep.all()):
            break
        pos = int(posv[-1])
    return torch.cat(out)


# ------------------------------------------------- Chung-Lu, planted communities


def _powerlaw_weights(n: int, mean: float, gamma: float, dmax: float) -> np.ndarray:
    """Expected degrees at the quantiles (i + 0.5) / n of a Pareto law with
    exponent gamma, capped at dmax; the minimum is tuned so the mean matches."""
    u = (np.arange(n, dtype=np.float64) + 0.5) / n
    shape = (1.0 - u) ** (-1.0 / (gamma - 1.0))

    def mean_for(dmin):
        return float(np.minimum(dmin * shape, dmax).mean())

    lo, hi = 1e-3, mean
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mean_for(mid) < mean:
            lo = mid
        else:
            hi = mid
    return np.minimum(hi * shape, dmax)


def _community_sizes(n: int, smin: int, smax: int, tau: float, rng: np.random.Generator):
    """Power-law community sizes in [smin, smax] (exponent tau) covering n."""
    sizes = []
    total = 0
    xs = np.arange(smin, smax + 1, dtype=np.float64)
    pw = xs ** (-tau)
    pw /= pw.sum()
    while total < n:
        batch = rng.choice(xs.astype(np.int64), size=4096, p=pw)
        for s in batch:
            s = int(s)
            if total + s > n:
                s = n - total
            sizes.append(s)
            total += s
            if total >= n:
                break
    if len(sizes) > 1 and sizes[-1] < smin:
        last = sizes.pop()
        sizes[-1] += last
    return sizes


def chung_lu_planted(n: int, m: int, gamma: float, mixing: float, seed: int, device="cpu",
                     comm_min: int = 20, comm_max: int = 5000, comm_tau: float = 2.0,
                     k_is_degree: bool = True, max_rounds: int = 8, return_communities: bool = False):
    """Chung-Lu graph with planted communities.

    Expected degrees follow a power law with exponent ``gamma`` (max capped at
    sqrt(2m)).  Community sizes follow a power law on [comm_min, comm_max]
    (exponent ``comm_tau``); vertices are matched to community slots by rank
    of log expected degree against log community size, both jittered by unit
    Gaussian noise, so high-degree vertices tend to sit in large communities
    (as in LFR-style benchmarks) without the assignment being sorted.  Edges
    are drawn in rounds until ``m`` distinct edges exist: a ``mixing`` fraction
    of each round has both endpoints chosen proportionally to expected degree
    over all vertices, the rest has the second endpoint chosen proportionally
    to expected degree inside the first endpoint's community.  Self-loops and
    repeats are dropped; the final edge set is a uniform subset of size m (or
    everything drawn, if ``max_rounds`` runs out first).  k = degree (the
    modularity setting) unless ``k_is_degree`` is False (then k = 1).  With
    ``return_communities`` returns (graph, comm) where comm (int64 numpy, in
    the relabelled vertex ids) is each vertex's planted community."""
    device = torch.device(device)
    gen = _gen(seed, device)
    rng = np.random.default_rng(seed)
    w = _powerlaw_weights(n, 2.0 * m / n, gamma, math.sqrt(2.0 * m))
    sizes = _community_sizes(n, comm_min, comm_max, comm_tau, rng)
    # slot j belongs to community comm_of_slot[j]; slots of one community are consecutive
    comm_start = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    comm_of_slot_np = np.repeat(np.arange(len(sizes)), sizes)
    slot_key = np.log(np.asarray(sizes, dtype=np.float64))[comm_of_slot_np] + rng.standard_normal(n)
    vert_key = np.log(w) + rng.standard_normal(n)
    # the vertex with the r-th largest key takes the slot with the r-th largest key
    slot_vertex_np = np.empty(n, dtype=np.int64)
    slot_vertex_np[np.argsort(-slot_key, kind="stable")] = np.argsort(-vert_key, kind="stable")
    slot_vertex = torch.from_numpy(slot_vertex_np).to(device)
    # cumulative weights on the host: a sequential sum rounds the same way on
    # every run (a parallel device scan of floats need not)
    cum_np = np.zeros(n + 1, dtype=np.float64)
    np.cumsum(w[slot_vertex_np], out=cum_np[1:])
    cum = torch.from_numpy(cum_np).to(device)
    total = float(cum_np[-1])
    comm_of_slot = torch.from_numpy(comm_of_slot_np).to(device)
    cs_t = torch.from_numpy(comm_start).to(device)
    keys = torch.zeros(0, dtype=torch.int64, device=device)
    chunk = 1 << 25
    for _ in range(max_rounds):
        need = m - int(keys.numel())
        if need <= 0:
            break
        draw = int(need * 1.1) + 16
        n_glob = int(round(mixing * draw))
        parts = [keys]
        done = 0
        while done < draw:
            cnt = min(chunk, draw - done)
            r1 = torch.rand(cnt, generator=gen, device=device, dtype=torch.float64) * total
            a = torch.clamp(torch.searchsorted(cum, r1, right=True) - 1, 0, n - 1)
            r2 = torch.rand(cnt, generator=gen, device=device, dtype=torch.float64)
            is_glob = torch.arange(done, done + cnt, device=device) < n_glob
            ca = comm_of_slot[a]
            lo = torch.where(is_glob, torch.zeros_like(a), cs_t[ca])
            hi = torch.where(is_glob, torch.full_like(a, n), cs_t[ca + 1])
            r = cum[lo] + r2 * (cum[hi] - cum[lo])
            b = torch.searchsorted(cum, r, right=True) - 1
            b = torch.minimum(torch.maximum(b, lo), hi - 1)
            u = slot_vertex[a]
            v = slot_vertex[b]
            keep = u != v
            u, v = u[keep], v[keep]
            parts.append(torch.minimum(u, v) * n + torch.maximum(u, v))
            done += cnt
        keys = torch.unique(torch.cat(parts))
        del parts
    if keys.numel() > m:
        # a seeded uniform subset of size m: the m keys of smallest hash
        # (stable sort: the same subset on every run at any size)
        pick = torch.sort(_hash64(keys, 2 * seed + 1), stable=True).indices[:m]
        keys = torch.sort(keys[pick]).values
        del pick
    u, v = keys // n, keys % n
    del keys
    perm = _hash_perm(n, 2 * seed + 2, device)
    off, col = csr_relabeled(n, u, v, perm)
    del u, v
    deg = off[1:] - off[:-1]
    k = deg.clone() if k_is_degree else torch.ones(n, dtype=torch.int64, device=device)
    if return_communities:
        comm = np.empty(n, dtype=np.int64)
        comm[perm.cpu().numpy()[slot_vertex_np]] = comm_of_slot_np
        return HostGraph(off, col, k), comm
    return HostGraph(off, col, k)


# ------------------------------------------------------------------- rMAT

def rmat(scale: int, m: int, seed: int, a: float = 0.5, b: float = 0.1, c: float = 0.1, device="cpu",
         k_is_degree: bool = False, chunk: int = 1 << 24) -> HostGraph:
    """rMAT graph (Chakrabarti, Zhan, Faloutsos 2004) on n = 2^scale vertices:
    m edge draws, each descending `scale` levels of the adjacency matrix and
    taking the quadrant (top-left, top-right, bottom-left, bottom-right) with
    probabilities (a, b, c, 1 - a - b - c); the paper's scalability graphs
    use a = 0.5, b = c = 0.1.  Self-loops and repeated edges are dropped (so
    fewer than m edges remain), then vertices get a seeded random relabel.
    k = 1 (the correlation-clustering setting) unless k_is_degree."""
    device = torch.device(device)
    gen = _gen(seed, device)
    n = 1 << scale
    parts = []
    done = 0
    while done < m:
        cnt = min(chunk, m - done)
        u = torch.zeros(cnt, dtype=torch.int64, device=device)
        v = torch.zeros(cnt, dtype=torch.int64, device=device)
        for _ in range(scale):
            r = torch.rand(cnt, generator=gen, device=device, dtype=torch.float64)
            down = (r >= a + b).to(torch.int64)  # bottom half: quadrants c and d
            right = ((r >= a) & (r < a + b) | (r >= a + b + c)).to(torch.int64)  # quadrants b and d
            u = (u << 1) | down
            v = (v << 1) | right
        keep = u != v
        u, v = u[keep], v[keep]
        parts.append(torch.unique(torch.minimum(u, v) * n + torch.maximum(u, v)))
        done += cnt
    keys = torch.unique(torch.cat(parts))
    del parts
    u, v = keys // n, keys % n
    del keys
    perm = _hash_perm(n, 2 * seed + 2, device)
    off, col = csr_relabeled(n, u, v, perm)
    deg = off[1:] - off[:-1]
    k = deg.clone() if k_is_degree else torch.ones(n, dtype=torch.int64, device=device)
    return HostGraph(off, col, k)


# ----------------------------------------------------------- weighted k-NN


def knn_gaussian(npoints: int, centers: int, dim: int, knn: int, sigma: float, seed: int,
                 device="cpu", chunk: int = 4096) -> HostGraph:
    """Cosine k-NN graph of a Gaussian mixture (centers ~ N(0, I), points =
    center + sigma * N(0, I)), symmetrized by union; weight = round(cos * 2^15)
    clamped to [-32768, 32767] (Q1.15, stored as int16); k = 1."""
    device = torch.device(device)
    gen = _gen(seed, device)
    C = torch.randn(centers, dim, generator=gen, device=device, dtype=torch.float32)
    lab = torch.randint(0, centers, (npoints,), generator=gen, device=device)
    X = C[lab] + sigma * torch.randn(npoints, dim, generator=gen, device=device,
                                     dtype=torch.float32)
    X = X / X.norm(dim=1, keepdim=True).clamp_min(1e-12)
    us, vs, ws = [], [], []
    for s in range(0, npoints, chunk):
        e = min(npoints, s + chunk)
        sim = X[s:e] @ X.T
        rows = torch.arange(s, e, device=device)
        sim[torch.arange(e - s, device=device), rows] = -3.0  # exclude self
        val, idx = torch.topk(sim, knn, dim=1)
        us.append(rows.repeat_interleave(knn))
        vs.append(idx.reshape(-1))
        ws.append(val.reshape(-1))
    u = torch.cat(us)
    v = torch.cat(vs)
    cosv = torch.cat(ws).to(torch.float64)
    q = torch.clamp(torch.round(cosv * 32768.0), -32768, 32767).to(torch.int64)
    # cosine is symmetric up to rounding of the float dot product: take the
    # weight of the (min, max) orientation's first occurrence for both arcs
    off, col, wt = csr_from_edges(npoints, u, v, q, device=device)
    perm = torch.randperm(npoints, generator=gen, device=device)
    off, col, wt = relabel(off, col, wt, perm)
    k = torch.ones(npoints, dtype=torch.int64, device=device)
    return HostGraph(off, col, k, wt=wt.to(torch.int16), wt_kind="i16")


# ------------------------------------------------------------- small graphs


def random_signed(n: int, m: int, seed: int, wmin: int = -3, wmax: int = 5, kmax: int = 3,
                  unit: bool = False) -> HostGraph:
    """Small random graph (numpy, host): m edge draws over n vertices (repeats
    and self-loops dropped), integer weights uniform in [wmin, wmax] (0
    allowed), k uniform in [0, kmax].  ``unit`` gives unit weights, k = 1."""
    rng = np.random.default_rng(seed)
    u = rng.integers(0, max(n, 1), size=m)
    v = rng.integers(0, max(n, 1), size=m)
    w = rng.integers(wmin, wmax + 1, size=m)
    if n == 0:
        return HostGraph(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int64),
                         None if unit else np.zeros(0, np.int64), wt_kind="none" if unit else "i64")
    off, col, wt = csr_from_edges(n, torch.from_numpy(u), torch.from_numpy(v),
                                  None if unit else torch.from_numpy(w), device="cpu")
    if unit:
        k = np.ones(n, dtype=np.int64)
        return HostGraph(off.numpy(), col.numpy(), k)
    k = rng.integers(0, kmax + 1, size=n).astype(np.int64)
    return HostGraph(off.numpy(), col.numpy(), k, wt=wt.numpy().astype(np.int64), wt_kind="i64")


def c1_sbm(seed: int = 1, device="cpu") -> HostGraph:
    """The small plain-method workload: 10,000 vertices in 20 blocks of 500,
    p_in = 0.02, p_out = 0.0005, k = 1 (run with lambda = 1/100)."""
    return sbm([500] * 20, 0.02, 0.0005, seed, device)


# ------------------------------------------------------------- batched jobs


def sbm_blocks(n: int, block: int, avg_deg: float, mixing: float, seed: int, device="cpu") -> HostGraph:
    """SBM on n vertices in max(1, round(n / block)) near-equal blocks with
    expected degree avg_deg, a fraction `mixing` of it across blocks.  Every
    pair is an independent Bernoulli trial (p_in inside a block, p_out
    across): all pairs are drawn at p_out and the pairs inside blocks again at
    (p_in - p_out) / (1 - p_out); the union has the SBM law.  Unit weights,
    k = 1, seeded vertex relabel."""
    device = torch.device(device)
    gen = _gen(seed, device)
    nb = max(1, int(round(n / block)))
    base_size, extra = divmod(n, nb)
    sizes = torch.full((nb,), base_size, dtype=torch.int64, device=device)
    sizes[:extra] += 1
    starts = torch.zeros(nb, dtype=torch.int64, device=device)
    starts[1:] = torch.cumsum(sizes, 0)[:-1]
    smax = base_size + (1 if extra else 0)
    mean_s = n / nb
    p_in = min(1.0, avg_deg * (1.0 - mixing) / max(mean_s - 1.0, 1.0)) if mean_s > 1 else 0.0
    p_out = min(1.0, avg_deg * mixing / max(n - mean_s, 1.0)) if nb > 1 else 0.0
    us, vs = [], []
    if p_out > 0:
        idx = _bernoulli_positions(n * n, p_out, gen, device)
        i, j = idx // n, idx % n
        keep = i < j
        us.append(i[keep])
        vs.append(j[keep])
    p2 = (p_in - p_out) / (1.0 - p_out) if p_out < 1.0 else 0.0
    if p2 > 0 and smax > 1:
        idx = _bernoulli_positions(nb * smax * smax, p2, gen, device)
        blk = idx // (smax * smax)
        r = idx % (smax * smax)
        i, j = r // smax, r % smax
        sz = sizes[blk]
        keep = (i < j) & (j < sz)
        us.append(i[keep] + starts[blk[keep]])
        vs.append(j[keep] + starts[blk[keep]])
    u = torch.cat(us) if us else torch.zeros(0, dtype=torch.int64, device=device)
    v = torch.cat(vs) if vs else torch.zeros(0, dtype=torch.int64, device=device)
    off, col, _ = csr_from_edges(n, u, v, device=device)
    perm = torch.randperm(n, generator=gen, device=device)
    off, col, _ = relabel(off, col, None, perm)
    return HostGraph(off, col, torch.ones(n, dtype=torch.int64, device=device))


def sbm_job_spec(i: int, seed: int = 0, nmin: int = 100, nmax: int = 50000):
    """Shape of job i of the many-graph batch: n log-uniform in [nmin, nmax],
    average degree uniform in [8, 40], lambda = p / 1000 with p uniform in
    [1, 500].  Returns (n, avg_deg, p, q)."""
    rng = np.random.default_rng([seed, i])
    n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    d = float(rng.uniform(8.0, 40.0))
    p = int(rng.integers(1, 501))
    return n, d, p, 1000


def pack(graphs) -> tuple:
    """Packs graphs block-diagonally into one HostGraph (numpy arrays).
    Returns (graph, job_start int64[len(graphs) + 1]).  Weight storage must
    agree (all unit or all the same integer type); missing s is 0 and missing
    kk is k^2."""
    gs = [g.numpy() for g in graphs]
    ns = np.array([g.n for g in gs], dtype=np.int64)
    ms = np.array([g.arcs for g in gs], dtype=np.int64)
    vstart = np.zeros(len(gs) + 1, dtype=np.int64)
    vstart[1:] = np.cumsum(ns)
    astart = np.zeros(len(gs) + 1, dtype=np.int64)
    astart[1:] = np.cumsum(ms)
    kinds = {g.wt_kind if g.wt is not None else "none" for g in gs}
    if len(kinds) > 1:
        raise ValueError(f"mixed weight storage in one batch: {sorted(kinds)}")
    kind = kinds.pop() if kinds else "none"
    off = np.concatenate([np.asarray(g.off[:-1], dtype=np.int64) + astart[j] for j, g in enumerate(gs)] +
                         [np.array([astart[-1]], dtype=np.int64)])
    col = np.concatenate([np.asarray(g.col, dtype=np.int64) + vstart[j] for j, g in enumerate(gs)] +
                         [np.zeros(0, dtype=np.int64)]).astype(np.int32)
    k = np.concatenate([np.asarray(g.k, dtype=np.int64) for g in gs] + [np.zeros(0, dtype=np.int64)])
    wt = None
    if kind != "none":
        wt = np.concatenate([np.asarray(g.wt) for g in gs])
    s = None
    if any(g.s is not None for g in gs):
        s = np.concatenate([np.asarray(g.s, dtype=np.int64) if g.s is not None else np.zeros(g.n, dtype=np.int64)
                            for g in gs])
    kk = None
    if any(g.kk is not None for g in gs):
        kk = np.concatenate([np.asarray(g.kk, dtype=np.int64) if g.kk is not None
                             else np.asarray(g.k, dtype=np.int64) ** 2 for g in gs])
    return HostGraph(off, col, k, wt, s, kk, kind), vstart


def job_slice(g: HostGraph, job_start, j: int) -> HostGraph:
    """Job j of a packed graph as a graph of its own (numpy arrays)."""
    h = g.numpy()
    a, b = int(job_start[j]), int(job_start[j + 1])
    off = np.asarray(h.off[a:b + 1], dtype=np.int64)
    e0, e1 = int(off[0]), int(off[-1])
    col = (np.asarray(h.col[e0:e1], dtype=np.int64) - a).astype(np.int32)
    return HostGraph(off - e0, col, np.asarray(h.k[a:b]), None if h.wt is None else np.asarray(h.wt[e0:e1]),
                     None if h.s is None else np.asarray(h.s[a:b]), None if h.kk is None else np.asarray(h.kk[a:b]),
                     h.wt_kind)


def pack_torch(graphs, device) -> tuple:
    """pack() for graphs held as torch tensors (e.g. on the GPU): the packed
    arrays are built on `device`.  Returns (graph, job_start int64 numpy)."""
    ns = [g.n for g in graphs]
    ms = [g.arcs for g in graphs]
    vstart = np.zeros(len(graphs) + 1, dtype=np.int64)
    vstart[1:] = np.cumsum(ns)
    astart = np.zeros(len(graphs) + 1, dtype=np.int64)
    astart[1:] = np.cumsum(ms)
    kinds = {g.wt_kind if g.wt is not None else "none" for g in graphs}
    if len(kinds) > 1:
        raise ValueError(f"mixed weight storage in one batch: {sorted(kinds)}")
    kind = kinds.pop() if kinds else "none"
    t = lambda a, dt: torch.as_tensor(a).to(device=device, dtype=dt)
    off = torch.cat([t(g.off[:-1], torch.int64) + int(astart[j]) for j, g in enumerate(graphs)] +
                    [torch.tensor([int(astart[-1])], dtype=torch.int64, device=device)])
    col = torch.cat([(t(g.col, torch.int32) + int(vstart[j])) for j, g in enumerate(graphs)] +
                    [torch.zeros(0, dtype=torch.int32, device=device)])
    k = torch.cat([t(g.k, torch.int64) for g in graphs] + [torch.zeros(0, dtype=torch.int64, device=device)])
    wt = None
    if kind != "none":
        wt = torch.cat([torch.as_tensor(g.wt).to(device) for g in graphs])
    s = None
    if any(g.s is not None for g in graphs):
        s = torch.cat([t(g.s, torch.int64) if g.s is not None else torch.zeros(g.n, dtype=torch.int64, device=device)
                       for g in graphs])
    kk = None
    if any(g.kk is not None for g in graphs):
        kk = torch.cat([t(g.kk, torch.int64) if g.kk is not None else t(g.k, torch.int64) ** 2 for g in graphs])
    return HostGraph(off, col, k, wt, s, kk, kind), vstart


def sbm_batch(jobs: int, seed: int = 0, device="cpu", nmin: int = 100, nmax: int = 50000, block: int = 500,
              mixing: float = 0.2):
    """The many-graph batch: job i is sbm_blocks(n_i, block, d_i, mixing,
    seed = i) with (n_i, d_i, lambda_i) from sbm_job_spec(i, seed).  Returns
    (graphs, lambdas as (p, q))."""
    graphs, lams = [], []
    for i in range(jobs):
        n, d, p, q = sbm_job_spec(i, seed, nmin, nmax)
        graphs.append(sbm_blocks(n, block, d, mixing, seed=i, device=device))
        lams.append((p, q))
    return graphs, lams
