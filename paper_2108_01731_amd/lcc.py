"""Python binding of liblcc (include/lcc.h): argument marshalling only.

Every computation runs in the HIP library; this module converts torch tensors
(device memory) and Python numbers into the C structs, calls the exported
function of the same name and converts the outputs back.  There is no CPU
fallback: if ``liblcc.so`` is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblcc.so")

LCC_OK, LCC_ERR_INVALID_ARG, LCC_ERR_OVERFLOW, LCC_ERR_OUT_OF_MEMORY, LCC_ERR_DEVICE, LCC_ERR_UNSUPPORTED = range(6)
LCC_WT_UNIT, LCC_WT_I16, LCC_WT_I32, LCC_WT_I64 = range(4)
LCC_FRONTIER_ALL, LCC_FRONTIER_NBR, LCC_FRONTIER_CLUSTERS = 0, 1, 2
LCC_TERM_NO_MOVES, LCC_TERM_NUM_ITER, LCC_TERM_STOPPED = 0, 1, 2
LCC_HUB_LIMIT_MAX = 8601  # default and largest Params.hub_limit
LCC_NOALLOC_MAX_N = 1048576  # largest graph lcc_objective_noalloc accepts
LCC_SMALL_LEVEL_MAX = 8192  # largest Params.small_level
MAX_ITER_STATS = 64
MAX_LEVELS = 64

_WT_KIND = {"none": LCC_WT_UNIT, "i16": LCC_WT_I16, "i32": LCC_WT_I32, "i64": LCC_WT_I64}
_WT_DTYPE = {LCC_WT_I16: torch.int16, LCC_WT_I32: torch.int32, LCC_WT_I64: torch.int64}


class LccError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"liblcc error {code}: {msg}")
        self.code = code


class _Graph(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("arcs", ctypes.c_int64), ("off", ctypes.c_void_p), ("col", ctypes.c_void_p),
        ("wt", ctypes.c_void_p), ("wt_kind", ctypes.c_int32), ("reserved0", ctypes.c_int32),
        ("k", ctypes.c_void_p), ("s", ctypes.c_void_p), ("kk", ctypes.c_void_p),
    ]


class _Lambda(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int64), ("q", ctypes.c_int64)]


class _Params(ctypes.Structure):
    _fields_ = [
        ("S", ctypes.c_int32), ("num_iter", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("frontier", ctypes.c_int32), ("refine", ctypes.c_int32), ("allow_isolate", ctypes.c_int32),
        ("max_levels", ctypes.c_int32), ("stop_after_subrounds", ctypes.c_int64),
        ("validate", ctypes.c_int32), ("timing", ctypes.c_int32), ("hub_limit", ctypes.c_int32),
        ("queue_ahead", ctypes.c_int32), ("small_level", ctypes.c_int32), ("low_merge", ctypes.c_int32),
        ("hub_row_limit", ctypes.c_int32), ("score_pruning", ctypes.c_int32), ("async_moves", ctypes.c_int32), ("no_graph_replay", ctypes.c_int32),
    ]


class _BMStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32), ("subrounds", ctypes.c_int32), ("moved_any", ctypes.c_int32),
        ("term", ctypes.c_int32), ("moves", ctypes.c_int64), ("arcs_scanned", ctypes.c_int64),
        ("vertices_processed", ctypes.c_int64), ("candidates", ctypes.c_int64),
        ("active_per_iter", ctypes.c_int64 * MAX_ITER_STATS), ("moves_per_iter", ctypes.c_int64 * MAX_ITER_STATS),
    ]


class _Objective(ctypes.Structure):
    _fields_ = [("num_hi", ctypes.c_int64), ("num_lo", ctypes.c_uint64), ("den", ctypes.c_int64),
                ("value", ctypes.c_double)]


class _ClusterStats(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32), ("top_moved", ctypes.c_int32),
        ("n_level", ctypes.c_int64 * MAX_LEVELS), ("arcs_level", ctypes.c_int64 * MAX_LEVELS),
        ("iters_coarsen", ctypes.c_int32 * MAX_LEVELS), ("iters_refine", ctypes.c_int32 * MAX_LEVELS),
        ("moves_total", ctypes.c_int64), ("arcs_scanned_total", ctypes.c_int64), ("clusters", ctypes.c_int64),
        ("ms_best_move", ctypes.c_double), ("ms_compress", ctypes.c_double), ("ms_total", ctypes.c_double),
    ]


class _JobOut(ctypes.Structure):
    _fields_ = [("obj", _Objective), ("clusters", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("top_moved", ctypes.c_int32)]


class _BatchStats(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32), ("reserved0", ctypes.c_int32),
        ("n_level", ctypes.c_int64 * MAX_LEVELS), ("arcs_level", ctypes.c_int64 * MAX_LEVELS),
        ("moves_total", ctypes.c_int64), ("arcs_scanned_total", ctypes.c_int64),
        ("ms_best_move", ctypes.c_double), ("ms_compress", ctypes.c_double), ("ms_total", ctypes.c_double),
    ]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


class _KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 64), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("items", ctypes.c_double)]


EXPORTS = (
    "lcc_params_default", "lcc_last_error", "lcc_ctx_create", "lcc_ctx_destroy", "lcc_best_move", "lcc_compress",
    "lcc_graph_owned_view", "lcc_graph_owned_free", "lcc_objective", "lcc_objective_noalloc", "lcc_cluster",
    "lcc_cluster_batch", "lcc_sweep", "lcc_ctx_kernel_stats", "lcc_ctx_reset_kernel_stats",
)

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads liblcc.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run paper_2108_01731_amd.build.build() first")
    lib = ctypes.CDLL(path)
    P, i32, i64, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32
    gp = ctypes.POINTER(_Graph)
    lib.lcc_params_default.restype = None
    lib.lcc_params_default.argtypes = [ctypes.POINTER(_Params)]
    lib.lcc_last_error.restype = ctypes.c_char_p
    lib.lcc_last_error.argtypes = []
    lib.lcc_ctx_create.restype = st
    lib.lcc_ctx_create.argtypes = [i32, ctypes.POINTER(_Allocator), ctypes.POINTER(P)]
    lib.lcc_ctx_destroy.restype = st
    lib.lcc_ctx_destroy.argtypes = [P]
    lib.lcc_best_move.restype = st
    lib.lcc_best_move.argtypes = [P, gp, _Lambda, ctypes.POINTER(_Params), i32, i32, P, ctypes.POINTER(_BMStats), P]
    lib.lcc_compress.restype = st
    lib.lcc_compress.argtypes = [P, gp, P, ctypes.POINTER(P), P, P]
    lib.lcc_graph_owned_view.restype = st
    lib.lcc_graph_owned_view.argtypes = [P, gp]
    lib.lcc_graph_owned_free.restype = st
    lib.lcc_graph_owned_free.argtypes = [P, P]
    lib.lcc_objective.restype = st
    lib.lcc_objective.argtypes = [P, gp, _Lambda, P, ctypes.POINTER(_Objective), P]
    lib.lcc_objective_noalloc.restype = st
    lib.lcc_objective_noalloc.argtypes = [P, gp, _Lambda, P, ctypes.POINTER(_Objective), P]
    lib.lcc_cluster.restype = st
    lib.lcc_cluster.argtypes = [P, gp, _Lambda, ctypes.POINTER(_Params), P, ctypes.POINTER(_Objective),
                                ctypes.POINTER(_ClusterStats), P]
    lib.lcc_cluster_batch.restype = st
    lib.lcc_cluster_batch.argtypes = [P, gp, i64, ctypes.POINTER(i64), ctypes.POINTER(_Lambda),
                                      ctypes.POINTER(_Params), P, ctypes.POINTER(_JobOut),
                                      ctypes.POINTER(_BatchStats), P]
    lib.lcc_sweep.restype = st
    lib.lcc_sweep.argtypes = [P, gp, i64, ctypes.POINTER(_Lambda), ctypes.POINTER(_Params), P,
                              ctypes.POINTER(_JobOut), ctypes.POINTER(_BatchStats), P]
    lib.lcc_ctx_kernel_stats.restype = st
    lib.lcc_ctx_kernel_stats.argtypes = [P, ctypes.POINTER(_KernelStat), i32, ctypes.POINTER(i32)]
    lib.lcc_ctx_reset_kernel_stats.restype = st
    lib.lcc_ctx_reset_kernel_stats.argtypes = [P]
    _lib = lib
    return lib


def _check(rc: int):
    if rc != LCC_OK:
        raise LccError(rc, _lib.lcc_last_error().decode(errors="replace"))


# ------------------------------------------------------------------ data


@dataclass
class DeviceGraph:
    """CSR arrays as torch tensors on one GPU (see lcc_graph in include/lcc.h)."""

    off: torch.Tensor
    col: torch.Tensor
    k: torch.Tensor
    wt: Optional[torch.Tensor] = None
    s: Optional[torch.Tensor] = None
    kk: Optional[torch.Tensor] = None

    @property
    def n(self) -> int:
        return int(self.off.shape[0]) - 1

    @property
    def arcs(self) -> int:
        return int(self.col.shape[0])

    @property
    def wt_kind(self) -> int:
        if self.wt is None:
            return LCC_WT_UNIT
        return {torch.int16: LCC_WT_I16, torch.int32: LCC_WT_I32, torch.int64: LCC_WT_I64}[self.wt.dtype]

    @staticmethod
    def from_host(h, device="cuda") -> "DeviceGraph":
        """From a graphgen.HostGraph (numpy or torch arrays)."""
        t = h.to(device)
        return DeviceGraph(off=t.off.contiguous(), col=t.col.contiguous(), k=t.k.contiguous(),
                           wt=None if t.wt is None else t.wt.contiguous(),
                           s=None if t.s is None else t.s.contiguous(),
                           kk=None if t.kk is None else t.kk.contiguous())

    def _c(self) -> _Graph:
        def ptr(t):
            return None if t is None else t.data_ptr()

        for name, t, dt in (("off", self.off, torch.int64), ("col", self.col, torch.int32), ("k", self.k, torch.int64),
                            ("s", self.s, torch.int64), ("kk", self.kk, torch.int64)):
            if t is not None and (t.dtype != dt or not t.is_contiguous()):
                raise TypeError(f"{name} must be a contiguous {dt} tensor")
        if self.wt is not None and not self.wt.is_contiguous():
            raise TypeError("wt must be contiguous")
        return _Graph(self.n, self.arcs, ptr(self.off), ptr(self.col), ptr(self.wt), self.wt_kind, 0,
                      ptr(self.k), ptr(self.s), ptr(self.kk))


@dataclass
class Params:
    S: int = 4
    num_iter: int = 10
    seed: int = 1
    frontier: int = LCC_FRONTIER_NBR
    refine: int = 1
    allow_isolate: int = 1
    max_levels: int = 64
    stop_after_subrounds: int = 0
    validate: int = 1
    timing: int = 0
    hub_limit: int = 0
    queue_ahead: int = 0
    small_level: int = 0
    low_merge: int = 0
    hub_row_limit: int = 0
    score_pruning: int = 0
    async_moves: int = 0
    no_graph_replay: int = 0

    def _c(self) -> _Params:
        p = _Params()
        p.S, p.num_iter, p.seed = self.S, self.num_iter, self.seed & (2**64 - 1)
        p.frontier, p.refine, p.allow_isolate = self.frontier, self.refine, self.allow_isolate
        p.max_levels, p.stop_after_subrounds = self.max_levels, self.stop_after_subrounds
        p.validate, p.timing, p.hub_limit = self.validate, self.timing, self.hub_limit
        p.queue_ahead, p.small_level, p.low_merge = self.queue_ahead, self.small_level, self.low_merge
        p.hub_row_limit, p.score_pruning = self.hub_row_limit, self.score_pruning
        p.async_moves, p.no_graph_replay = self.async_moves, self.no_graph_replay
        return p


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class TorchAllocator:
    """lcc_allocator callbacks backed by torch's caching allocator: the
    library's scratch and contracted graphs come from the same pool as the
    caller's tensors, and a growing buffer goes back to the pool instead of
    through hipFree.  The callbacks must outlive the context that uses them
    (Context keeps a reference)."""

    def __init__(self, device: int = 0):
        self.device = device
        self.live = {}  # ptr -> bytes, for diagnostics and tests

        def alloc(user, nbytes, stream):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0))
            except Exception:  # out of memory: the library reports LCC_ERR_OUT_OF_MEMORY
                return None
            self.live[ptr] = int(nbytes)
            return ptr

        def free(user, ptr, nbytes, stream):
            try:
                self.live.pop(ptr, None)
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:
                pass

        self._alloc_fn = _ALLOC_FN(alloc)
        self._free_fn = _FREE_FN(free)
        self.c = _Allocator(self._alloc_fn, self._free_fn, None)


class Context:
    """An lcc_ctx bound to one GPU; `allocator` (a TorchAllocator, or None
    for hipMalloc) supplies its device memory."""

    def __init__(self, device: int = 0, allocator: Optional[TorchAllocator] = None):
        lib = load_library()
        self.device = device
        self.allocator = allocator
        h = ctypes.c_void_p()
        _check(lib.lcc_ctx_create(device, ctypes.byref(allocator.c) if allocator else None, ctypes.byref(h)))
        self._h = h

    def close(self):
        if self._h:
            _check(_lib.lcc_ctx_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def kernel_stats(self) -> dict:
        cnt = ctypes.c_int32()
        _check(_lib.lcc_ctx_kernel_stats(self._h, None, 0, ctypes.byref(cnt)))
        arr = (_KernelStat * max(cnt.value, 1))()
        _check(_lib.lcc_ctx_kernel_stats(self._h, arr, cnt.value, ctypes.byref(cnt)))
        return {arr[i].name.decode(): {"launches": arr[i].launches, "ms": arr[i].total_ms, "bytes": arr[i].bytes,
                                       "items": arr[i].items} for i in range(cnt.value)}

    def reset_kernel_stats(self):
        _check(_lib.lcc_ctx_reset_kernel_stats(self._h))


_contexts = {}


def context(device: int = 0) -> Context:
    if device not in _contexts:
        _contexts[device] = Context(device)
    return _contexts[device]


def _lam(p: int, q: int) -> _Lambda:
    return _Lambda(int(p), int(q))


def _bm_stats(st: _BMStats) -> dict:
    it = min(st.iterations, MAX_ITER_STATS)
    return {"iterations": st.iterations, "subrounds": st.subrounds, "moved_any": st.moved_any, "term": st.term,
            "moves": st.moves, "arcs_scanned": st.arcs_scanned, "vertices_processed": st.vertices_processed,
            "candidates": st.candidates, "active_per_iter": list(st.active_per_iter[:it]),
            "moves_per_iter": list(st.moves_per_iter[:it])}


# ------------------------------------------------------------- entry points


def _check_ids(C: torch.Tensor):
    """A clustering argument: the library reads it as int32[n] in place."""
    if not isinstance(C, torch.Tensor) or C.dtype != torch.int32 or not C.is_contiguous():
        raise TypeError("C must be a contiguous int32 tensor")


def lcc_best_move(ctx: Context, g: DeviceGraph, p: int, q: int, params: Params, C: torch.Tensor, level: int = 0,
                  phase: int = 0, stream=None) -> dict:
    """Best-Moves from clustering C (int32 device tensor, updated in place)."""
    _check_ids(C)
    st = _BMStats()
    cg, cp = g._c(), params._c()
    _check(_lib.lcc_best_move(ctx._h, ctypes.byref(cg), _lam(p, q), ctypes.byref(cp), level, phase,
                              C.data_ptr() if C.numel() else None, ctypes.byref(st), _stream_ptr(stream)))
    return _bm_stats(st)


def _hip_copy(dst: torch.Tensor, src_ptr: int, nbytes: int):
    if nbytes == 0:
        return
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.restype = ctypes.c_int
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    rc = hip.hipMemcpy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src_ptr), nbytes, 3)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed with {rc}")


def lcc_compress(ctx: Context, g: DeviceGraph, C: torch.Tensor, stream=None):
    """Returns (contracted DeviceGraph, map int32 tensor)."""
    _check_ids(C)
    dev = g.off.device
    mp = torch.empty(g.n, dtype=torch.int32, device=dev)
    h = ctypes.c_void_p()
    cg = g._c()
    _check(_lib.lcc_compress(ctx._h, ctypes.byref(cg), C.data_ptr() if C.numel() else None, ctypes.byref(h),
                             mp.data_ptr() if mp.numel() else None, _stream_ptr(stream)))
    try:
        v = _Graph()
        _check(_lib.lcc_graph_owned_view(h, ctypes.byref(v)))
        n2, m2 = v.n, v.arcs
        out = DeviceGraph(off=torch.empty(n2 + 1, dtype=torch.int64, device=dev),
                          col=torch.empty(m2, dtype=torch.int32, device=dev),
                          k=torch.empty(n2, dtype=torch.int64, device=dev),
                          wt=torch.empty(m2, dtype=_WT_DTYPE[v.wt_kind], device=dev),
                          s=torch.empty(n2, dtype=torch.int64, device=dev),
                          kk=torch.empty(n2, dtype=torch.int64, device=dev))
        torch.cuda.synchronize(dev)
        _hip_copy(out.off, v.off, (n2 + 1) * 8)
        _hip_copy(out.col, v.col, m2 * 4)
        _hip_copy(out.wt, v.wt, m2 * out.wt.element_size())
        _hip_copy(out.k, v.k, n2 * 8)
        _hip_copy(out.s, v.s, n2 * 8)
        _hip_copy(out.kk, v.kk, n2 * 8)
    finally:
        _check(_lib.lcc_graph_owned_free(ctx._h, h))
    return out, mp


def _num(o: _Objective) -> int:
    return (o.num_hi << 64) | o.num_lo


def lcc_objective(ctx: Context, g: DeviceGraph, p: int, q: int, C: torch.Tensor, stream=None) -> int:
    """Exact numerator N of the objective (value N / q)."""
    _check_ids(C)
    o = _Objective()
    cg = g._c()
    _check(_lib.lcc_objective(ctx._h, ctypes.byref(cg), _lam(p, q), C.data_ptr() if C.numel() else None,
                              ctypes.byref(o), _stream_ptr(stream)))
    return _num(o)


def lcc_objective_noalloc(ctx: Context, g: DeviceGraph, p: int, q: int, C: torch.Tensor, stream=None) -> int:
    """As lcc_objective, through the entry point that allocates no device
    memory (graphs of at most LCC_NOALLOC_MAX_N vertices)."""
    _check_ids(C)
    o = _Objective()
    cg = g._c()
    _check(_lib.lcc_objective_noalloc(ctx._h, ctypes.byref(cg), _lam(p, q), C.data_ptr() if C.numel() else None,
                                      ctypes.byref(o), _stream_ptr(stream)))
    return _num(o)


def lcc_cluster(ctx: Context, g: DeviceGraph, p: int, q: int, params: Params, stream=None):
    """Parallel-CC with refinement.  Returns (labels int32 tensor, N, stats)."""
    lab = torch.empty(g.n, dtype=torch.int32, device=g.off.device)
    o = _Objective()
    cs = _ClusterStats()
    cg, cp = g._c(), params._c()
    _check(_lib.lcc_cluster(ctx._h, ctypes.byref(cg), _lam(p, q), ctypes.byref(cp),
                            lab.data_ptr() if lab.numel() else None, ctypes.byref(o), ctypes.byref(cs),
                            _stream_ptr(stream)))
    L = cs.levels
    stats = {"levels": L, "top_moved": cs.top_moved, "n_level": list(cs.n_level[:L]),
             "arcs_level": list(cs.arcs_level[:L]), "iters_coarsen": list(cs.iters_coarsen[:L]),
             "iters_refine": list(cs.iters_refine[:L]), "moves_total": cs.moves_total,
             "arcs_scanned_total": cs.arcs_scanned_total, "clusters": cs.clusters,
             "ms_best_move": cs.ms_best_move, "ms_compress": cs.ms_compress, "ms_total": cs.ms_total}
    return lab, _num(o), stats


SWEEP_MAX = 16


def _batch_results(outs, bs, J):
    jobs = [{"N": _num(outs[j].obj), "clusters": outs[j].clusters, "levels": outs[j].levels,
             "top_moved": outs[j].top_moved} for j in range(J)]
    L = bs.levels
    stats = {"levels": L, "n_level": list(bs.n_level[:L]), "arcs_level": list(bs.arcs_level[:L]),
             "moves_total": bs.moves_total, "arcs_scanned_total": bs.arcs_scanned_total,
             "ms_best_move": bs.ms_best_move, "ms_compress": bs.ms_compress, "ms_total": bs.ms_total}
    return jobs, stats


def lcc_sweep(ctx: Context, g: DeviceGraph, lambdas, params: Params, stream=None):
    """Parallel-CC of one graph under up to 16 resolutions (p, q) at once;
    resolution j gives exactly lcc_cluster(g, *lambdas[j]).  Returns (labels
    int32 tensor of shape [len(lambdas), n], per-resolution list of dicts
    {N, clusters, levels, top_moved}, batch stats)."""
    J = len(lambdas)
    lams = (_Lambda * max(J, 1))(*[_lam(int(p), int(q)) for p, q in lambdas])
    outs = (_JobOut * max(J, 1))()
    bs = _BatchStats()
    lab = torch.empty((J, g.n), dtype=torch.int32, device=g.off.device)
    cg, cp = g._c(), params._c()
    _check(_lib.lcc_sweep(ctx._h, ctypes.byref(cg), J, lams, ctypes.byref(cp),
                          lab.data_ptr() if lab.numel() else None, outs, ctypes.byref(bs), _stream_ptr(stream)))
    jobs, stats = _batch_results(outs, bs, J)
    return lab, jobs, stats


def lcc_cluster_batch(ctx: Context, g: DeviceGraph, job_start, lambdas, params: Params, stream=None):
    """Parallel-CC on jobs packed block-diagonally in g (job j owns vertices
    [job_start[j], job_start[j+1])), each with its own (p, q).  Returns
    (labels int32 tensor of job-local canonical labels, per-job list of dicts
    {N, clusters, levels, top_moved}, batch stats)."""
    J = len(lambdas)
    if len(job_start) != J + 1:
        raise ValueError("job_start needs one more entry than lambdas")
    starts = (ctypes.c_int64 * (J + 1))(*[int(x) for x in job_start])
    lams = (_Lambda * max(J, 1))(*[_lam(int(p), int(q)) for p, q in lambdas])
    outs = (_JobOut * max(J, 1))()
    bs = _BatchStats()
    lab = torch.empty(g.n, dtype=torch.int32, device=g.off.device)
    cg, cp = g._c(), params._c()
    _check(_lib.lcc_cluster_batch(ctx._h, ctypes.byref(cg), J, starts, lams, ctypes.byref(cp),
                                  lab.data_ptr() if lab.numel() else None, outs, ctypes.byref(bs),
                                  _stream_ptr(stream)))
    jobs, stats = _batch_results(outs, bs, J)
    return lab, jobs, stats
