"""CPU parity oracle for the LambdaCC best-move / compress / objective path.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The product library
(``paper_2108_01731_amd``) never imports this package, and this package never
imports the product library.

The arithmetic lives in ``lcc_oracle.c`` (plain C, integer only; see its
header for the paper passages it follows).  It is built twice from the same
source: ``liblcc_oracle.so`` single-threaded, and ``liblcc_oracle_omp.so``
with OpenMP, whose only parallel loop is the per-vertex decisions of a
sub-round against one snapshot (identical results; ``use_openmp()`` selects
it).  This module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lcc_oracle.c")
_LIB = os.path.join(_HERE, "liblcc_oracle.so")
_LIB_OMP = os.path.join(_HERE, "liblcc_oracle_omp.so")

OK, INVALID, OVERFLOW, NOMEM = 0, 1, 2, 3
FRONTIER_ALL, FRONTIER_NBR, FRONTIER_CLUSTERS = 0, 1, 2
TERM_NO_MOVES, TERM_NUM_ITER, TERM_STOPPED = 0, 1, 2
ISO = -1
MAX_ITER_STATS = 64
MAX_LEVELS = 64


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, -O2): the single-threaded
    library and the OpenMP one."""
    for out, extra in ((_LIB, ["-Wno-unknown-pragmas"]), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out):
            tmp = out + ".tmp"
            subprocess.check_call(
                ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", *extra, "-shared", "-fPIC", _SRC, "-o", tmp]
            )
            os.replace(tmp, out)
    return _LIB


def use_openmp(on: bool = True):
    """Route the module-level functions to the OpenMP build (True) or the
    single-threaded one (False).  Returns the previous selection."""
    if on and not os.path.exists(_LIB_OMP):
        build(force=True)
    return use_library(_LIB_OMP if on else None)


def num_threads() -> int:
    """Threads the selected build's decision loop uses (1 single-threaded)."""
    return int(_load().orc_num_threads())


class _Graph(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("arcs", ctypes.c_int64),
        ("off", ctypes.c_void_p),
        ("col", ctypes.c_void_p),
        ("wt", ctypes.c_void_p),
        ("k", ctypes.c_void_p),
        ("s", ctypes.c_void_p),
        ("kk", ctypes.c_void_p),
    ]


class _GraphOut(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("arcs", ctypes.c_int64),
        ("off", ctypes.POINTER(ctypes.c_int64)),
        ("col", ctypes.POINTER(ctypes.c_int32)),
        ("wt", ctypes.POINTER(ctypes.c_int64)),
        ("k", ctypes.POINTER(ctypes.c_int64)),
        ("s", ctypes.POINTER(ctypes.c_int64)),
        ("kk", ctypes.POINTER(ctypes.c_int64)),
    ]


class _Params(ctypes.Structure):
    _fields_ = [
        ("S", ctypes.c_int32),
        ("num_iter", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("frontier", ctypes.c_int32),
        ("refine", ctypes.c_int32),
        ("allow_isolate", ctypes.c_int32),
        ("max_levels", ctypes.c_int32),
        ("stop_after_subrounds", ctypes.c_int64),
    ]


class _BMStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("subrounds", ctypes.c_int32),
        ("moved_any", ctypes.c_int32),
        ("term", ctypes.c_int32),
        ("moves", ctypes.c_int64),
        ("arcs_scanned", ctypes.c_int64),
        ("vertices_processed", ctypes.c_int64),
        ("active_per_iter", ctypes.c_int64 * MAX_ITER_STATS),
        ("moves_per_iter", ctypes.c_int64 * MAX_ITER_STATS),
    ]


class _ClusterStats(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32),
        ("top_moved", ctypes.c_int32),
        ("n_level", ctypes.c_int64 * MAX_LEVELS),
        ("arcs_level", ctypes.c_int64 * MAX_LEVELS),
        ("iters_coarsen", ctypes.c_int32 * MAX_LEVELS),
        ("iters_refine", ctypes.c_int32 * MAX_LEVELS),
        ("moves_total", ctypes.c_int64),
        ("arcs_scanned_total", ctypes.c_int64),
        ("clusters", ctypes.c_int64),
    ]


_libs = {}


def build_variant(src_text: str, out_path: str) -> str:
    """Compile a modified copy of the oracle source (used by the tests that
    plant a mistake in the oracle and check that some pin catches it)."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-w", "-shared", "-fPIC", src, "-o", out_path])
    return out_path


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


_current = [None]


def use_library(path=None):
    """Select the shared library the module-level functions call (None = the
    regular oracle build).  Returns the previous selection."""
    prev = _current[0]
    _current[0] = path
    return prev


def _load():
    path = _current[0] or _LIB
    if path not in _libs:
        if path == _LIB and not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, u64, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32
        gp = ctypes.POINTER(_Graph)
        sig = {
            "orc_mix64": (u64, [u64]),
            "orc_num_threads": (ctypes.c_int, []),
            "orc_round_hash": (u64, [u64, i32, i32, i32]),
            "orc_color": (i32, [u64, i64, i32]),
            "orc_validate": (ctypes.c_int, [gp]),
            "orc_precheck": (ctypes.c_int, [gp, i64, i64]),
            "orc_check_symmetric": (ctypes.c_int, [gp]),
            "orc_subround": (i64, [gp, i64, i64, i32, P, P, i64, P]),
            "orc_decide_many": (ctypes.c_int, [gp, i64, i64, i32, P, P, i64, P]),
            "orc_frontier_nbr": (None, [gp, P, i64, P]),
            "orc_best_move": (
                ctypes.c_int,
                [gp, i64, i64, ctypes.POINTER(_Params), i32, i32, P, ctypes.POINTER(_BMStats)],
            ),
            "orc_compress": (ctypes.c_int, [gp, P, ctypes.POINTER(_GraphOut), P]),
            "orc_graph_free": (None, [ctypes.POINTER(_GraphOut)]),
            "orc_objective": (
                ctypes.c_int,
                [gp, i64, i64, P, ctypes.POINTER(i64), ctypes.POINTER(u64)],
            ),
            "orc_canonical_labels": (ctypes.c_int, [i64, P, P]),
            "orc_cluster": (
                ctypes.c_int,
                [
                    gp, i64, i64, ctypes.POINTER(_Params), P,
                    ctypes.POINTER(i64), ctypes.POINTER(u64), ctypes.POINTER(_ClusterStats),
                ],
            ),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _libs[path] = lib
    return _libs[path]


# ----------------------------------------------------------------- data types


@dataclass
class Graph:
    """A host CSR graph for the oracle.  ``wt`` None means unit weights;
    ``s`` None means zero self weights; ``kk`` None means kk = k^2."""

    off: np.ndarray
    col: np.ndarray
    k: np.ndarray
    wt: Optional[np.ndarray] = None
    s: Optional[np.ndarray] = None
    kk: Optional[np.ndarray] = None

    def __post_init__(self):
        self.off = np.ascontiguousarray(self.off, dtype=np.int64)
        self.col = np.ascontiguousarray(self.col, dtype=np.int32)
        self.k = np.ascontiguousarray(self.k, dtype=np.int64)
        if self.wt is not None:
            self.wt = np.ascontiguousarray(self.wt, dtype=np.int64)
        if self.s is not None:
            self.s = np.ascontiguousarray(self.s, dtype=np.int64)
        if self.kk is not None:
            self.kk = np.ascontiguousarray(self.kk, dtype=np.int64)

    @property
    def n(self) -> int:
        return len(self.off) - 1

    @property
    def arcs(self) -> int:
        return len(self.col)

    def _c(self) -> _Graph:
        def ptr(a):
            return None if a is None else a.ctypes.data

        return _Graph(self.n, self.arcs, ptr(self.off), ptr(self.col), ptr(self.wt),
                      ptr(self.k), ptr(self.s), ptr(self.kk))


@dataclass
class Params:
    S: int = 4
    num_iter: int = 10
    seed: int = 1
    frontier: int = FRONTIER_NBR
    refine: int = 1
    allow_isolate: int = 1
    max_levels: int = 64
    stop_after_subrounds: int = 0

    def _c(self) -> _Params:
        return _Params(self.S, self.num_iter, self.seed & (2**64 - 1), self.frontier, self.refine,
                       self.allow_isolate, self.max_levels, self.stop_after_subrounds)


def _chk(rc: int, what: str):
    if rc != OK:
        raise OracleError(rc, what)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


# ------------------------------------------------------------------ functions


def mix64(x: int) -> int:
    return int(_load().orc_mix64(x & (2**64 - 1)))


def round_hash(seed: int, level: int, phase: int, it: int) -> int:
    return int(_load().orc_round_hash(seed & (2**64 - 1), level, phase, it))


def color(h: int, v: int, S: int) -> int:
    return int(_load().orc_color(h & (2**64 - 1), v, S))


def validate(g: Graph) -> int:
    cg = g._c()
    return int(_load().orc_validate(ctypes.byref(cg)))


def precheck(g: Graph, p: int, q: int) -> int:
    cg = g._c()
    return int(_load().orc_precheck(ctypes.byref(cg), p, q))


def check_symmetric(g: Graph) -> bool:
    cg = g._c()
    return bool(_load().orc_check_symmetric(ctypes.byref(cg)))


def subround(g: Graph, p: int, q: int, C, U, allow_isolate: int = 1):
    """One synchronous sub-round over the explicit vertex list U.
    Returns (C_after, D, moved)."""
    C = _i32(C).copy()
    U = _i32(U)
    D = np.zeros(max(len(U), 1), dtype=np.int32)
    cg = g._c()
    moved = _load().orc_subround(ctypes.byref(cg), p, q, allow_isolate, C.ctypes.data,
                                 U.ctypes.data, len(U), D.ctypes.data)
    if moved < 0:
        raise OracleError(INVALID, "subround")
    return C, D[: len(U)], int(moved)


def decide_many(g: Graph, p: int, q: int, C, U, allow_isolate: int = 1) -> np.ndarray:
    C = _i32(C)
    U = _i32(U)
    D = np.zeros(max(len(U), 1), dtype=np.int32)
    cg = g._c()
    _chk(_load().orc_decide_many(ctypes.byref(cg), p, q, allow_isolate, C.ctypes.data,
                                 U.ctypes.data, len(U), D.ctypes.data), "decide_many")
    return D[: len(U)]


def frontier_nbr(g: Graph, movers) -> np.ndarray:
    movers = _i32(movers)
    flags = np.zeros(max(g.n, 1), dtype=np.uint8)
    cg = g._c()
    _load().orc_frontier_nbr(ctypes.byref(cg), movers.ctypes.data, len(movers), flags.ctypes.data)
    return flags[: g.n]


def _bm_stats(st: _BMStats) -> dict:
    it = min(st.iterations, MAX_ITER_STATS)
    return {
        "iterations": st.iterations,
        "subrounds": st.subrounds,
        "moved_any": st.moved_any,
        "term": st.term,
        "moves": st.moves,
        "arcs_scanned": st.arcs_scanned,
        "vertices_processed": st.vertices_processed,
        "active_per_iter": list(st.active_per_iter[:it]),
        "moves_per_iter": list(st.moves_per_iter[:it]),
    }


def best_move(g: Graph, p: int, q: int, params: Params, C=None, level: int = 0, phase: int = 0):
    """Best-Moves from clustering C (identity if None).  Returns (C, stats)."""
    C = np.arange(g.n, dtype=np.int32) if C is None else _i32(C).copy()
    st = _BMStats()
    cp = params._c()
    cg = g._c()
    _chk(_load().orc_best_move(ctypes.byref(cg), p, q, ctypes.byref(cp), level, phase,
                               C.ctypes.data, ctypes.byref(st)), "best_move")
    return C, _bm_stats(st)


def compress(g: Graph, C):
    """Returns (coarse Graph with int64 weights, map)."""
    C = _i32(C)
    out = _GraphOut()
    mp = np.zeros(max(g.n, 1), dtype=np.int32)
    cg = g._c()
    lib = _load()
    _chk(lib.orc_compress(ctypes.byref(cg), C.ctypes.data, ctypes.byref(out), mp.ctypes.data),
         "compress")
    try:
        n2, m2 = out.n, out.arcs

        def take(ptr, cnt, dt):
            if cnt == 0:
                return np.zeros(0, dtype=dt)
            return np.ctypeslib.as_array(ptr, shape=(cnt,)).astype(dt, copy=True)

        g2 = Graph(off=take(out.off, n2 + 1, np.int64), col=take(out.col, m2, np.int32),
                   k=take(out.k, n2, np.int64), wt=take(out.wt, m2, np.int64),
                   s=take(out.s, n2, np.int64), kk=take(out.kk, n2, np.int64))
    finally:
        lib.orc_graph_free(ctypes.byref(out))
    return g2, mp[: g.n]


def objective(g: Graph, p: int, q: int, C) -> int:
    """Exact numerator N of the unordered-pair objective (value N / q)."""
    C = _i32(C)
    hi, lo = ctypes.c_int64(), ctypes.c_uint64()
    cg = g._c()
    _chk(_load().orc_objective(ctypes.byref(cg), p, q, C.ctypes.data, ctypes.byref(hi),
                               ctypes.byref(lo)), "objective")
    return (hi.value << 64) | lo.value


def canonical_labels(C) -> np.ndarray:
    C = _i32(C)
    lab = np.zeros(max(len(C), 1), dtype=np.int32)
    _chk(_load().orc_canonical_labels(len(C), C.ctypes.data, lab.ctypes.data), "labels")
    return lab[: len(C)]


def cluster(g: Graph, p: int, q: int, params: Params):
    """Parallel-CC with refinement.  Returns (labels, N, stats)."""
    lab = np.zeros(max(g.n, 1), dtype=np.int32)
    hi, lo = ctypes.c_int64(), ctypes.c_uint64()
    cs = _ClusterStats()
    cp = params._c()
    cg = g._c()
    _chk(_load().orc_cluster(ctypes.byref(cg), p, q, ctypes.byref(cp), lab.ctypes.data,
                             ctypes.byref(hi), ctypes.byref(lo), ctypes.byref(cs)), "cluster")
    L = cs.levels
    stats = {
        "levels": L,
        "top_moved": cs.top_moved,
        "n_level": list(cs.n_level[:L]),
        "arcs_level": list(cs.arcs_level[:L]),
        "iters_coarsen": list(cs.iters_coarsen[:L]),
        "iters_refine": list(cs.iters_refine[:L]),
        "moves_total": cs.moves_total,
        "arcs_scanned_total": cs.arcs_scanned_total,
        "clusters": cs.clusters,
    }
    return lab[: g.n], (hi.value << 64) | lo.value, stats
