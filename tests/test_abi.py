"""The C ABI library on a machine without a GPU: it loads, exports every
function include/lcc.h declares, its structs have the layout the header
gives, and host-side argument errors come back without touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2108_01731_amd import lcc as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lcc.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2108_01731_amd import build

        build.build()
    return L.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lcc_[a-z_]+)\s*\(", text)))


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert "lcc_best_move" in names and "lcc_cluster" in names
    assert "lcc_compress" in names and "lcc_objective" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.EXPORTS)


def test_struct_layout_matches_header(tmp_path):
    """sizeof / offsetof of the ABI structs from a C compiler vs ctypes."""
    fields = {
        "lcc_graph": (L._Graph, ["n", "arcs", "off", "col", "wt", "wt_kind", "k", "s", "kk"]),
        "lcc_params": (L._Params, ["S", "num_iter", "seed", "frontier", "stop_after_subrounds", "validate", "timing",
                                   "hub_limit", "low_merge", "hub_row_limit", "score_pruning", "async_moves",
                                   "no_graph_replay"]),
        "lcc_bm_stats": (L._BMStats, ["iterations", "moves", "candidates", "active_per_iter", "moves_per_iter"]),
        "lcc_objective_out": (L._Objective, ["num_hi", "num_lo", "den", "value"]),
        "lcc_cluster_stats": (L._ClusterStats, ["levels", "n_level", "iters_refine", "clusters", "ms_total"]),
        "lcc_job_out": (L._JobOut, ["obj", "clusters", "levels", "top_moved"]),
        "lcc_batch_stats": (L._BatchStats, ["levels", "n_level", "arcs_level", "moves_total", "ms_total"]),
        "lcc_kernel_stat": (L._KernelStat, ["name", "launches", "total_ms", "bytes", "items"]),
        "lcc_allocator": (L._Allocator, ["alloc", "free", "user"]),
    }
    src = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for s, (_, fl) in fields.items():
        src.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for f in fl:
            src.append(f'printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", str(c), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    for s, (cls, fl) in fields.items():
        assert int(got[s]) == ctypes.sizeof(cls), s
        for f in fl:
            assert int(got[f"{s}.{f}"]) == getattr(cls, f).offset, f"{s}.{f}"


def test_params_default(lib):
    p = L._Params()
    lib.lcc_params_default(ctypes.byref(p))
    assert (p.S, p.num_iter, p.seed, p.frontier, p.refine, p.allow_isolate, p.max_levels) == (4, 10, 1, 1, 1, 1, 64)
    assert p.stop_after_subrounds == 0 and p.validate == 1 and p.timing == 0
    d = L.Params()
    assert (d.S, d.num_iter, d.seed, d.frontier, d.refine, d.allow_isolate, d.max_levels) == (4, 10, 1, 1, 1, 1, 64)


def test_host_side_argument_errors(lib):
    assert lib.lcc_ctx_create(0, None, None) == L.LCC_ERR_INVALID_ARG
    # an allocator needs both callbacks (checked before any device call)
    half = L._Allocator(L._ALLOC_FN(lambda u, b, s: None), L._FREE_FN(), None)
    h = ctypes.c_void_p()
    assert lib.lcc_ctx_create(0, ctypes.byref(half), ctypes.byref(h)) == L.LCC_ERR_INVALID_ARG
    assert b"callback" in lib.lcc_last_error()
    assert b"NULL" in lib.lcc_last_error()
    g = L._Graph()
    p = L._Params()
    lib.lcc_params_default(ctypes.byref(p))
    st = L._BMStats()
    rc = lib.lcc_best_move(None, ctypes.byref(g), L._Lambda(1, 2), ctypes.byref(p), 0, 0, None, ctypes.byref(st), None)
    assert rc == L.LCC_ERR_INVALID_ARG
    o = L._Objective()
    assert lib.lcc_objective(None, ctypes.byref(g), L._Lambda(1, 2), None, ctypes.byref(o), None) == L.LCC_ERR_INVALID_ARG
    assert lib.lcc_cluster(None, ctypes.byref(g), L._Lambda(1, 2), ctypes.byref(p), None, None, None, None) == \
        L.LCC_ERR_INVALID_ARG
    cnt = ctypes.c_int32()
    assert lib.lcc_ctx_kernel_stats(None, None, 0, ctypes.byref(cnt)) == L.LCC_ERR_INVALID_ARG


def test_product_package_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2108_01731_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "lcc_oracle" not in text and "orc_" not in text, f


def test_hub_limit_bound_matches_the_kernel_tables():
    """lcc.h's LCC_HUB_LIMIT_MAX (and the binding's copy) equals the hub
    partition's default limit, and stays below the claim stop of its LDS
    table: a partition that refuses a claim must then count as overflowing."""
    hdr = open(HEADER).read()
    header_max = int(re.search(r"#define LCC_HUB_LIMIT_MAX (\d+)", hdr).group(1))
    src = open(os.path.join(ROOT, "paper_2108_01731_amd", "csrc", "bestmove.hip")).read()
    slots = int(re.search(r"constexpr int HP_SLOTS = (\d+);", src).group(1))
    nt = int(re.search(r"constexpr int HP_NT = (\d+);", src).group(1))
    assert re.search(r"constexpr int HP_LIMIT = HP_SLOTS \* 7 / 10;", src)
    assert re.search(r"constexpr int HP_STOP = HP_SLOTS - 2 \* HP_NT;", src)
    assert header_max == slots * 7 // 10 == L.LCC_HUB_LIMIT_MAX
    assert header_max < slots - 2 * nt


def test_binding_rejects_clusterings_of_the_wrong_type():
    """The library reads a clustering as int32[n]: the binding refuses other
    dtypes and non-contiguous views before anything reaches the C ABI."""
    import torch

    g = L.DeviceGraph(off=torch.zeros(5, dtype=torch.int64), col=torch.zeros(0, dtype=torch.int32),
                      k=torch.ones(4, dtype=torch.int64))
    bad = [torch.zeros(4, dtype=torch.int64), torch.zeros(8, dtype=torch.int32)[::2], [0, 0, 0, 0]]
    for C in bad:
        with pytest.raises(TypeError):
            L.lcc_best_move(None, g, 1, 2, L.Params(), C)
        with pytest.raises(TypeError):
            L.lcc_compress(None, g, C)
        with pytest.raises(TypeError):
            L.lcc_objective(None, g, 1, 2, C)


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """There is no fallback: without liblcc.so the binding raises."""
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        L.load_library(str(tmp_path / "liblcc.so"))
