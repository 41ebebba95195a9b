"""Benchmark of the LambdaCC hot path on one MI355X.

A step is one full Parallel-CC clustering (every level's Best-Moves,
compression, flatten, refinement, canonical labels and the exact objective)
of a synthetic graph already resident in HBM.  Prints ONE JSON line on stdout;
details go to stderr.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (generator kwargs, description)
    "chung_lu_4m": (dict(n=4_000_000, m=100_000_000, gamma=2.1, mixing=0.3, seed=1),
                    "Chung-Lu with planted communities, n=4M, m=100M undirected, degree exponent 2.1, "
                    "community sizes power-law in [20,5000], mixing 0.3; modularity setting k=degree, "
                    "lambda=1/(2m) as p/q"),
    "chung_lu_65m": (dict(n=65_608_366, m=1_806_067_135, gamma=2.2, mixing=0.4, seed=1),
                     "Chung-Lu with planted communities, n=65.6M, m=1.806B undirected, degree exponent 2.2, "
                     "mixing 0.4; modularity setting k=degree, lambda=1/(2m)"),
    "sbm_10k": (None, "SBM 20 blocks x 500, p_in=0.02, p_out=0.0005, k=1, lambda=1/100"),
}

# Many-job workloads: one lcc_cluster_batch call against the plain path (one
# lcc_cluster call per job, back to back), with every job's result compared.
BATCH_WORKLOADS = {
    "batch_sbm_4096": (dict(kind="sbm", jobs=4096, seed=0),
                       "4096 SBM graphs, n log-uniform in [100, 50000], blocks of ~500, average degree "
                       "uniform in [8, 40] (20% across blocks), k=1, lambda_i = p_i/1000 with p_i uniform "
                       "in [1, 500], graph seed i"),
    "sweep_knn_1m": (dict(kind="sweep", points=1_000_000, centers=1000, dim=64, knn=50, sigma=1.0, seed=1,
                          count=16),
                     "16-value lambda sweep on one cosine kNN graph: 1M points of a 1000-center 64-d Gaussian "
                     "mixture (centers N(0,I), sigma 1.0), k=50 exact neighbours symmetrized by union, weights "
                     "round(cos*2^15) as int16 (Q1.15), k_v=1; lambda = r*2^15 for r geometric in "
                     "[0.01, 0.85] as p/1000"),
}

HBM_PEAK_GBS = 8000.0

# Reports beyond the headline (see their functions): the paper's scalability
# study on rMAT graphs and its quality study against ground truth.
REPORTS = {}  # filled below: name -> (function, description)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chung_lu_65m",
                    choices=sorted(WORKLOADS) + sorted(BATCH_WORKLOADS) + ["serve_mixed"] + sorted(REPORTS))
    ap.add_argument("--slots", type=int, default=3, help="serve_mixed: concurrent batches")
    ap.add_argument("--jobs", type=int, default=0, help="batch workloads: use only the first JOBS jobs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 1 GiB device-to-device copy, a reference for HBM byte counters")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarize two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, each with "
                         "--calibrate-copy) per kernel and exit")
    args = ap.parse_args()
    if args.pmc_summary:
        return pmc_summary(*args.pmc_summary)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding this path over several "
              "GPUs is described, not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2108_01731_amd import graphgen as G
    from paper_2108_01731_amd import lcc

    dev = "cuda:0"
    if args.calibrate_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 1073741824 bytes read, 1073741824 bytes written")
        del src, dst
    if args.workload in BATCH_WORKLOADS:
        return run_batch(args, dev)
    if args.workload in REPORTS:
        return REPORTS[args.workload][0](args, dev)
    if args.workload == "serve_mixed":
        return run_serve(args, dev)
    gen_kw, desc = WORKLOADS[args.workload]
    t0 = time.time()
    if gen_kw is None:
        h = G.c1_sbm(1, device=dev)
        p, q = 1, 100
    else:
        kw = dict(gen_kw)
        h = G.chung_lu_planted(kw.pop("n"), kw.pop("m"), kw.pop("gamma"), kw.pop("mixing"), kw.pop("seed"),
                               device=dev)
        p, q = 1, int(h.arcs)  # lambda = 1/(2m)
    g = lcc.DeviceGraph.from_host(h, dev)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # the generator's scratch goes back to the device for the library
    log(f"workload {args.workload}: n={g.n} arcs={g.arcs} generated in {time.time() - t0:.1f}s")

    ctx = lcc.context(0)
    prm = lcc.Params()
    for i in range(args.warmup):
        lab, N, st = lcc.lcc_cluster(ctx, g, p, q, prm)
        log(f"warmup {i}: {st['ms_total']:.1f} ms, levels={st['levels']} clusters={st['clusters']} N={N}")
    arcs_total = 0
    Ns = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        lab, N, st = lcc.lcc_cluster(ctx, g, p, q, prm)
        arcs_total += st["arcs_scanned_total"]
        Ns.append(N)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if len(set(Ns)) != 1:
        log(f"WARNING: the timed steps disagree on the objective numerator: {Ns}")
    ms_per_step = dt * 1e3 / args.steps
    # one more step with HIP events around every launch (on the launch
    # stream): per-kernel times for the table below and the roofline
    ctx.reset_kernel_stats()
    _, N_t, st_t = lcc.lcc_cluster(ctx, g, p, q, lcc.Params(timing=1))
    log(f"instrumented step: {st_t['ms_total']:.1f} ms")
    log("levels (n, arcs, coarsening iterations, refinement iterations):")
    for lv in range(st_t["levels"]):
        log(f"  {lv:2d} n={st_t['n_level'][lv]:>10d} arcs={st_t['arcs_level'][lv]:>11d} "
            f"it={st_t['iters_coarsen'][lv]:2d} ref={st_t['iters_refine'][lv]:2d}")
    if N_t != Ns[-1]:
        log(f"WARNING: the instrumented step's objective numerator {N_t} differs from {Ns[-1]}")
    ks = ctx.kernel_stats()
    for name, v in sorted(ks.items(), key=lambda kv: -kv[1]["ms"]):
        sec = v["ms"] * 1e-3
        log(f"  {name:24s} launches={v['launches']:6d} ms/step={v['ms']:8.2f} "
            f"GB/s={(v['bytes'] / sec / 1e9) if sec > 0 else 0:8.1f} "
            f"Gitems/s={(v['items'] / sec / 1e9) if sec > 0 else 0:7.2f}")
    # the dominant kernel class among every aggregation class of Best-Moves
    # (the hub-row class bm_flat_seq* is a short sequence of launches timed as one)
    agg = {k: v for k, v in ks.items() if k.startswith(AGG_CLASSES)}
    dom_name, dom = max(agg.items(), key=lambda kv: kv[1]["ms"])
    achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, dom_name)
    agg_ms = sum(v["ms"] for v in agg.values())
    agg_arcs = sum(v["items"] for v in agg.values())
    log(f"last step: best-move {st['ms_best_move']:.1f} ms, compress {st['ms_compress']:.1f} ms, "
        f"total {st['ms_total']:.1f} ms (host wall time)")
    log(f"step: {ms_per_step:.1f} ms; levels={st['levels']} clusters={st['clusters']} "
        f"objective={N / q:.4f} (modularity-scaled {N / q / (g.arcs / 2):.6f})")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(h, p, q, prm.S)

    out = {
        "metric": "best-move edges/s",
        "value": arcs_total / dt,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n": g.n, "arcs": g.arcs,
                   "lambda": f"{p}/{q}", "S": prm.S, "num_iter": prm.num_iter, "frontier": "neighbors-of-moved",
                   "refine": True, "e2e_cluster_ms": ms_per_step,
                   "best_move_arcs_per_step": arcs_total // args.steps,
                   "best_move_kernel_edges_per_s": agg_arcs / (agg_ms * 1e-3) if agg_ms > 0 else None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_unit": "bytes/launch",
                     "algorithmic_bytes_per_launch": dom["bytes"] / dom["launches"], "kernel": dom_name,
                     "avg_launch_ms": dom["ms"] / dom["launches"], "launches": dom["launches"]},
        "cpu_baseline": cpu,
    }
    with_copy_peak(out["roofline"], dev)
    print(json.dumps(out), flush=True)


AGG_CLASSES = ("bm_aggregate", "bm_single", "bm_flat_seq")


def host_cpu():
    """(logical CPUs this process may run on, CPU model name)."""
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return ncpu, model


def cpu_baseline(h, p, q, S):
    """The oracle timed on this host on a bounded sample of the workload:
    level 0's first Best-Moves iteration (every vertex, S sub-rounds) with
    the oracle's OpenMP build on all the threads OpenMP gives it (its results
    equal the single-threaded build's), and, for reference, the
    single-threaded build deciding a prefix of the vertices."""
    import numpy as np

    import oracle as O

    hn = h.numpy()
    g_o = O.Graph(off=hn.off, col=hn.col, k=hn.k, wt=None if hn.wt is None else hn.wt.astype(np.int64))
    ncpu, model = host_cpu()
    prev = O.use_openmp(True)
    try:
        threads = O.num_threads()
        t1 = time.perf_counter()
        _, so = O.best_move(g_o, p, q, O.Params(S=S, num_iter=1))
        cdt = time.perf_counter() - t1
    finally:
        O.use_library(prev)
    # single-threaded: decisions of the lowest-numbered vertices against the
    # singleton clustering (the snapshot of level 0's first sub-round), up to
    # about 1.5e8 arcs
    deg = np.diff(hn.off)
    U = np.arange(g_o.n, dtype=np.int64)[np.cumsum(deg) <= 150_000_000].astype(np.int32)
    t2 = time.perf_counter()
    O.decide_many(g_o, p, q, np.arange(g_o.n, dtype=np.int32), U)
    sdt = time.perf_counter() - t2
    one = float(deg[U].sum()) / sdt if sdt > 0 else None
    out = {"value": so["arcs_scanned"] / cdt, "unit": "edges/s", "cores": threads, "kind": "oracle",
           "sample": f"first Best-Moves iteration of level 0 ({S} sub-rounds over all {g_o.n} vertices, "
                     f"{so['arcs_scanned']} arcs scanned) on the same graph, {cdt:.1f} s with the oracle's "
                     f"OpenMP build on {threads} threads; single-threaded build deciding {len(U)} vertices "
                     f"against the singleton clustering ({int(deg[U].sum())} arcs): {one:.3e} arcs/s",
           "single_thread_value": one, "host_cpus": ncpu, "cpu_model": model}
    log(f"cpu oracle: {out['value']:.3e} arcs/s over {cdt:.1f}s on {threads} threads "
        f"({one:.3e} arcs/s single-threaded); host: {ncpu} CPUs, {model}")
    return out


KERNEL_SOURCES = ("common.hpp", "prims.hpp", "ops.hpp", "bestmove.hip")


def kernel_source_sha1():
    """Hash of the sources the aggregation kernels are compiled from."""
    import hashlib

    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2108_01731_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, kernel_class):
    """HBM bytes per launch of the kernel class from the committed rocprofv3
    counter runs (FETCH_SIZE and WRITE_SIZE, scaled by the copy calibration),
    or None when there is none for this workload and class or the kernel
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            entries = json.load(f)
    except (OSError, ValueError):
        return None
    sha = kernel_source_sha1()
    for e in entries:
        if e.get("workload") == workload and e.get("class") == kernel_class and e.get("source_sha1") == sha:
            return e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]
    return None


def read_counter_csv(path):
    """{kernel name: [values per dispatch]} of one counter from a rocprofv3
    counter-collection CSV (column names located by keyword)."""
    import csv

    out = {}
    with open(path, newline="") as f:
        rd = csv.DictReader(f)
        cols = rd.fieldnames or []
        kcol = next(c for c in cols if "Kernel_Name" in c)
        vcol = next(c for c in cols if "Counter_Value" in c)
        for row in rd:
            out.setdefault(row[kcol], []).append(float(row[vcol]))
    return out


def pmc_summary(fetch_csv, write_csv):
    """Per-kernel HBM traffic from FETCH_SIZE and WRITE_SIZE counter runs
    (KiB per dispatch), scaled by what the same counters read for the 1 GiB
    calibration copy (the copy reads and writes 1073741824 bytes).  Prints a
    markdown table, heaviest kernels first."""
    fe = read_counter_csv(fetch_csv)
    wr = read_counter_csv(write_csv)
    copy = next(k for k in fe if "copyBuffer" in k)
    kib = (1 << 30) / 1024.0
    fs = kib / fe[copy][0]
    ws = kib / wr[copy][0]
    print(f"calibration copy: FETCH_SIZE {fe[copy][0]:.2f} KiB -> scale {fs:.4f}; "
          f"WRITE_SIZE {wr[copy][0]:.2f} KiB -> scale {ws:.4f}")
    print("| kernel | dispatches | fetch bytes / dispatch | write bytes / dispatch | total GB |")
    print("|---|---:|---:|---:|---:|")
    rows = []
    for k, v in fe.items():
        if k == copy:
            continue
        w = wr.get(k, [0.0])
        f_b = sum(v) / len(v) * 1024 * fs
        w_b = sum(w) / len(w) * 1024 * ws
        rows.append((f_b * len(v) + w_b * len(w), k, len(v), f_b, w_b))
    for tot, k, nd, f_b, w_b in sorted(rows, reverse=True)[:40]:
        print(f"| `{k[:90]}` | {nd} | {f_b:,.0f} | {w_b:,.0f} | {tot / 1e9:.3f} |")


def copy_bandwidth_gbs(dev, nbytes=1 << 30, reps=5):
    """Device-to-device copy rate (bytes read + written per second, GB/s):
    the HBM rate a plain streaming kernel reaches on this GPU, measured after
    the timed steps and reported next to the nominal peak."""
    import torch

    src = torch.empty(nbytes, dtype=torch.uint8, device=dev).fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    gbs = 2.0 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def with_copy_peak(roof, dev):
    gbs = copy_bandwidth_gbs(dev)
    log(f"device copy: {gbs:.0f} GB/s (read + write)")
    roof["copy_gbs_measured"] = gbs
    roof["frac_of_copy"] = roof["achieved"] / gbs
    if roof.get("traffic"):
        # the counter-measured bytes per launch over the same launch time:
        # the rate the kernel actually moves through the fabric
        roof["traffic_gbs"] = roof["traffic"] / (roof["avg_launch_ms"] * 1e-3) / 1e9
        roof["traffic_frac"] = roof["traffic_gbs"] / HBM_PEAK_GBS
    return roof


def dominant_kernel(ks):
    agg = {k: v for k, v in ks.items() if k.startswith(AGG_CLASSES)}
    name, d = max(agg.items(), key=lambda kv: kv[1]["ms"])
    achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": name,
            "avg_launch_ms": d["ms"] / d["launches"], "launches": d["launches"]}


def run_batch(args, dev):
    import numpy as np
    import torch

    from paper_2108_01731_amd import graphgen as G
    from paper_2108_01731_amd import lcc

    spec, desc = BATCH_WORKLOADS[args.workload]
    t0 = time.time()
    if spec["kind"] == "sbm":
        jobs = args.jobs or spec["jobs"]
        graphs, lams = G.sbm_batch(jobs, spec["seed"], device=dev)
    else:
        h = G.knn_gaussian(spec["points"], spec["centers"], spec["dim"], spec["knn"], spec["sigma"], spec["seed"],
                           device=dev)
        rs = np.geomspace(0.01, 0.85, spec["count"])
        lams = [(int(round(r * 1000)) * 32768, 1000) for r in rs]
        if args.jobs:
            lams = lams[:args.jobs]
        graphs = [h] * len(lams)
    P, start = G.pack_torch(graphs, dev)
    gp = lcc.DeviceGraph.from_host(P, dev)
    singles = [lcc.DeviceGraph.from_host(g, dev) for g in graphs]
    torch.cuda.synchronize()
    J = len(graphs)
    log(f"workload {args.workload}: {J} jobs, n={gp.n} arcs={gp.arcs} generated in {time.time() - t0:.1f}s")
    ctx = lcc.context(0)
    prm = lcc.Params()
    sweep = spec["kind"] == "sweep"

    def run_one(params):
        # a sweep clusters the one graph under every lambda in one call; a
        # batch takes the jobs packed block-diagonally
        if sweep:
            return lcc.lcc_sweep(ctx, singles[0], lams, params)
        return lcc.lcc_cluster_batch(ctx, gp, start, lams, params)

    for i in range(args.warmup):
        _, _, st = run_one(prm)
        log(f"warmup {i}: {st['ms_total']:.1f} ms, levels={st['levels']}")
    for j in range(min(J, 4)):
        lcc.lcc_cluster(ctx, singles[j], *lams[j], prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        lab_b, jobs_b, st = run_one(prm)
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t0) / args.steps
    log(f"{'sweep' if sweep else 'batched'}: {dt_b * 1e3:.1f} ms per call ({J} jobs, levels={st['levels']})")
    dt_pk = None
    if sweep:
        # the same jobs as a plain packed batch (no shared rows), for reference
        lcc.lcc_cluster_batch(ctx, gp, start, lams, prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            lab_pk, jobs_pk, _ = lcc.lcc_cluster_batch(ctx, gp, start, lams, prm)
        torch.cuda.synchronize()
        dt_pk = (time.perf_counter() - t0) / args.steps
        log(f"packed batch of the same jobs: {dt_pk * 1e3:.1f} ms; sweep speedup {dt_pk / dt_b:.2f}x")
        lab_b = lab_b.reshape(-1)
    # the plain path: one job at a time
    labs_p, Ns_p = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(J):
        lab, N, _ = lcc.lcc_cluster(ctx, singles[j], *lams[j], prm)
        labs_p.append(lab)
        Ns_p.append(N)
    torch.cuda.synchronize()
    dt_p = time.perf_counter() - t0
    log(f"plain: {dt_p * 1e3:.1f} ms for {J} jobs one at a time; speedup {dt_p / dt_b:.2f}x")
    same = all(torch.equal(lab_b[int(start[j]):int(start[j + 1])], labs_p[j]) and jobs_b[j]["N"] == Ns_p[j]
               for j in range(J))
    if sweep:
        same = same and all(torch.equal(lab_pk[int(start[j]):int(start[j + 1])], labs_p[j]) and
                            jobs_pk[j]["N"] == Ns_p[j] for j in range(J))
    log(f"every job identical to its plain run: {same}")
    # kernel classes of one more run, timed per launch
    ctx.reset_kernel_stats()
    run_one(lcc.Params(timing=1))
    ks = ctx.kernel_stats()
    for name, v in sorted(ks.items(), key=lambda kv: -kv[1]["ms"])[:12]:
        sec = v["ms"] * 1e-3
        log(f"  {name:24s} launches={v['launches']:6d} ms={v['ms']:8.2f} "
            f"GB/s={(v['bytes'] / sec / 1e9) if sec > 0 else 0:8.1f} "
            f"Gitems/s={(v['items'] / sec / 1e9) if sec > 0 else 0:7.2f}")
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O

        t1 = time.perf_counter()
        arcs_o, done = 0, 0
        for j in range(J):
            hn = G.HostGraph(graphs[j].off, graphs[j].col, graphs[j].k, graphs[j].wt, None, None,
                             graphs[j].wt_kind).numpy()
            g_o = O.Graph(off=hn.off, col=hn.col, k=hn.k, wt=None if hn.wt is None else hn.wt.astype(np.int64))
            O.cluster(g_o, *lams[j], O.Params())
            arcs_o += g_o.arcs
            done += 1
            if time.perf_counter() - t1 > 15.0:
                break
        cdt = time.perf_counter() - t1
        cpu = {"value": arcs_o / cdt, "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": f"full clustering of the first {done} of the {J} jobs ({arcs_o} arcs), "
                         f"{cdt:.1f} s single-threaded"}
        log(f"cpu oracle: {cpu['value']:.3e} arcs/s over {cdt:.1f}s ({done} jobs)")
    out = {
        "metric": "batched clustering edges/s",
        "value": gp.arcs / dt_b,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt_b * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "jobs": J, "n_total": gp.n,
                   "arcs_total": gp.arcs, "entry": "lcc_sweep" if sweep else "lcc_cluster_batch",
                   "batched_ms": dt_b * 1e3, "plain_ms": dt_p * 1e3,
                   "speedup_vs_plain": dt_p / dt_b, "jobs_per_s_batched": J / dt_b,
                   "jobs_per_s_plain": J / dt_p, "identical_results": same,
                   **({"packed_batch_ms": dt_pk * 1e3, "speedup_vs_packed_batch": dt_pk / dt_b} if sweep else {})},
        "roofline": with_copy_peak(dominant_kernel(ks), dev),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if not same:
        sys.exit(1)


def run_serve(args, dev):
    """Seeded Poisson stream of mixed requests (SBM, Chung-Lu, Q1.15 kNN; m
    log-uniform in [1k, 5M] edges; lambda per request), replayed through the
    plain path (one request at a time) and the continuous-batching server."""
    import numpy as np
    import torch

    from paper_2108_01731_amd import serve as V

    count = args.jobs or 400
    t0 = time.time()
    trace = V.make_trace(count, qps=1.0, seed=0, mmin=1000, mmax=5_000_000, device=dev)
    arcs = sum(r.graph.arcs for r in trace)
    log(f"serve_mixed: {count} requests, {arcs} arcs in total, generated in {time.time() - t0:.1f}s")
    plain = V.Server(0, plain=True)
    srv = V.Server(0, slots=args.slots, hbm_budget=96 << 30)
    burst = V.retime(trace, 0.0)  # every request at t = 0: throughput at saturation
    # steady state: one untimed pass of the same burst through each path, so
    # the library buffers of every slot have reached their working size (a
    # buffer that grows inside the timed pass frees and reallocates, which
    # stalls the whole device)
    plain.serve(burst)
    srv.serve(burst)
    sp = plain.serve(burst)
    ss = srv.serve(burst)
    P, S = sp.summary(), ss.summary()
    same = all(np.array_equal(a.labels, b.labels) and a.N == b.N for a, b in zip(sp.done, ss.done))
    log(f"saturation: plain {P['throughput_rps']:.1f} req/s, served {S['throughput_rps']:.1f} req/s "
        f"({S['batches']} batches); identical results: {same}")
    qps = 0.7 * P["throughput_rps"]
    lp = plain.serve(V.retime(trace, qps, seed=1)).summary()
    ls = srv.serve(V.retime(trace, qps, seed=1)).summary()
    log(f"at {qps:.1f} req/s: plain p50 {lp['p50_ms']:.1f} ms p99 {lp['p99_ms']:.1f} ms; "
        f"served p50 {ls['p50_ms']:.1f} ms p99 {ls['p99_ms']:.1f} ms")
    qps_s = 0.7 * S["throughput_rps"]
    lh = srv.serve(V.retime(trace, qps_s, seed=2)).summary()
    log(f"at {qps_s:.1f} req/s: served p50 {lh['p50_ms']:.1f} ms p99 {lh['p99_ms']:.1f} ms")
    plain.close()
    srv.close()
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O

        t1 = time.perf_counter()
        done, a_o = 0, 0
        for r in trace:
            h = r.graph.numpy()
            g_o = O.Graph(off=h.off, col=h.col, k=h.k, wt=None if h.wt is None else h.wt.astype(np.int64))
            O.cluster(g_o, r.p, r.q, O.Params())
            done += 1
            a_o += h.arcs
            if time.perf_counter() - t1 > 15.0:
                break
        cdt = time.perf_counter() - t1
        cpu = {"value": done / cdt, "unit": "requests/s", "cores": 1, "kind": "oracle",
               "sample": f"full clustering of the first {done} requests of the trace ({a_o} arcs), "
                         f"{cdt:.1f} s single-threaded"}
    out = {
        "metric": "served requests/s",
        "value": S["throughput_rps"],
        "unit": "requests/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": S["makespan_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "serve_mixed", "requests": count, "arcs_total": arcs, "slots": args.slots,
                   "hbm_budget_bytes": 96 << 30, "plain_rps": P["throughput_rps"],
                   "speedup_vs_plain": S["throughput_rps"] / P["throughput_rps"],
                   "saturation": {"plain": P, "served": S},
                   "latency_at_qps": {"qps": qps, "plain": lp, "served": ls},
                   "latency_at_served_qps": {"qps": qps_s, "served": lh},
                   "identical_results": same},
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if not same:
        sys.exit(1)


def sweep_labels(ctx, g, lams, prm):
    """Labels of g under every (p, q) of lams, through lcc_sweep calls of at
    most 16 resolutions each; returns (labels list, per-lambda job dicts)."""
    from paper_2108_01731_amd import lcc

    labs, jobs = [], []
    for a in range(0, len(lams), lcc.SWEEP_MAX):
        lab, jb, _ = lcc.lcc_sweep(ctx, g, lams[a:a + lcc.SWEEP_MAX], prm)
        labs += list(lab.cpu().numpy())
        jobs += jb
    return labs, jobs


def run_quality(args, dev):
    """Average precision / recall against the planted communities of a
    Chung-Lu graph (1M vertices, 10M edges, degree exponent 2.1, mixing 0.3),
    the synthetic counterpart of the paper's quality curves (Sec. 4.3): the
    correlation-clustering objective (k = 1) over lambda in {0.01 x : x = 1..99}
    and modularity (k = degree) over gamma in {0.02 * 1.2^x : x = 1..99}
    (lambda = gamma / 2m), keeping the gamma values within the int64 bounds.
    Each community is matched to the cluster sharing most of its vertices;
    the 5000 largest communities are scored."""
    import numpy as np
    import torch

    from paper_2108_01731_amd import graphgen as G
    from paper_2108_01731_amd import lcc
    from paper_2108_01731_amd import quality as Q

    t0 = time.time()
    h, comm = G.chung_lu_planted(1_000_000, 10_000_000, 2.1, 0.3, seed=1, device=dev, k_is_degree=False,
                                 return_communities=True)
    g_cc = lcc.DeviceGraph.from_host(h, dev)
    deg = (g_cc.off[1:] - g_cc.off[:-1]).contiguous()
    g_mod = lcc.DeviceGraph(off=g_cc.off, col=g_cc.col, k=deg)
    m2 = g_cc.arcs
    log(f"quality workload: n={g_cc.n} arcs={m2} communities={len(np.unique(comm))} "
        f"generated in {time.time() - t0:.1f}s")
    ctx = lcc.context(0)
    prm = lcc.Params()
    lam_cc = [(x, 100) for x in range(1, 100)]
    # modularity: lambda = gamma / (2m) = (gamma * 1000) / (2m * 1000), within
    # q * sum|w| <= 2^63 - 1 and p * floor((sum k)^2 / 4) <= 2^63 - 1
    lim = (1 << 63) - 1
    q_mod = m2 * 1000
    lam_mod, gam = [], []
    for x in range(1, 100):
        gmm = 0.02 * 1.2 ** x
        pm = max(1, int(round(gmm * 1000)))
        if q_mod * (m2 // 2) <= lim and pm * ((m2 * m2) // 4) <= lim:
            lam_mod.append((pm, q_mod))
            gam.append(gmm)
    curves = {}
    for name, g, lams, xs in (("cc", g_cc, lam_cc, [p / 100 for p, _ in lam_cc]), ("mod", g_mod, lam_mod, gam)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        labs, jobs = sweep_labels(ctx, g, lams, prm)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        rows = []
        for x, lab, jb in zip(xs, labs, jobs):
            pr, rc, nc = Q.precision_recall(lab, comm, top=5000)
            rows.append({"param": x, "precision": pr, "recall": rc, "clusters": jb["clusters"]})
        curves[name] = {"rows": rows, "seconds": dt}
        log(f"{name}: {len(lams)} resolutions in {dt:.2f}s")
        for r in rows[:: max(1, len(rows) // 12)]:
            log(f"  {'lambda' if name == 'cc' else 'gamma'}={r['param']:<10.4g} precision={r['precision']:.3f} "
                f"recall={r['recall']:.3f} clusters={r['clusters']}")

    def f1(r):
        s = r["precision"] + r["recall"]
        return 2 * r["precision"] * r["recall"] / s if s > 0 else 0.0

    best = max(curves["cc"]["rows"], key=f1)
    out = {"metric": "average precision / recall vs planted communities", "value": f1(best),
           "unit": "F1 of the best lambda", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "dtype": "int64", "config": {"workload": args.workload, "description": REPORTS[args.workload][1],
                                        "n": g_cc.n, "arcs": m2, "best_cc": best, "curves": curves}}
    print(json.dumps(out), flush=True)


def run_rmat(args, dev):
    """The paper's scalability study (Sec. 4.2) on one GPU: rMAT graphs
    (a = 0.5, b = c = 0.1, d = 0.3) with m = 5n, 50n and n^1.5 edge draws,
    clustered with the correlation objective (k = 1) at lambda = 0.01 and
    0.85; end-to-end time of lcc_cluster against the number of edges."""
    import torch

    from paper_2108_01731_amd import graphgen as G
    from paper_2108_01731_amd import lcc

    ctx = lcc.context(0)
    prm = lcc.Params()
    sizes = [(16, "5n"), (16, "50n"), (16, "n^1.5"), (18, "5n"), (18, "50n"), (18, "n^1.5"), (20, "5n"),
             (20, "50n"), (22, "5n"), (22, "50n"), (20, "n^1.5")]
    rows = []
    for scale, kind in sizes:
        n = 1 << scale
        m = 5 * n if kind == "5n" else 50 * n if kind == "50n" else int(round(n ** 1.5))
        t0 = time.time()
        h = G.rmat(scale, m, seed=scale, device=dev)
        g = lcc.DeviceGraph.from_host(h, dev)
        del h
        gen_s = time.time() - t0
        for p, q in ((1, 100), (85, 100)):
            lcc.lcc_cluster(ctx, g, p, q, prm)  # warm
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            reps = 3
            for _ in range(reps):
                _, N, st = lcc.lcc_cluster(ctx, g, p, q, prm)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t1) * 1e3 / reps
            rows.append({"scale": scale, "m_rule": kind, "n": g.n, "edges": g.arcs // 2, "lambda": p / q,
                         "ms": ms, "levels": st["levels"], "clusters": st["clusters"],
                         "best_move_arcs": st["arcs_scanned_total"]})
            log(f"rmat scale={scale} m={kind:6s} edges={g.arcs // 2:>11d} lambda={p / q:.2f}: {ms:9.2f} ms "
                f"levels={st['levels']} clusters={st['clusters']} (generated in {gen_s:.1f}s)")
        del g
        torch.cuda.empty_cache()
    big = max(rows, key=lambda r: (r["edges"], -r["lambda"]))
    out = {"metric": "end-to-end cluster time vs edges (rMAT)", "value": big["edges"] / (big["ms"] * 1e-3),
           "unit": "edges/s (largest graph, lambda 0.01)", "n_gpus": 1, "higher_is_better": True,
           "data": "synthetic", "dtype": "int64",
           "config": {"workload": args.workload, "description": REPORTS[args.workload][1], "rows": rows}}
    print(json.dumps(out), flush=True)


def run_ablation(args, dev):
    """The S / frontier / refine ablation (the deterministic analog of the
    paper's tuning study, Sec. 4.1): every combination of S in {1, 2, 4, 8},
    frontier in {all vertices, neighbors of movers, neighbors of clusters}
    and refinement on/off, on the 10k-vertex SBM (lambda = 1/100) and the
    4M-vertex Chung-Lu modularity graph; end-to-end time, objective,
    hierarchy depth and Best-Moves arcs per configuration."""
    import torch

    from paper_2108_01731_amd import graphgen as G
    from paper_2108_01731_amd import lcc

    ctx = lcc.context(0)
    graphs = []
    h = G.c1_sbm(1, device=dev)
    graphs.append(("sbm_10k", lcc.DeviceGraph.from_host(h, dev), 1, 100))
    h = G.chung_lu_planted(4_000_000, 100_000_000, 2.1, 0.3, seed=1, device=dev)
    graphs.append(("chung_lu_4m", lcc.DeviceGraph.from_host(h, dev), 1, int(h.arcs)))
    del h
    names = {0: "all", 1: "nbr_movers", 2: "nbr_clusters"}
    rows = []
    for gname, g, p, q in graphs:
        for S in (1, 2, 4, 8):
            for fr in (0, 1, 2):
                for rf in (0, 1):
                    prm = lcc.Params(S=S, frontier=fr, refine=rf)
                    lcc.lcc_cluster(ctx, g, p, q, prm)  # warm
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, N, st = lcc.lcc_cluster(ctx, g, p, q, prm)
                    torch.cuda.synchronize()
                    ms = (time.perf_counter() - t0) * 1e3
                    rows.append({"graph": gname, "S": S, "frontier": names[fr], "refine": rf, "ms": ms,
                                 "objective": N / q, "levels": st["levels"], "top_moved": st["top_moved"],
                                 "clusters": st["clusters"], "best_move_arcs": st["arcs_scanned_total"]})
                    log(f"{gname:12s} S={S} frontier={names[fr]:12s} refine={rf}: {ms:8.1f} ms "
                        f"objective={N / q:.6g} levels={st['levels']:2d} clusters={st['clusters']} "
                        f"arcs={st['arcs_scanned_total']}")
    ref = [r for r in rows if r["graph"] == "chung_lu_4m" and r["S"] == 4 and r["frontier"] == "nbr_movers"
           and r["refine"] == 1][0]
    out = {"metric": "ablation: time and objective per (S, frontier, refine)", "value": ref["ms"],
           "unit": "ms (4M-vertex graph, default settings)", "n_gpus": 1, "higher_is_better": False,
           "data": "synthetic", "dtype": "int64",
           "config": {"workload": args.workload, "description": REPORTS[args.workload][1], "rows": rows}}
    print(json.dumps(out), flush=True)


def run_async(args, dev):
    """The asynchronous mode against the deterministic schedule (the paper
    reports its asynchronous setting as the better one, Sec. 3.2.1, 4.1):
    the 4M-vertex Chung-Lu modularity graph and the 65.6M-vertex one, five
    seeds each, end-to-end time and objective (modularity-scaled) of the
    default deterministic schedule (S = 4) and of asynchronous moves (S = 1,
    the paper's setting, and S = 4).
    The asynchronous results differ from run to run; the report gives their
    distribution."""
    import numpy as np
    import torch

    from paper_2108_01731_amd import graphgen as G
    from paper_2108_01731_amd import lcc

    ctx = lcc.context(0)
    rows = []
    for gname, kw in (("chung_lu_4m", WORKLOADS["chung_lu_4m"][0]), ("chung_lu_65m", WORKLOADS["chung_lu_65m"][0])):
        kw = dict(kw)
        h = G.chung_lu_planted(kw.pop("n"), kw.pop("m"), kw.pop("gamma"), kw.pop("mixing"), kw.pop("seed"),
                               device=dev)
        g = lcc.DeviceGraph.from_host(h, dev)
        p, q = 1, int(h.arcs)
        del h
        torch.cuda.empty_cache()
        for mode, base in (("sync", dict()), ("async", dict(S=1, async_moves=1)),
                           ("async_s4", dict(S=4, async_moves=1))):
            lcc.lcc_cluster(ctx, g, p, q, lcc.Params(**base))  # warm
            for seed in range(1, 6):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, N, st = lcc.lcc_cluster(ctx, g, p, q, lcc.Params(seed=seed, **base))
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3
                mod = N / q / (g.arcs / 2)
                rows.append({"graph": gname, "mode": mode, "seed": seed, "ms": ms, "modularity_scaled": mod,
                             "levels": st["levels"], "clusters": st["clusters"]})
                log(f"{gname:12s} {mode:5s} seed={seed}: {ms:8.1f} ms objective/m={mod:.6f} "
                    f"levels={st['levels']} clusters={st['clusters']}")
        del g
        torch.cuda.empty_cache()
    summ = {}
    for gname in ("chung_lu_4m", "chung_lu_65m"):
        for mode in ("sync", "async", "async_s4"):
            r = [x for x in rows if x["graph"] == gname and x["mode"] == mode]
            summ[f"{gname}/{mode}"] = {"ms_mean": float(np.mean([x["ms"] for x in r])),
                                       "objective_mean": float(np.mean([x["modularity_scaled"] for x in r])),
                                       "objective_min": float(min(x["modularity_scaled"] for x in r)),
                                       "objective_max": float(max(x["modularity_scaled"] for x in r))}
            log(f"{gname}/{mode}: {summ[f'{gname}/{mode}']}")
    big = summ["chung_lu_65m/async"]
    out = {"metric": "asynchronous vs deterministic schedule: time and objective over seeds",
           "value": big["ms_mean"], "unit": "ms (65.6M-vertex graph, asynchronous, mean of 5 seeds)",
           "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "int64",
           "config": {"workload": args.workload, "description": REPORTS[args.workload][1], "summary": summ,
                      "rows": rows}}
    print(json.dumps(out), flush=True)


REPORTS.update({
    "async_vs_sync": (run_async, "asynchronous moves (S=1 and S=4) vs the deterministic schedule (S=4) on the 4M "
                                 "and 65.6M-vertex Chung-Lu modularity graphs, 5 seeds each"),
    "ablation": (run_ablation, "S in {1,2,4,8} x frontier {all, neighbors of movers, neighbors of clusters} x "
                               "refine {0,1} on the 10k SBM and the 4M Chung-Lu modularity graph"),
    "quality_chung_lu_1m": (run_quality, "average precision/recall vs planted communities on a 1M-vertex, 10M-edge "
                                         "Chung-Lu graph (mixing 0.3), lambda grid 0.01..0.99 (k=1) and gamma "
                                         "grid 0.02*1.2^x (k=degree)"),
    "rmat_scaling": (run_rmat, "rMAT a=0.5 b=c=0.1 d=0.3, n = 2^16..2^22, m = 5n, 50n, n^1.5 edge draws; "
                               "k=1, lambda 0.01 and 0.85; end-to-end lcc_cluster time vs edges"),
})


if __name__ == "__main__":
    main()
