#!/usr/bin/env python3
"""Benchmark: Dynamic Frontier PageRank updates on one MI355X.

Workload (default): R-MAT scale 22 (4,194,304 vertices), edge factor 16,
a=0.57 b=0.19 c=0.19 d=0.05, duplicates removed, a self-loop on every vertex,
FP64 ranks, alpha 0.85, tol 1e-10 (L-inf), frontier tolerance 1e-13.  A
sequence of uniformly random batches (80% insertions of new pairs, 20%
deletions of existing edges) cycling through 1e-7, 1e-5 and 1e-3 of |E|,
every batch distinct, with the ranks carried from one batch to the next.

One step = apply the batch to both device CSRs + one Dynamic Frontier
update (initial marking, iterations to convergence), with the batch already
in device memory.  value = in-edges gathered by all timed updates divided by
the wall time of the timed steps (GTEPS).  Latency p50/p99 are over the
timed steps.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS (edges/s) + update latency p50/p99 per batch; FP32 vs FP64 at 1e-9 L∞"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_iter_traffic.json")
# sources whose text fixes the iteration kernel's code, launch shape and
# the vertex numbering it runs on (all of which move its memory traffic)
KERNEL_SRC = [os.path.join(ROOT, "paper_2401_03256_amd", "csrc", f)
              for f in ("iter.h", "common.h", "rank.hip", "graph.hip")]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def code_text(src):
    """Source text without comments and with whitespace collapsed: edits to
    comments do not change the kernel the counters were taken on."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_hash():
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, encoding="utf-8") as f:
            h.update(code_text(f.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per iteration (launches that ran an iteration; those queued
    after a call converged return at once and move nothing) from committed
    rocprofv3 counter runs, if they were taken on the current kernel source
    for this workload."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash() or t.get("workload") != workload:
        return None
    return t.get("bytes_per_iteration")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=15)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--fracs", default="1e-7,1e-5,1e-3")
    ap.add_argument("--frontier-tol", type=float, default=1e-13)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparators", action="store_true",
                    help="skip the untimed comparator calls (for profiler runs)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the R-MAT scale 22 line, without the precision-form, grid "
                         "and serving workloads that follow it by default")
    ap.add_argument("--permute", action="store_true",
                    help="relabel the R-MAT vertices by a seeded permutation")
    ap.add_argument("--workload", default="rmat22",
                    choices=["rmat22", "grid", "fp32", "serve", "sweep"],
                    help="rmat22: the headline line; grid: 4096x4096 grid, uniform and "
                         "localised batches; fp32: R-MAT scale 24, FP32 storage form vs FP64; "
                         "serve: 12 resident R-MAT graphs, Poisson update stream; sweep: "
                         "frontier tolerance and insertion/deletion mixes on R-MAT scale 22")
    ap.add_argument("--serve", action="store_true", help="same as --workload serve")
    ap.add_argument("--serve-requests", type=int, default=96)
    ap.add_argument("--serve-load", type=float, default=0.9,
                    help="arrival rate as a fraction of one-at-a-time FP64 capacity")
    ap.add_argument("--serve-scales", default="16,18,20,22")
    ap.add_argument("--serve-slots", type=int, default=8)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs the whole update on a "
              "single MI355X; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py is single-process", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2401_03256_amd import dfpr, synth

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    dfpr.lib()
    if args.serve or args.workload == "serve":
        print(json.dumps(serve_bench(args, dfpr, synth)), flush=True)
        return
    if args.workload == "grid":
        print(json.dumps(grid_bench(args, dfpr, synth)), flush=True)
        return
    if args.workload == "fp32":
        print(json.dumps(fp32_bench(args, dfpr, synth)), flush=True)
        return
    if args.workload == "sweep":
        sweep_bench(args, dfpr, synth)
        return
    out = headline_bench(args, dfpr, synth)
    if not args.headline_only:
        # the metric's other parts, on their own workloads (not timed into
        # `value`): FP32 vs FP64 on R-MAT scale 24, the high-diameter grid,
        # and the serving form
        t = time.time()
        out["precision_form"] = fp32_bench(args, dfpr, synth, per_size=2, oracle_check=True)
        out["grid"] = grid_bench(args, dfpr, synth, per_kind=3, tol_sweep=False)
        out["serving"] = serve_bench(args, dfpr, synth, nreq=min(args.serve_requests, 48))
        log(f"side workloads: {time.time() - t:.1f}s")
    print(json.dumps(out), flush=True)


def headline_bench(args, dfpr, synth):
    """R-MAT scale 22 Dynamic Frontier steps (the `value`), the kernel's
    roofline, comparators and the CPU oracle baseline."""
    import torch
    fracs = [float(x) for x in args.fracs.split(",")]
    workload = f"rmat{args.scale}_ef{args.edge_factor}{'_perm' if args.permute else ''}_df_fp64"

    t = time.time()
    n, src, dst = synth.rmat(args.scale, args.edge_factor, seed=1, permute=args.permute)
    log(f"R-MAT scale {args.scale}: n={n} edges={src.size} ({time.time() - t:.1f}s)")
    t = time.time()
    g = dfpr.Graph(n, src, dst)
    g.use_torch_stream()
    m = g.m
    log(f"loaded on GPU: m={m} incl. self-loops ({time.time() - t:.1f}s)")

    total = args.warmup + args.steps
    counts = [synth.batch_counts(fracs[i % len(fracs)], m) for i in range(total)]
    counts += [synth.batch_counts(f, m) for f in fracs]   # comparator batches
    seq = synth.batch_sequence(src, dst, n, counts, seed=2)
    dev = [[torch.from_numpy(np.ascontiguousarray(x)).cuda()
            for x in (b.del_src, b.del_dst, b.ins_src, b.ins_dst)] for b in seq]
    torch.cuda.synchronize()
    p = dfpr.params(frontier_tol=args.frontier_tol)
    p32 = dfpr.params(frontier_tol=args.frontier_tol, precision=dfpr.FP32_KAHAN)
    pa = dfpr.params(frontier_tol=args.frontier_tol, mode=dfpr.ASYNC)

    t = time.time()
    R0, st0 = g.static(p)
    log(f"static: {st0.iterations} it, {st0.ms_device:.2f} ms device "
        f"({st0.edges_processed / st0.ms_device / 1e6:.1f} GTEPS)")

    def step(i):
        g.apply_batch_device(*dev[i])
        return g.dynamic_frontier_device(*dev[i], p=p)

    # warmup steps; each is also run in the FP32 form from the same previous
    # ranks (untimed), so that both can be compared with the oracle below
    warm_ranks, warm32 = [], []
    for i in range(args.warmup):
        R_prev = g.ranks()
        st = step(i)
        warm_ranks.append(g.ranks())
        g.set_ranks(R_prev)
        s32 = g.dynamic_frontier_device(*dev[i], p=p32)
        warm32.append((g.ranks(), s32.refine_sweeps))
        g.set_ranks(warm_ranks[-1])
        log(f"warmup {i}: batch {seq[i].size}, {st.iterations} it, "
            f"affected {st.affected_final}, {st.ms_device:.2f} ms; FP32 form {s32.ms_device:.2f} ms")

    g.profile_reset(True)
    lat, edges, per = [], 0, {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.warmup, total):
        ts = time.perf_counter()
        st = step(i)
        dt = time.perf_counter() - ts
        lat.append(dt * 1e3)
        edges += st.edges_processed
        f = fracs[i % len(fracs)]
        per.setdefault(f, []).append((dt * 1e3, st.iterations, st.affected_final,
                                      st.edges_processed, st.ms_apply, st.ms_mark, st.ms_iter))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.profile()
    g.profile_reset(False)
    elapsed = t1 - t0
    value = edges / elapsed / 1e9
    log(f"timed: {args.steps} steps in {elapsed * 1e3:.1f} ms, {value:.2f} GTEPS")

    # comparators (not timed): for one more batch of each size, Dynamic
    # Frontier, Naive-dynamic and Static on the same updated graph, the two
    # dynamic methods starting from the same previous ranks
    comparators = {"by_frac": {}}
    for j, f in enumerate([] if args.no_comparators else fracs):
        i = total + j
        R_prev = g.ranks()
        g.apply_batch_device(*dev[i])
        st_df = g.dynamic_frontier_device(*dev[i], p=p)
        R_df = g.ranks()
        g.set_ranks(R_prev)
        st_32 = g.dynamic_frontier_device(*dev[i], p=p32)
        R_32 = g.ranks()
        g.set_ranks(R_prev)
        _, st_nv = g.naive_dynamic(None, p=p, out=False)
        R_nv = g.ranks()
        g.set_ranks(R_prev)
        _, st_dt = g.dynamic_traversal(seq[i], p=p, out=False)
        R_dt = g.ranks()
        g.set_ranks(R_prev)
        st_as = g.dynamic_frontier_device(*dev[i], p=pa)
        R_as = g.ranks()
        _, st_st = g.static(p, out=False)
        R_st = g.ranks()
        comparators["by_frac"][str(f)] = {
            "df_ms": round(st_df.ms_device, 3), "df_iterations": st_df.iterations,
            "df_affected": st_df.affected_final,
            "naive_ms": round(st_nv.ms_device, 3), "naive_iterations": st_nv.iterations,
            "static_ms": round(st_st.ms_device, 3), "static_iterations": st_st.iterations,
            "speedup_vs_static": round(st_st.ms_device / st_df.ms_device, 2),
            "speedup_vs_naive": round(st_nv.ms_device / st_df.ms_device, 2),
            "dt_ms": round(st_dt.ms_device, 3), "dt_iterations": st_dt.iterations,
            "dt_affected": st_dt.affected_final,
            "speedup_vs_dt": round(st_dt.ms_device / st_df.ms_device, 2),
            "linf_dt_vs_static": float(np.max(np.abs(R_dt - R_st))),
            "df_async_ms": round(st_as.ms_device, 3), "df_async_iterations": st_as.iterations,
            "linf_df_async_vs_static": float(np.max(np.abs(R_as - R_st))),
            "fp32_form_ms": round(st_32.ms_device, 3),
            "fp32_form_iterations": st_32.iterations,
            "fp32_form_refine_sweeps": st_32.refine_sweeps,
            "fp32_form_linf_vs_fp64_df": float(np.max(np.abs(R_32 - R_df))),
            "fp32_form_l1_vs_fp64_df": float(np.sum(np.abs(R_32 - R_df))),
            "linf_df_vs_static": float(np.max(np.abs(R_df - R_st))),
            "linf_naive_vs_static": float(np.max(np.abs(R_nv - R_st))),
        }
        g.set_ranks(R_df)
        log(f"comparators {f}: DF {st_df.ms_device:.2f} ms ({st_df.iterations} it), async DF "
            f"{st_as.ms_device:.2f} ms ({st_as.iterations} it), naive {st_nv.ms_device:.2f} ms, "
            f"DT {st_dt.ms_device:.2f} ms, static {st_st.ms_device:.2f} ms")
    comparators["df_ms_mean_by_frac_timed"] = {
        str(f): round(float(np.mean([x[0] for x in v])), 3) for f, v in sorted(per.items())}

    achieved = prof.bytes / (prof.ms / 1e3) / 1e9 if prof.ms > 0 else 0.0
    iters_timed = int(sum(x[1] for v in per.values() for x in v))
    tb = measured_traffic(workload)
    copy_gbs = copy_bandwidth(torch)
    log(f"achievable copy bandwidth {copy_gbs:.0f} GB/s")
    roofline = {
        # the Dynamic Frontier iteration: k_iter on the class lists and the
        # first iterations on the full schedule, k_iter_wide<true, false, 8, 6144>
        # on the full schedule once the host has seen it (one launch per
        # iteration either way)
        "bound": "hbm",
        "kernel": "k_iter<true, false> + k_iter_wide<true, false, 8, 6144> "
                  "(FP64 Dynamic Frontier iteration: pull + Delta r + L-inf + expand)",
        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        # measured HBM bytes (committed counter runs on these sources) over
        # the same kernel time as `achieved`
        "traffic": (None if tb is None or prof.ms <= 0 else
                    round(tb * iters_timed / (prof.ms / 1e3) / 1e9, 1)),
        "traffic_bytes_per_launch": (None if tb is None else
                                     round(tb * iters_timed / max(prof.launches, 1), 1)),
        # every launch of the kernel, as rocprofv3 counts them: the
        # iterations plus the few launches queued after a call converged,
        # which return at once
        "launches": prof.launches, "avg_launch_us": round(prof.ms * 1e3 / max(prof.launches, 1), 2),
        # the iterations alone (the returning launches cost ~4 us each)
        "iterations": iters_timed,
        "avg_iteration_us": round(prof.ms * 1e3 / max(iters_timed, 1), 2),
        "algorithmic_bytes_per_launch": round(prof.bytes / max(prof.launches, 1), 1),
        "kernel_gteps": round(prof.edges / prof.ms / 1e6, 2) if prof.ms > 0 else None,
        "achievable_copy_GBps": round(copy_gbs, 1),
        "frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs > 0 else None,
    }

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(n, src, dst, seq, R0, warm_ranks, warm32, args, log)
    g.close()
    del dev
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "graph": f"R-MAT scale {args.scale}", "n": n, "m": m,
                   "vertex_ids": "seeded permutation" if args.permute else "as generated",
                   "edge_factor": args.edge_factor, "rmat_abcd": [0.57, 0.19, 0.19, 0.05],
                   "batch_fracs": fracs, "insert_frac": 0.8, "alpha": 0.85, "tol": 1e-10,
                   "frontier_tol": args.frontier_tol, "parallelism": "single GPU"},
        "latency_ms": {"p50": round(pct(lat, 50), 3), "p99": round(pct(lat, 99), 3),
                       "by_frac_p50": {str(f): round(pct([x[0] for x in v], 50), 3)
                                       for f, v in sorted(per.items())},
                       # device time per step by phase (HIP events): batch
                       # applier, set-up and initial marking, iterations
                       "device_split_mean_by_frac": {
                           str(f): {k: round(float(np.mean([x[j] for x in v])), 3)
                                    for k, j in (("apply", 4), ("mark", 5), ("iterate", 6))}
                           for f, v in sorted(per.items())}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "comparators": comparators,
    }
    return out


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Read + write bandwidth of a plain device copy of `nbytes` (torch's
    copy kernel), best of `reps`: the achievable streaming rate beside the
    8 TB/s peak."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    best = 0.0
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = max(best, 2 * nbytes / (e0.elapsed_time(e1) / 1e3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return best


def current_edges(g):
    """Non-self-loop edges of a library graph (caller ids), for drawing a
    batch against its current edge set."""
    off, idx = g.csr(True)
    src = np.repeat(np.arange(g.n, dtype=np.int32), np.diff(off))
    keep = src != idx
    return src[keep], idx[keep].astype(np.int32)


def cpu_model():
    """Host CPU model name (Linux), or the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(n, src, dst, seq, R0, warm_ranks, warm32, args, log):
    """The oracle (plain C, OpenMP) on the host cores, timed over marking +
    iterations (Section 5.1.5 excludes the graph update), on the first
    batches of the same sequence until about --cpu-seconds have been spent;
    the first batch is also timed on one thread.  Also reports how far the
    GPU's FP64 ranks and its FP32 form for those batches are from the
    oracle's (each from the same previous ranks)."""
    import oracle
    oracle.build(force=False)
    t = time.time()
    o = oracle.OracleGraph(n, src, dst)
    cores = oracle.num_threads()
    log(f"oracle loaded ({time.time() - t:.1f}s, {cores} threads)")
    R = R0
    spent, edges, used = 0.0, 0, 0
    err64 = {"linf": 0.0, "l1": 0.0}
    err32 = {"linf": 0.0, "l1": 0.0}
    one = None
    for i, b in enumerate(seq[: len(warm_ranks)]):
        o.apply_batch(b)
        if i == 0:
            oracle.set_num_threads(1)
            t = time.perf_counter()
            _, st1 = o.dynamic_frontier(b, R, frontier_tol=args.frontier_tol)
            dt1 = time.perf_counter() - t
            oracle.set_num_threads(cores)
            one = {"value": round(st1.edges_processed / dt1 / 1e9, 4), "unit": "GTEPS",
                   "cores": 1, "seconds": round(dt1, 2),
                   "sample": f"Dynamic Frontier on the first batch ({b.size} edges)"}
            log(f"oracle batch 0 on one thread: {dt1:.2f}s")
        t = time.perf_counter()
        Rn, st = o.dynamic_frontier(b, R, frontier_tol=args.frontier_tol)
        dt = time.perf_counter() - t
        spent += dt
        edges += st.edges_processed
        used += 1
        # the GPU's batch i started from its own result of batch i - 1, the
        # oracle's from its own: the two agree to ~1e-17 at every step
        for e, Rg in ((err64, warm_ranks[i]), (err32, warm32[i][0])):
            d = np.abs(Rg - Rn)
            e["linf"] = max(e["linf"], float(np.max(d)))
            e["l1"] = max(e["l1"], float(np.sum(d)))
        R = Rn
        log(f"oracle batch {i}: {b.size} edges, {st.iterations} it, {dt:.2f}s")
        if spent >= args.cpu_seconds:
            break
    return {"value": round(edges / spent / 1e9, 4), "unit": "GTEPS",
            "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"Dynamic Frontier (mark + iterate) on the first {used} batches of the "
                      f"same sequence and graph, {spent:.1f}s of CPU time",
            "one_thread": one,
            "gpu_fp64_vs_oracle": err64, "gpu_fp32_form_vs_oracle": err32,
            "batches_compared": used}


def grid_bench(args, dfpr, synth, side=4096, kinds=("uniform", "localised"), per_kind=5,
               tol_sweep=True):
    """High-diameter workload: side x side grid with bidirectional
    4-neighbour edges and diagonal shortcuts for 5% of the vertices;
    batches of 1e-5 |E|, uniform and localised to one square window.
    tol_sweep adds fixed and adaptive frontier tolerances on one more
    localised batch."""
    t = time.time()
    n, src, dst = synth.grid2d(side, 0.05, seed=1)
    g = dfpr.Graph(n, src, dst)
    m = g.m
    log(f"grid {side}x{side}: n={n} m={m} ({time.time() - t:.1f}s)")
    p = dfpr.params(frontier_tol=args.frontier_tol)
    R0, st0 = g.static(p, out=False)
    nd, ni = synth.batch_counts(1e-5, m)
    uni = synth.batch_sequence(src, dst, n, [(nd, ni)] * per_kind, seed=2)
    loc = [synth.localized_batch(src, dst, side, nd, ni, seed=10 + k) for k in range(per_kind)]
    res = {}
    for kind, batches in (("uniform", uni), ("localised", loc)):
        rows = []
        for b in batches:
            R_prev = g.ranks()
            g.apply_batch(b)
            _, st = g.dynamic_frontier(b, p=p, out=False)
            rows.append(st)
            log(f"{kind}: batch {b.size}, {st.iterations} it ({st.loop_iterations} in the "
                f"small-frontier loop), affected {st.affected_final}, {st.ms_device:.2f} ms")
        ms = [r.ms_device for r in rows]
        # Naive-dynamic and Dynamic Traversal for the last batch, from the
        # same previous ranks as its Dynamic Frontier call
        R_df = g.ranks()
        g.set_ranks(R_prev)
        _, st_nv = g.naive_dynamic(None, p=p, out=False)
        g.set_ranks(R_prev)
        _, st_dt = g.dynamic_traversal(batches[-1], p=p, out=False)
        g.set_ranks(R_df)
        res[kind] = {
            "df_ms_p50": round(pct(ms, 50), 3), "df_ms_p99": round(pct(ms, 99), 3),
            "df_iterations_mean": round(float(np.mean([r.iterations for r in rows])), 1),
            "df_affected_mean": int(np.mean([r.affected_final for r in rows])),
            "df_us_per_iteration": round(float(np.sum(ms) * 1e3 / np.sum([r.iterations for r in rows])), 1),
            "df_gteps": round(float(np.sum([r.edges_processed for r in rows]) / np.sum(ms) / 1e6), 2),
            "df_ms_last": round(rows[-1].ms_device, 3),
            "df_loop_iterations_mean": round(float(np.mean([r.loop_iterations for r in rows])), 1),
            "naive_ms": round(st_nv.ms_device, 3), "naive_iterations": st_nv.iterations,
            "speedup_vs_naive": round(st_nv.ms_device / rows[-1].ms_device, 2),
            "dt_ms": round(st_dt.ms_device, 3), "dt_iterations": st_dt.iterations,
            "dt_affected": st_dt.affected_final,
            "speedup_vs_dt": round(st_dt.ms_device / rows[-1].ms_device, 2),
        }
    out = {"metric": METRIC, "workload": f"grid{side}_diag5_df_fp64", "n": n, "m": m,
           "batch": [nd, ni], "static_ms": round(st0.ms_device, 3),
           "static_iterations": st0.iterations,
           "static_gteps": round(st0.edges_processed / st0.ms_device / 1e6, 2), "kinds": res}
    for kind in res:
        res[kind]["speedup_vs_static"] = round(st0.ms_device / res[kind]["df_ms_p50"], 2)
    if not tol_sweep:
        g.close()
        return out
    # frontier tolerance on localised batches (the paper leaves an adaptive
    # tau_f to future work; this compares fixed values): one more localised
    # batch, each tau_f from the same previous ranks, L1 against a reference
    # Static of the updated graph
    # Each variant starts from the reference ranks of the graph before the
    # batch: on this graph (mean rank 6e-8) ranks that stopped at an L-inf
    # change of tau carry an L1 error of ~1e-4 that would hide tau_f.
    # fixed and adaptive tau_f on one more batch of each kind
    pref = dfpr.params(tol=0.0, max_iters=500)
    R_df_end = g.ranks()
    extras = {"localised": synth.localized_batch(src, dst, side, nd, ni, seed=99),
              "uniform": synth.random_batch(*current_edges(g), n, nd, ni, seed=98)}
    for kind, extra in extras.items():
        R_prev, _ = g.static(pref)
        g.apply_batch(extra)
        Rr, _ = g.static(pref)
        ftol_cmp = {}
        for f in (1e-11, 1e-12, 1e-13, 1e-15, "adaptive"):
            g.set_ranks(R_prev)
            ft = dfpr.FTOL_ADAPTIVE if f == "adaptive" else f
            R, st = g.dynamic_frontier(extra, p=dfpr.params(frontier_tol=ft))
            ftol_cmp[str(f)] = {"df_ms": round(st.ms_device, 3), "iterations": st.iterations,
                                "affected": st.affected_final,
                                "frontier_tol_used": st.frontier_tol_used,
                                "l1": float(np.sum(np.abs(R - Rr)))}
            log(f"{kind}, tau_f {f}: {ftol_cmp[str(f)]}")
        g.set_ranks(R_prev)
        R, st = g.naive_dynamic(p=dfpr.params())
        ftol_cmp["naive_dynamic"] = {"ms": round(st.ms_device, 3), "iterations": st.iterations,
                                     "l1": float(np.sum(np.abs(R - Rr)))}
        out[f"{kind}_frontier_tol"] = ftol_cmp
        g.set_ranks(R)
    g.close()
    return out


def fp32_bench(args, dfpr, synth, scale=24, per_size=5, oracle_check=False):
    """Precision form on R-MAT scale 24: for each batch, from the same
    previous ranks, plain FP64 Dynamic Frontier, the FP32 storage form (FP32
    phase + FP64 refinement) and the FP32 phase alone (the same call capped
    at its FP32 iterations), with max-abs and L1 differences from the GPU's
    FP64 result.  With oracle_check, the first batch of each size is also
    run by the FP64 oracle from the same previous ranks (and capped at the
    FP32 phase's iterations), and all three are compared with it."""
    import torch
    t = time.time()
    n, src, dst = synth.rmat(scale, 16, seed=1)
    log(f"R-MAT scale {scale}: n={n} edges={src.size} ({time.time() - t:.1f}s)")
    g = dfpr.Graph(n, src, dst)
    m = g.m
    p64 = dfpr.params(frontier_tol=args.frontier_tol)
    p32 = dfpr.params(frontier_tol=args.frontier_tol, precision=dfpr.FP32_KAHAN)
    g.static(p64, out=False)
    sizes = (1e-6, 1e-4)
    counts = [synth.batch_counts(f, m) for f in sizes * per_size]
    seq = synth.batch_sequence(src, dst, n, counts, seed=2)
    o = None
    if oracle_check:
        import oracle
        oracle.build(force=False)
        t = time.time()
        o = oracle.OracleGraph(n, src, dst)
        log(f"oracle loaded at scale {scale} ({time.time() - t:.1f}s)")
    del src, dst
    by, vs_oracle = {}, {}
    for i, b in enumerate(seq):
        f = sizes[i % 2]
        R_prev = g.ranks()
        g.apply_batch(b)
        # each variant starts from the same resident ranks (set outside the
        # timed call); FP64 runs last so its result carries on
        _, s32 = g.dynamic_frontier(b, p=p32, out=False)
        R32 = g.ranks()
        k32 = s32.iterations - s32.refine_sweeps
        p32c = dfpr.params(frontier_tol=args.frontier_tol, precision=dfpr.FP32_KAHAN, max_iters=k32)
        g.set_ranks(R_prev)
        _, s32p = g.dynamic_frontier(b, p=p32c, out=False)
        R32p = g.ranks()
        g.set_ranks(R_prev)
        _, s64 = g.dynamic_frontier(b, p=p64, out=False)
        R64 = g.ranks()
        row = {"fp64_ms": s64.ms_device, "fp64_iterations": s64.iterations,
               "fp32_ms": s32.ms_device, "fp32_iterations": s32.iterations,
               "fp32_refine_sweeps": s32.refine_sweeps,
               "linf": float(np.max(np.abs(R32 - R64))), "l1": float(np.sum(np.abs(R32 - R64))),
               "linf_fp32_phase": float(np.max(np.abs(R32p - R64))),
               "l1_fp32_phase": float(np.sum(np.abs(R32p - R64)))}
        by.setdefault(str(f), []).append(row)
        log(f"{f}: batch {b.size}: FP64 {s64.ms_device:.2f} ms {s64.iterations} it; FP32 form "
            f"{s32.ms_device:.2f} ms ({s32.refine_sweeps} refine); Linf {row['linf']:.2e}")
        if o is not None and i < len(sizes):
            t = time.time()
            o.apply_batch(b)
            Rd, sd = o.dynamic_frontier(b, R_prev, frontier_tol=args.frontier_tol)
            Rk, _ = o.dynamic_frontier(b, R_prev, frontier_tol=args.frontier_tol, max_iters=k32)
            cmp_ = {}
            for name, R, ref in (("fp64", R64, Rd), ("fp32_form", R32, Rd),
                                 ("fp32_phase", R32p, Rk)):
                d = np.abs(R - ref)
                cmp_[name] = {"linf": float(np.max(d)), "l1": float(np.sum(d)),
                              "max_rel": float(np.max(d / ref))}
            cmp_["oracle_iterations"] = sd.iterations
            cmp_["fp32_phase_iterations"] = k32
            vs_oracle[str(f)] = cmp_
            log(f"{f}: oracle ({time.time() - t:.1f}s): {cmp_}")
    summ = {}
    for f, rows in by.items():
        t64 = [r["fp64_ms"] for r in rows]
        t32 = [r["fp32_ms"] for r in rows]
        summ[f] = {"fp64_ms_p50": round(pct(t64, 50), 3), "fp32_form_ms_p50": round(pct(t32, 50), 3),
                   "fp32_form_updates_per_s_vs_fp64": round(sum(t64) / sum(t32), 3),
                   "fp64_updates_per_s": round(len(t64) / (sum(t64) / 1e3), 2),
                   "fp32_form_updates_per_s": round(len(t32) / (sum(t32) / 1e3), 2),
                   "fp32_refine_sweeps_mean": round(float(np.mean([r["fp32_refine_sweeps"] for r in rows])), 1),
                   "max_linf_vs_fp64": max(r["linf"] for r in rows),
                   "max_l1_vs_fp64": max(r["l1"] for r in rows),
                   "max_linf_fp32_phase_vs_fp64": max(r["linf_fp32_phase"] for r in rows),
                   "max_l1_fp32_phase_vs_fp64": max(r["l1_fp32_phase"] for r in rows)}
    g.close()
    del g, o
    torch.cuda.empty_cache()
    return {"metric": "FP32 vs FP64 at 1e-9 L-inf", "workload": f"rmat{scale}_ef16_fp32_form_vs_fp64",
            "n": n, "m": m, "batches_per_size": per_size, "by_frac": summ,
            "vs_fp64_oracle": vs_oracle}


def sweep_bench(args, dfpr, synth, scale=22):
    """Frontier tolerance sweep (Section 4.3, Figure 3) and batch mixes
    (Section 5.2: insertions only, deletions only, 80/20) on R-MAT scale 22.
    Errors are L1 against a reference Static on the updated graph (tolerance
    0, at most 500 iterations: Section 5.1.5), computed on the GPU."""
    t = time.time()
    n, src, dst = synth.rmat(scale, 16, seed=1)
    g = dfpr.Graph(n, src, dst)
    m = g.m
    log(f"R-MAT scale {scale}: n={n} m={m} ({time.time() - t:.1f}s)")
    tol = 1e-10
    pref = dfpr.params(tol=0.0, max_iters=500)
    g.static(dfpr.params(), out=False)

    def reference():
        R_keep = g.ranks()
        Rr, sr = g.static(pref)
        g.set_ranks(R_keep)
        return Rr

    def l1(R, Rr):
        return float(np.sum(np.abs(R - Rr)))

    out = {"metric": METRIC, "workload": f"rmat{scale}_ef16_sweep", "n": n, "m": m}
    # frontier tolerance, three 1e-5 |E| batches
    ftols = [tol / 10 ** k for k in range(6)] + ["adaptive"]
    seq = synth.batch_sequence(src, dst, n, [synth.batch_counts(1e-5, m)] * 3, seed=40)
    sweep = {str(f): {"ms": [], "l1": [], "affected": [], "iterations": [], "used": []}
             for f in ftols}
    nv = {"ms": [], "l1": []}
    for b in seq:
        R_prev = g.ranks()
        g.apply_batch(b)
        Rr = reference()
        for f in ftols:
            g.set_ranks(R_prev)
            ft = dfpr.FTOL_ADAPTIVE if f == "adaptive" else f
            R, st = g.dynamic_frontier(b, p=dfpr.params(tol=tol, frontier_tol=ft))
            d = sweep[str(f)]
            d["ms"].append(st.ms_device)
            d["l1"].append(l1(R, Rr))
            d["affected"].append(st.affected_final)
            d["iterations"].append(st.iterations)
            d["used"].append(st.frontier_tol_used)
        g.set_ranks(R_prev)
        R, st = g.naive_dynamic(p=dfpr.params(tol=tol))
        nv["ms"].append(st.ms_device)
        nv["l1"].append(l1(R, Rr))
        g.set_ranks(R)
    out["frontier_tol_sweep"] = {
        f: {"df_ms_mean": round(float(np.mean(d["ms"])), 3),
            "l1_mean": float(np.mean(d["l1"])),
            "affected_mean": int(np.mean(d["affected"])),
            "iterations_mean": round(float(np.mean(d["iterations"])), 1),
            "frontier_tol_used": sorted(set(d["used"]))}
        for f, d in sweep.items()}
    out["frontier_tol_sweep"]["naive_dynamic"] = {"ms_mean": round(float(np.mean(nv["ms"])), 3),
                                                  "l1_mean": float(np.mean(nv["l1"]))}
    for f, d in out["frontier_tol_sweep"].items():
        log(f"tau_f {f}: {d}")
    # batch mixes
    mixes = {}
    fp = dfpr.params(tol=tol, frontier_tol=args.frontier_tol)
    for frac in (1e-7, 1e-5, 1e-3):
        bsz = max(1, int(round(frac * m)))
        for kind, cnt in (("insertions", (0, bsz)), ("deletions", (bsz, 0)),
                          ("mixed_80_20", synth.batch_counts(frac, m))):
            b = synth.batch_sequence(src, dst, n, [cnt], seed=50 + len(mixes))[0]
            R_prev = g.ranks()
            g.apply_batch(b)
            Rr = reference()
            g.set_ranks(R_prev)
            Rd, sd = g.dynamic_frontier(b, p=fp)
            g.set_ranks(R_prev)
            Rn, sn = g.naive_dynamic(p=fp)
            Rs, ss = g.static(fp)
            key = f"{kind}_{frac}"
            mixes[key] = {"df_ms": round(sd.ms_device, 3), "naive_ms": round(sn.ms_device, 3),
                          "static_ms": round(ss.ms_device, 3),
                          "speedup_vs_static": round(ss.ms_device / sd.ms_device, 2),
                          "speedup_vs_naive": round(sn.ms_device / sd.ms_device, 2),
                          "df_l1": l1(Rd, Rr), "naive_l1": l1(Rn, Rr), "static_l1": l1(Rs, Rr),
                          "df_affected": sd.affected_final, "df_iterations": sd.iterations,
                          "naive_iterations": sn.iterations, "static_iterations": ss.iterations}
            g.set_ranks(Rd)
            log(f"{key}: {mixes[key]}")
    out["batch_mixes"] = mixes
    print(json.dumps(out), flush=True)


def serve_bench(args, dfpr, synth, nreq=None):
    """Serving form: resident R-MAT graphs of scales 16..22 (three seeds
    each), update batches of log-uniform size in [1e-7, 1e-3] |E| for a
    uniformly chosen graph, FP32 storage on one graph of every scale.
    Two request sets run one after the other on two copies of the graphs:
    a closed-loop set (all requests at t = 0; saturation throughput) and an
    open-loop set with Poisson arrivals at --serve-load of the one-at-a-time
    capacity (latency).  The comparator serves every request alone, in
    arrival order, with plain FP64 Dynamic Frontier; its latencies follow
    from the measured service times on a FIFO timeline."""
    scales = [int(x) for x in args.serve_scales.split(",")]
    graphs = []                      # (name, n, src, dst, precision)
    t = time.time()
    for sc in scales:
        for k in range(3):
            n, s_, d_ = synth.rmat(sc, 16, seed=100 + 10 * sc + k)
            graphs.append((f"rmat{sc}s{k}", n, s_, d_, dfpr.FP32_KAHAN if k == 1 else dfpr.FP64))
    log(f"generated {len(graphs)} graphs ({time.time() - t:.1f}s)")
    G = len(graphs)
    rng = synth.rng_for(7)
    nreq = nreq or args.serve_requests

    def request_set(tag):
        gid = rng.integers(0, G, size=nreq)
        u = rng.random(nreq)
        gaps = rng.exponential(1.0, size=nreq)
        fr = np.exp(np.log(1e-7) + u * (np.log(1e-3) - np.log(1e-7)))
        return {"tag": tag, "gid": gid, "frac": fr, "gaps": gaps}

    sets = [request_set("closed"), request_set("open")]
    # per graph: the batches of both sets, in order, as one disjoint sequence
    batches = {}
    for gi, (name, n, s_, d_, prec) in enumerate(graphs):
        m = s_.size + n
        order = [(si, k) for si, rs in enumerate(sets) for k in range(nreq) if rs["gid"][k] == gi]
        counts = [synth.batch_counts(sets[si]["frac"][k], m) for si, k in order]
        seq = synth.batch_sequence(s_, d_, n, counts, seed=200 + gi)
        for (si, k), b in zip(order, seq):
            batches[(si, k)] = b

    pdef = dfpr.params(frontier_tol=args.frontier_tol)
    pg = [dfpr.params(frontier_tol=args.frontier_tol, precision=gr[4]) for gr in graphs]
    t = time.time()
    base = [dfpr.Graph(gr[1], gr[2], gr[3]) for gr in graphs]
    mine = [dfpr.Graph(gr[1], gr[2], gr[3]) for gr in graphs]
    for g in base + mine:
        g.static(pdef, out=False)
    log(f"loaded and solved 2 x {G} graphs ({time.time() - t:.1f}s)")

    def one_at_a_time(si):
        svc = []
        for k in range(nreq):
            g = base[sets[si]["gid"][k]]
            b = batches[(si, k)]
            ts = time.perf_counter()
            g.apply_batch(b)
            g.dynamic_frontier(b, p=pdef, out=False)
            svc.append((time.perf_counter() - ts) * 1e3)
        return svc

    def serve(si, arrivals):
        srv = dfpr.Server(max_slots=args.serve_slots, hbm_budget_bytes=200 << 30)
        ids = [srv.add_graph(g, p) for g, p in zip(mine, pg)]
        rids = [srv.submit(ids[sets[si]["gid"][k]], arrivals[k], batches[(si, k)])
                for k in range(nreq)]
        st = srv.run()
        res = [srv.result(r) for r in rids]
        srv.close()
        return st, res

    def fifo(arrivals, svc):
        done, lat, t_free = [], [], 0.0
        for a, s_ in zip(arrivals, svc):
            t_free = max(t_free, a) + s_
            lat.append(t_free - a)
        return lat, t_free

    out = {"metric": "serving: update latency p50/p99 and updates/s", "n_gpus": 1,
           "data": "synthetic", "dtype": "f64+f32-storage",
           "config": {"workload": "serving_rmat" + "_".join(map(str, scales)) + "_x3",
                      "graphs": [gr[0] for gr in graphs],
                      "fp32_graphs": [gr[0] for gr in graphs if gr[4] == dfpr.FP32_KAHAN],
                      "requests_per_set": nreq, "batch_frac_range": [1e-7, 1e-3],
                      "slots": args.serve_slots, "frontier_tol": args.frontier_tol}}
    # closed loop: everything at t = 0
    svc0 = one_at_a_time(0)
    cap = nreq / (sum(svc0) / 1e3)
    st0, res0 = serve(0, [0.0] * nreq)
    log(f"closed loop: one-at-a-time {cap:.1f} updates/s, served {st0['updates_per_s']:.1f} "
        f"updates/s, max active {st0['max_active']}, steps {st0['steps']}")
    out["closed_loop"] = {"one_at_a_time_updates_per_s": round(cap, 2),
                          "served_updates_per_s": round(st0["updates_per_s"], 2),
                          "speedup": round(st0["updates_per_s"] / cap, 3),
                          "served_max_active": st0["max_active"], "served_steps": st0["steps"]}
    # open loop: Poisson arrivals at a fraction of the one-at-a-time capacity
    rate = args.serve_load * cap / 1e3                       # per ms
    arr = list(np.cumsum(sets[1]["gaps"]) / rate)
    arr = [a - arr[0] for a in arr]
    svc1 = one_at_a_time(1)
    lat_b, end_b = fifo(arr, svc1)
    st1, res1 = serve(1, arr)
    lat_s = [r["done_ms"] - r["arrival_ms"] for r in res1]
    log(f"open loop at {args.serve_load:.2f} load: one-at-a-time p50 {pct(lat_b, 50):.2f} p99 "
        f"{pct(lat_b, 99):.2f} ms; served p50 {pct(lat_s, 50):.2f} p99 {pct(lat_s, 99):.2f} ms")
    out["open_loop"] = {
        "load": args.serve_load, "rate_per_s": round(rate * 1e3, 2),
        "one_at_a_time": {"p50_ms": round(pct(lat_b, 50), 3), "p99_ms": round(pct(lat_b, 99), 3),
                          "mean_ms": round(float(np.mean(lat_b)), 3),
                          "updates_per_s": round(nreq / (end_b / 1e3), 2)},
        "served": {"p50_ms": round(st1["latency_p50_ms"], 3),
                   "p99_ms": round(st1["latency_p99_ms"], 3),
                   "mean_ms": round(st1["latency_mean_ms"], 3),
                   "queue_p50_ms": round(st1["queue_p50_ms"], 3),
                   "queue_p99_ms": round(st1["queue_p99_ms"], 3),
                   "updates_per_s": round(st1["updates_per_s"], 2),
                   "max_active": st1["max_active"], "steps": st1["steps"]},
    }
    # final ranks: FP64 graphs bitwise equal to one-at-a-time, FP32 storage
    # graphs within the tolerance
    acc = {}
    for gi, gr in enumerate(graphs):
        Ra, Rb = base[gi].ranks(), mine[gi].ranks()
        acc[gr[0]] = {"precision": "fp32" if gr[4] else "fp64",
                      "bitwise_equal": bool(np.array_equal(Ra, Rb)),
                      "linf": float(np.max(np.abs(Ra - Rb))),
                      "l1": float(np.sum(np.abs(Ra - Rb)))}
    out["final_ranks_vs_one_at_a_time"] = acc
    fails = [r for r in res0 + res1 if r["status"] != 0 or not r["converged"]]
    out["failed_or_unconverged"] = len(fails)
    out["value"] = round(st0["updates_per_s"], 3)
    out["unit"] = "updates/s"
    out["higher_is_better"] = True
    for g in base + mine:
        g.close()
    return out


if __name__ == "__main__":
    main()
