"""Benchmark of the proximal message-passing hot path on one MI355X.

A step is one full message-passing iteration (line + device prox, node
aggregation and price update, FP64 residual norms, stopping test and
adaptive penalty) over the whole synthetic workload, resident in HBM.

Prints one JSON line: ADMM iterations/s of the FP32 iterate on the Large
workload (10,000 nodes, 13,000 lines, T = 96, K = 200), with the roofline
of the dominant kernel measured live with HIP events, the FP64 rate,
time-to-tolerance, and the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E, published
METRIC = "ADMM iters/s, time-to-1e-3 residual, HBM GB/s fraction (FP32 vs FP64, 1 GPU)"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ["opf_kernels.hip", "opf_device.h", "opf_internal.h"]:
        with open(os.path.join(ROOT, "paper_2410_17203_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_hash, workload, dtype):
    """HBM bytes per launch of a sweep kernel from committed counter runs
    (profiles/sweep_kernel_<workload>_<dtype>_traffic.json), if they were
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"sweep_kernel_{workload}_{dtype}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def time_iterations(solver, steps, warmup):
    import torch
    solver.iterate(warmup)
    solver.synchronize()
    solver.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.iterate(steps)
    solver.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = solver.kernel_times()
    solver.set_timing(False)
    return t1 - t0, kt


TUNING_CACHE = None


def _autotune(solver):
    """The library's autotuner (tiled vs node rows, period groups, grid) on
    this solver's instances, through the tuning cache when one is given, so
    that profiler runs time the configuration the plain run chose."""
    t = solver.autotune(trials=10, cache_path=TUNING_CACHE)
    return {k: t[k] for k in ("tiled", "tile_groups", "lanes_shift", "grid_factor")}


def batched_rates(iters, dtype, dual_dtype):
    """Aggregate instance-iterations/s of the 64 uneven instances as one batch
    and solved one at a time, both in 50-iteration graph blocks, each
    configuration picked by the autotuner first."""
    import torch
    from paper_2410_17203_amd import synth
    from paper_2410_17203_amd.binding import Solver
    insts = synth.batched()
    opts = dict(dtype=dtype, dual_dtype=dual_dtype, polish_fp64=0, eps=0.0, max_iter=iters)

    def run(arg):
        s = Solver(arg, **opts)
        _autotune(s)
        s.solve()  # warm-up: builds the graphs
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.solve()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s.close()
        return dt

    t_batch = run(insts)
    # one at a time: every instance in its own context (its configuration
    # from the autotuner, graphs built), solved one after another, then the
    # same contexts four at a time, each on its own stream from its own host
    # thread (the GPU runs four hardware queues per process)
    singles = []
    for x in insts:
        s = Solver(x, **opts)
        _autotune(s)
        s.solve()
        s.reset()
        singles.append(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in singles:
        s.solve()
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    for s in singles:
        s.reset()
    torch.cuda.synchronize()
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.perf_counter()
    with ThreadPoolExecutor(4) as ex:
        list(ex.map(lambda g: [s.solve() for s in g], [singles[w::4] for w in range(4)]))
    torch.cuda.synchronize()
    t_four = time.perf_counter() - t0
    for s in singles:
        s.close()
    n = len(insts)
    elems = sum((13 * i.L + 2 * (i.G + i.D + i.B) + 6 * i.N) * (i.K + 1) * i.T for i in insts)
    out = {"instances": n, "iters": iters, "state_dtype": dtype, "dual_dtype": dual_dtype,
           "batched_inst_iters_per_s": n * iters / t_batch,
           "one_at_a_time_inst_iters_per_s": n * iters / t_single,
           "four_streams_inst_iters_per_s": n * iters / t_four,
           "speedup": t_single / t_batch,
           "algorithmic_elements_per_iteration": elems}
    # per-kernel times of the batch (events around each launch, so no graphs)
    s = Solver(insts, dtype=dtype, dual_dtype=dual_dtype, polish_fp64=0, eps=0.0,
               min_iter=2**31 - 1, max_iter=2**31 - 1)
    out["tuning"] = _autotune(s)
    s.iterate(5)
    s.synchronize()
    s.set_timing(True)
    s.iterate(iters)
    s.synchronize()
    kt = s.kernel_times()
    s.close()
    sweep_ms = kt["sweep"]["ms"] / max(kt["sweep"]["launches"], 1)
    out["kernel_ms_per_launch"] = {k: v["ms"] / max(v["launches"], 1) for k, v in kt.items()}
    if dtype == dual_dtype:
        # contracted bytes of the sweep, as for the single-instance line
        S = 4 if dtype == "f32" else 8
        sweep_bytes = S * sum((13 * i.L + 6 * i.N) * (i.K + 1) * i.T for i in insts)
        traffic = traffic_from_profiles(kernel_source_hash(), "batch64", dtype)
        out["sweep_roofline"] = {
            "bound": "hbm", "kernel": "k_sweep_tile_batch", "ms_per_launch": sweep_ms,
            "algorithmic_bytes_per_launch": sweep_bytes,
            "achieved": sweep_bytes / (sweep_ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": sweep_bytes / (sweep_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "traffic": traffic,
            "frac_counters": (None if traffic is None
                              else traffic / (sweep_ms * 1e-3) / 1e9 / PEAK_HBM_GBS)}
    return out


def batched_time_to_tolerance(max_iter):
    """Wall-clock to eq. converge at 1e-3 (relative) of the 64 uneven
    instances: one batched solve (FP32 iterate, graph blocks, each instance
    stopping on its own) against the same instances solved one after
    another with the same arithmetic (FP32 iterate, no FP64 polish, which
    batches do not apply), so each instance stops at the same iteration
    either way."""
    import torch
    from paper_2410_17203_amd import synth
    from paper_2410_17203_amd.binding import Solver
    insts = synth.batched()
    b = Solver(insts, dtype="f32", eps=1e-3, max_iter=max_iter)
    _autotune(b)
    b.solve()  # warm-up: builds the graphs
    b.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.solve()
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    res = [b.residuals(i) for i in range(len(insts))]
    b.close()
    conv_b = [r["converged"] for r in res]
    iters_b = [r["iter"] for r in res]
    singles = []
    for inst in insts:
        s = Solver(inst, dtype="f32", eps=1e-3, max_iter=max_iter, polish_fp64=0)
        _autotune(s)
        s.solve()
        s.reset()
        singles.append(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = [s.solve() for s in singles]
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    conv_s = [r["status"] == "OPF_OK" for r in rs]
    iters_s = [r["iter"] for r in rs]
    # the same contexts four at a time, each on its own stream from its own thread
    for s in singles:
        s.reset()
    torch.cuda.synchronize()
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.perf_counter()
    with ThreadPoolExecutor(4) as ex:
        list(ex.map(lambda g: [s.solve() for s in g], [singles[w::4] for w in range(4)]))
    torch.cuda.synchronize()
    t_four = time.perf_counter() - t0
    for s in singles:
        s.close()
    return {"instances": len(insts), "eps": 1e-3, "max_iter": max_iter,
            "batched_s": t_batch, "one_at_a_time_s": t_single, "four_streams_s": t_four,
            "speedup": t_single / t_batch,
            "batched_converged": int(sum(conv_b)), "one_at_a_time_converged": int(sum(conv_s)),
            "batched_iters_max": int(max(iters_b)), "batched_iters_median": float(sorted(iters_b)[len(iters_b) // 2]),
            "one_at_a_time_iters_total": int(sum(iters_s))}


def medium_leg(steps=1000, warmup=50):
    """The Medium workload (500 nodes, 700 lines, T = 24, K = 50): FP32 and
    FP64 iterations/s with the sweep's bytes over its time (its state, about
    22 MB in FP32, stays in the 256 MB last-level cache, so that fraction is
    cache-resident, not HBM), and time to 1e-3 (FP32 + FP64 polish, and FP64
    throughout)."""
    import torch
    from paper_2410_17203_amd import synth
    from paper_2410_17203_amd.binding import Solver
    inst = synth.config("medium")
    out = {"workload": "medium: N=500 L=700 G=100 D=400 B=20 T=24 K=50 (synthetic, seed 500)"}
    never = dict(eps=0.0, min_iter=2**31 - 1, max_iter=2**31 - 1, polish_fp64=0)
    for dt in ("f32", "f64"):
        # kernel durations: direct launches with events around each kernel
        s = Solver(inst, dtype=dt, **never)
        el, kt = time_iterations(s, steps, warmup)
        sw = kt["sweep"]["ms"] / max(kt["sweep"]["launches"], 1)
        S = 4 if dt == "f32" else 8
        sweep_bytes = S * (inst.K + 1) * inst.T * (13 * inst.L + 6 * inst.N)
        s.close()
        # the rate: the same iterations in graph blocks without the events,
        # which cost about as much as a small instance's kernels
        s = Solver(inst, dtype=dt, polish_fp64=0, eps=0.0, max_iter=steps)
        s.solve()  # warm-up: builds the graphs
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve()
        torch.cuda.synchronize()
        el_graph = time.perf_counter() - t0
        s.close()
        out[dt] = {"iters_per_s": r["iter"] / el_graph,
                   "iters_per_s_with_kernel_events": steps / el, "sweep_ms": sw,
                   "sweep_GBps_contracted_cache_resident": sweep_bytes / (sw * 1e-3) / 1e9}
        s = Solver(inst, dtype=dt, eps=1e-3, max_iter=20000)
        s.solve()  # warm-up: builds the graphs
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve()
        torch.cuda.synchronize()
        out[dt].update({"time_to_tol_s": time.perf_counter() - t0, "time_to_tol_iters": r["iter"],
                        "time_to_tol_converged": r["status"] == "OPF_OK",
                        "objective": r["objective"]})
        s.close()
    out["f32_objective_rel_err_vs_fp64"] = (abs(out["f32"]["objective"] - out["f64"]["objective"])
                                            / abs(out["f64"]["objective"]))
    return out


def general_model_rate(inst, steps, warmup):
    """Iterations/s of the FP32 iterate on the same workload extended to the
    general line model: 3 HVDC links (the paper's network has 3 among about
    1,150 lines) and per-contingency changes (50 second outages, 100
    emergency ratings, 50 susceptance changes); the sweep then runs its
    general-line-model variant."""
    from paper_2410_17203_amd import synth
    from paper_2410_17203_amd.binding import Solver
    x = synth.with_contingency_changes(synth.with_dc_links(inst, 3, seed=1), seed=2,
                                       second_outages=50, rating_changes=100, sus_changes=50)
    s = Solver(x, dtype="f32", polish_fp64=0, eps=0.0, min_iter=2**31 - 1, max_iter=2**31 - 1)
    elapsed, kt = time_iterations(s, steps, warmup)
    sw = kt["sweep"]
    out = {"dc_links": 3, "changes": int(len(x.chg_k)), "iters_per_s": steps / elapsed,
           "sweep_ms": sw["ms"] / max(sw["launches"], 1)}
    s.close()
    return out


def planning_leg(steps, scenarios=8, workers_list=(1, 4)):
    """Wall-clock of the gradient-based planning loop (Section 5.6 shape:
    8 load scenarios of the 500-node grid with T = 24, here with K = 20
    contingencies; each step a warm-started recorded solve of 250..1000
    iterations and its adjoint per scenario), with the scenarios one after
    another and several at a time on their own streams."""
    import numpy as np
    import torch
    from paper_2410_17203_amd import synth
    from paper_2410_17203_amd.planning import plan_capacities
    sc = []
    for m in range(scenarios):
        x = synth.config("medium", K=20)
        rng = np.random.default_rng(200 + m)
        x.load_d = np.asarray(x.load_d) * rng.uniform(0.95, 1.05, np.shape(x.load_d))
        sc.append(x)
    L, G = len(sc[0].line_from), len(sc[0].gen_node)
    out = {"workload": f"{scenarios} scenarios of medium with K=20 (500 nodes, T=24), FP32",
           "steps": steps}
    for w in workers_list:
        t0 = time.perf_counter()
        r = plan_capacities(sc, steps=steps, step_size=1e-4, line_cost=np.full(L, 1.0),
                            gen_cost=np.full(G, 1.0), min_iters=250, max_iters=1000, eps=1e-3,
                            dtype="f32", workers=w)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"workers_{w}"] = {"s": dt, "s_per_evaluation": dt / (steps + 1),
                               "losses": [x.loss for x in r.steps],
                               "iterations": [x.iterations for x in r.steps]}
    return out


def adjoint_times(n_iters, every, dtype):
    """Wall-clock of the recorded forward run and of the adjoint on the
    differentiation workload (gradient of cost + <w, dispatch> w.r.t. load,
    line capacity and generator limits)."""
    import numpy as np
    import torch
    from paper_2410_17203_amd import synth
    from paper_2410_17203_amd.binding import Solver
    inst = synth.config("diff")
    J = len(inst.gen_node) + len(inst.load_node) + len(inst.bat_node)
    w = np.random.default_rng(2024).normal(size=(J, inst.T))
    s = Solver(inst, dtype=dtype, polish_fp64=0)
    if every is None:
        every = s.checkpoint_interval(n_iters)
    s.tape_forward(50, every)  # warm-up
    s.adjoint(w, 1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.tape_forward(n_iters, every)
    t1 = time.perf_counter()
    s.adjoint(w, 1.0)
    t2 = time.perf_counter()
    tape_gib = s.tape.numel() / 2**30
    plain = Solver(inst, dtype=dtype, polish_fp64=0, eps=0.0, min_iter=2**31 - 1,
                   max_iter=2**31 - 1)
    plain.iterate(20)
    plain.synchronize()
    t3 = time.perf_counter()
    plain.iterate(n_iters)
    plain.synchronize()
    t4 = time.perf_counter()
    s.close()
    plain.close()
    return {"workload": "diff: N=500 L=700 G=100 D=400 B=20 T=24 K=20 (synthetic, seed 2024)",
            "dtype": dtype, "iters": n_iters, "checkpoint_every": every, "tape_GiB": tape_gib,
            "forward_plain_s": t4 - t3, "forward_recorded_s": t1 - t0, "backward_s": t2 - t1,
            "backward_over_forward": (t2 - t1) / (t4 - t3)}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(inst, iters, threads):
    """Seconds per iteration of the FP64 oracle at the given thread count
    (one untimed iteration first: it builds the factorisations)."""
    import torch
    from oracle.mp import Options, Solver as Oracle
    old = torch.get_num_threads()
    torch.set_num_threads(threads)
    try:
        o = Oracle(inst, Options(eps=1e-12))
        o.step()
        t0 = time.perf_counter()
        for _ in range(iters):
            o.step()
        return (time.perf_counter() - t0) / iters
    finally:
        torch.set_num_threads(old)


def cpu_baseline(inst_name, sample_k, iters, medium_iters):
    """FP64 oracle on the host cores.  The headline figure: the workload's
    grid and horizon with sample_k contingencies, per-iteration time scaled
    linearly to the full K + 1 (the oracle's work is linear in K + 1), at
    all threads torch uses; the same sample at one thread; and the Medium
    workload run whole (no extrapolation) at all threads."""
    import torch
    from paper_2410_17203_amd import synth
    full = synth.CONFIGS[inst_name]
    threads = torch.get_num_threads()
    inst = synth.config(inst_name, K=sample_k)
    scale = (full["K"] + 1) / (sample_k + 1)
    dt = _oracle_rate(inst, iters, threads)
    dt1 = _oracle_rate(inst, max(2, iters // 4), 1)
    med = synth.config("medium")
    dtm = _oracle_rate(med, medium_iters, threads)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"value": 1.0 / (dt * scale), "unit": "iter/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"{inst_name} grid and horizon with K={sample_k} of {full['K']} "
                       f"contingencies, {iters} timed iterations after 1 untimed; "
                       f"{dt:.3f} s/iteration scaled by the (K+1) ratio {scale:.1f}"),
            "single_thread_value": 1.0 / (dt1 * scale),
            "single_thread_sample": f"the same sample, {max(2, iters // 4)} iterations, 1 thread",
            "medium_full_iters_per_s": 1.0 / dtm,
            "medium_full_sample": (f"medium workload whole (N=500 L=700 T=24 K=50), "
                                   f"{medium_iters} iterations, {threads} threads, not scaled"),
            "nproc": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": _cpu_model()}


def _read_csv(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _find(directory, *suffixes):
    for suffix in suffixes:
        for root, _, files in os.walk(directory):
            for f in sorted(files):
                if f.endswith(suffix):
                    return os.path.join(root, f)
    raise FileNotFoundError(f"no *{suffixes} under {directory}")


def _stats_rows(directory):
    """Per-kernel statistics: rocprofv3's own --stats table when present,
    else the same figures computed from its kernel trace."""
    try:
        return _read_csv(_find(directory, "kernel_stats.csv"))
    except FileNotFoundError:
        pass
    by = {}
    for r in _read_csv(_find(directory, "kernel_trace.csv")):
        by.setdefault(r["Kernel_Name"], []).append(
            int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    total = sum(sum(v) for v in by.values())
    rows = [{"Name": k, "Calls": len(v), "AverageNs": sum(v) / len(v), "MinNs": min(v),
             "MaxNs": max(v), "Percentage": 100.0 * sum(v) / total} for k, v in by.items()]
    return sorted(rows, key=lambda r: -r["Percentage"])


def summarize_stats(directory, out_path, command):
    """Markdown summary of a rocprofv3 --kernel-trace --stats run."""
    rows = _stats_rows(directory)
    lines = [f"# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share of GPU time |",
             "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f}% |")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_traffic(fetch_dir, write_dir, out_path, kernel, workload, command_fetch,
                      command_write, request_dir=None, command_request=None):
    """HBM bytes per launch of the kernels whose names contain one of the
    '|'-separated `kernel` patterns, from FETCH_SIZE and WRITE_SIZE runs
    (KiB per dispatch), each scaled by what the counter reads for a plain
    1 GiB -> 1 GiB elementwise copy in the same run."""
    patterns = [k for k in kernel.split("|") if k]

    def hit(name):
        return any(k in name for k in patterns)

    def per_kernel(directory, counter):
        rows = [r for r in _read_csv(_find(directory, "counter_collection.csv",
                                           "counter_collection_trace.csv"))
                if r["Counter_Name"] == counter]
        copy = [float(r["Counter_Value"]) for r in rows if "MulFunctor" in r["Kernel_Name"]]
        sweep = [float(r["Counter_Value"]) for r in rows if hit(r["Kernel_Name"])]
        if not copy or not sweep:
            raise RuntimeError(f"{counter}: copy or {kernel} dispatches missing")
        # dispatches with work: a solve replays whole graph blocks, and the
        # launches after every instance has stopped exit at once (they move
        # about 1% of a working launch's bytes)
        full = max(sweep)
        skipped[counter] = sum(1 for v in sweep if v < 0.5 * full)
        sweep = [v for v in sweep if v >= 0.5 * full]
        copy_kib = sum(copy) / len(copy)
        factor = 2.0**20 / copy_kib  # the copy moves exactly 1 GiB each way
        spread[counter] = [min(sweep), max(sweep)]
        return factor, copy_kib, sum(sweep) / len(sweep), len(sweep)
    spread, skipped = {}, {}
    fr, fcopy, fsweep, nf = per_kernel(fetch_dir, "FETCH_SIZE")
    wr, wcopy, wsweep, nw = per_kernel(write_dir, "WRITE_SIZE")
    read_b = fsweep * 1024 * fr
    write_b = wsweep * 1024 * wr
    d = {"kernel": kernel, "workload": workload,
         "kernel_source_hash": kernel_source_hash(),
         "fetch_kib_per_launch_raw": fsweep, "write_kib_per_launch_raw": wsweep,
         "copy_fetch_kib_raw": fcopy, "copy_write_kib_raw": wcopy,
         "fetch_scale": fr, "write_scale": wr, "launches": [nf, nw],
         "idle_launches_skipped": [skipped["FETCH_SIZE"], skipped["WRITE_SIZE"]],
         "min_max_kib_raw": spread,
         "hbm_read_bytes_per_launch": read_b, "hbm_write_bytes_per_launch": write_b,
         "hbm_bytes_per_launch": read_b + write_b,
         "command_fetch": command_fetch, "command_write": command_write}
    if request_dir:
        # read requests by size (32/64/128 bytes): exact read bytes, a check
        # on the copy-scaled FETCH_SIZE figure
        rows = _read_csv(_find(request_dir, "counter_collection.csv", "counter_collection_trace.csv"))
        per = {}
        for r in rows:
            if hit(r["Kernel_Name"]):
                per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        avg = {k: sum(v) / len(v) for k, v in per.items()}
        d["read_requests_per_launch"] = {k.replace("TCC_EA0_", ""): v for k, v in avg.items()}
        d["read_bytes_from_request_sizes"] = (32 * avg.get("TCC_EA0_RDREQ_32B_sum", 0.0) +
                                              64 * avg.get("TCC_EA0_RDREQ_64B_sum", 0.0) +
                                              128 * avg.get("TCC_EA0_RDREQ_128B_sum", 0.0))
        d["command_request"] = command_request
    with open(out_path, "w") as fh:
        json.dump(d, fh, indent=1)
        fh.write("\n")
    print(json.dumps(d, indent=1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="large")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--fp64-steps", type=int, default=50, help="0 skips the FP64 rate")
    ap.add_argument("--ttt", type=int, default=1, help="1: measure time to tolerance")
    ap.add_argument("--ttt-max-iter", type=int, default=10000)
    ap.add_argument("--batched", type=int, default=1,
                    help="1: also time the 64-instance batch against one-at-a-time solves")
    ap.add_argument("--batched-iters", type=int, default=200)
    ap.add_argument("--batched-ttt", type=int, default=1,
                    help="1: also time the 64-instance batch to 1e-3 against one-at-a-time solves")
    ap.add_argument("--batched-ttt-max-iter", type=int, default=20000)
    ap.add_argument("--medium", type=int, default=1,
                    help="1: also time the Medium workload (FP32 and FP64, iterations/s and "
                         "time to tolerance)")
    ap.add_argument("--general", type=int, default=1,
                    help="1: also time the general line model (DC links, per-contingency changes)")
    ap.add_argument("--adjoint", type=int, default=1,
                    help="1: also time 1000 unrolled iterations forward + adjoint (diff workload)")
    ap.add_argument("--planning", type=int, default=0,
                    help="N > 0: time N steps of the planning loop over 8 scenarios")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-sample-k", type=int, default=3)
    ap.add_argument("--cpu-iters", type=int, default=8)
    ap.add_argument("--cpu-medium-iters", type=int, default=40)
    ap.add_argument("--tuning-cache", default=None,
                    help="autotuner cache file for the batched legs (read, and appended "
                         "to when a configuration is new)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="1: first run a plain 1 GiB -> 1 GiB copy kernel three times "
                         "(reference for the HBM byte counters)")
    ap.add_argument("--summarize-stats", nargs=3, metavar=("DIR", "OUT", "COMMAND"),
                    help="host only: summarise a rocprofv3 --stats run and exit")
    ap.add_argument("--summarize-traffic", nargs="+",
                    metavar="ARG",
                    help="host only: FETCH_DIR WRITE_DIR OUT KERNEL WORKLOAD CMD_FETCH "
                         "CMD_WRITE [REQUEST_DIR CMD_REQUEST]: HBM bytes per launch of the "
                         "kernels matching KERNEL ('|'-separated name fragments) from "
                         "the --pmc runs, then exit")
    args = ap.parse_args()

    if args.summarize_stats:
        summarize_stats(*args.summarize_stats)
        return
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the contingency-sharded multi-GPU design is not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2410_17203_amd import synth
    from paper_2410_17203_amd.binding import Solver

    global TUNING_CACHE
    TUNING_CACHE = args.tuning_cache
    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.calibrate_copy:
        x = torch.ones(2**28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        del x, y
        torch.cuda.empty_cache()
    t = time.perf_counter()
    inst = synth.config(args.config)
    log(f"[bench] instance {args.config} built in {time.perf_counter() - t:.1f}s")
    cfg = synth.CONFIGS[args.config]
    workload = (f"{args.config}: N={cfg['N']} L={cfg['L']} G={cfg['G']} D={cfg['D']} "
                f"B={cfg['B']} T={cfg['T']} K={cfg['K']} (synthetic, seed {cfg['seed']})")
    never = dict(eps=0.0, min_iter=2**31 - 1, max_iter=2**31 - 1)

    # ---- throughput of the FP32 (or FP64) iterate --------------------------
    s = Solver(inst, dtype=args.dtype, polish_fp64=0, **never)
    log(f"[bench] workspace {s.workspace_bytes / 2**30:.2f} GiB; warmup {args.warmup}, steps {args.steps}")
    elapsed, kt = time_iterations(s, args.steps, args.warmup)
    value = args.steps / elapsed
    prox = kt["sweep"]
    prox_ms = prox["ms"] / max(prox["launches"], 1)
    prox_bytes = s.kernel_bytes("sweep")
    # algorithmic bytes of the sweep's work: per contingency and period,
    # every line array read and written (10 L), three of them read again for
    # the node averages (3 L) and the node arrays (6 N), at S bytes each
    S = 4 if args.dtype == "f32" else 8
    alg_bytes = S * (inst.K + 1) * inst.T * (13 * inst.L + 6 * inst.N)
    achieved = alg_bytes / (prox_ms * 1e-3) / 1e9
    kernel_ms = {k: v["ms"] / max(v["launches"], 1) for k, v in kt.items()}
    iter_bytes = prox_bytes + s.kernel_bytes("devices")
    log(f"[bench] {value:.2f} it/s; kernel ms/launch {kernel_ms}")
    res = s.residuals()
    s.close()
    del s
    torch.cuda.empty_cache()

    extra = {}
    # ---- FP64 rate ---------------------------------------------------------
    if args.fp64_steps > 0 and args.dtype == "f32":
        s = Solver(inst, dtype="f64", **never)
        el64, kt64 = time_iterations(s, args.fp64_steps, 5)
        extra["fp64_iters_per_s"] = args.fp64_steps / el64
        p64 = kt64["sweep"]
        ms64 = p64["ms"] / max(p64["launches"], 1)
        extra["fp64_sweep_GBps"] = s.kernel_bytes("sweep") / (ms64 * 1e-3) / 1e9
        log(f"[bench] fp64 {extra['fp64_iters_per_s']:.2f} it/s")
        s.close()
        del s
        torch.cuda.empty_cache()

    # ---- time to tolerance (FP32 with FP64 polish, graph blocks) ----------
    if args.ttt and args.config == "large":
        # the same grid and horizon without contingencies: a problem the
        # reference dispatch certifies feasible under any reading of the
        # contingency model
        k0 = synth.config(args.config, K=0)
        s = Solver(k0, dtype=args.dtype, eps=1e-3, max_iter=args.ttt_max_iter)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve()
        torch.cuda.synchronize()
        extra["k0_time_to_tol_s"] = time.perf_counter() - t0
        extra["k0_time_to_tol_iters"] = r["iter"]
        extra["k0_time_to_tol_converged"] = r["status"] == "OPF_OK"
        log(f"[bench] K=0 solve: {r['status']} after {r['iter']} it in {extra['k0_time_to_tol_s']:.1f}s")
        s.close()
        del s, k0
        torch.cuda.empty_cache()
    if args.ttt:
        s = Solver(inst, dtype=args.dtype, eps=1e-3, max_iter=args.ttt_max_iter)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve()
        torch.cuda.synchronize()
        extra["time_to_tol_s"] = time.perf_counter() - t0
        extra["time_to_tol_iters"] = r["iter"]
        extra["time_to_tol_converged"] = r["status"] == "OPF_OK"
        extra["time_to_tol_final_rms"] = max(r["rms_primal"], r["rms_dual"])
        extra["time_to_tol_threshold"] = r["threshold"]
        log(f"[bench] solve: {r['status']} after {r['iter']} it in {extra['time_to_tol_s']:.1f}s")
        obj32 = r["objective"]
        s.close()
        del s
        torch.cuda.empty_cache()
        # the same solve with an FP64 iterate throughout, and with BF16-stored
        # phase duals; objectives compared with the FP64 one (the FP64 path is
        # the one pinned to the oracle)
        legs = [("fp64", dict(dtype="f64")),
                ("bf16_duals", dict(dtype="f32", dual_dtype="bf16", polish_fp64=0))]
        for label, kw in legs:
            s = Solver(inst, eps=1e-3, max_iter=args.ttt_max_iter, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = s.solve()
            torch.cuda.synchronize()
            extra[f"{label}_time_to_tol_s"] = time.perf_counter() - t0
            extra[f"{label}_time_to_tol_iters"] = r["iter"]
            extra[f"{label}_time_to_tol_converged"] = r["status"] == "OPF_OK"
            extra[f"{label}_objective"] = r["objective"]
            log(f"[bench] {label} solve: {r['status']} after {r['iter']} it in "
                f"{extra[f'{label}_time_to_tol_s']:.1f}s")
            s.close()
            del s
            torch.cuda.empty_cache()
        ref = extra["fp64_objective"]
        extra["time_to_tol_objective_rel_err_vs_fp64"] = abs(obj32 - ref) / abs(ref)
        extra["bf16_duals_objective_rel_err_vs_fp64"] = abs(extra["bf16_duals_objective"] - ref) / abs(ref)
        s = Solver(inst, dtype="f32", dual_dtype="bf16", polish_fp64=0, **never)
        el, kt = time_iterations(s, max(args.steps // 2, 1), 5)
        extra["bf16_duals_iters_per_s"] = max(args.steps // 2, 1) / el
        extra["bf16_duals_sweep_ms"] = kt["sweep"]["ms"] / max(kt["sweep"]["launches"], 1)
        log(f"[bench] bf16 duals {extra['bf16_duals_iters_per_s']:.2f} it/s")
        s.close()
        del s
        torch.cuda.empty_cache()

    if args.batched:
        extra["batched"] = [batched_rates(args.batched_iters, "f32", "f32"),
                            batched_rates(args.batched_iters, "f32", "bf16")]
        for b in extra["batched"]:
            log(f"[bench] batch of {b['instances']} ({b['dual_dtype']} duals): "
                f"{b['batched_inst_iters_per_s']:.0f} vs {b['one_at_a_time_inst_iters_per_s']:.0f} "
                f"instance-iterations/s one at a time, "
                f"{b['four_streams_inst_iters_per_s']:.0f} four at a time on their own streams")

    if args.batched_ttt:
        extra["batched_time_to_tol"] = batched_time_to_tolerance(args.batched_ttt_max_iter)
        b = extra["batched_time_to_tol"]
        log(f"[bench] batch to 1e-3: {b['batched_s']:.2f}s vs {b['one_at_a_time_s']:.2f}s one at a "
            f"time, {b['four_streams_s']:.2f}s four at a time; converged "
            f"{b['batched_converged']}/{b['instances']}")

    if args.medium:
        extra["medium"] = medium_leg()
        m = extra["medium"]
        log(f"[bench] medium: fp32 {m['f32']['iters_per_s']:.0f} it/s, fp64 {m['f64']['iters_per_s']:.0f} "
            f"it/s; to 1e-3 fp32+polish {m['f32']['time_to_tol_iters']} it in "
            f"{m['f32']['time_to_tol_s']:.3f}s, fp64 {m['f64']['time_to_tol_iters']} it in "
            f"{m['f64']['time_to_tol_s']:.3f}s")

    if args.planning > 0:
        extra["planning"] = planning_leg(args.planning)
        pl = extra["planning"]
        log(f"[bench] planning, {args.planning} steps: " + ", ".join(
            f"{k} {v['s']:.2f}s" for k, v in pl.items() if k.startswith("workers_")))

    if args.general:
        extra["general_line_model"] = general_model_rate(inst, 100, 10)
        g = extra["general_line_model"]
        log(f"[bench] general line model: {g['iters_per_s']:.2f} it/s, sweep {g['sweep_ms']:.3f} ms")

    if args.adjoint:
        # checkpoint interval chosen by the memory rule (every iterate kept
        # when the tape fits in a quarter of free HBM), and every 50th kept
        extra["adjoint"] = [adjoint_times(1000, None, "f32"), adjoint_times(1000, None, "f64"),
                            adjoint_times(1000, 50, "f32")]
        for a in extra["adjoint"]:
            log(f"[bench] adjoint {a['dtype']} (checkpoints every {a['checkpoint_every']}): forward {a['forward_plain_s']:.3f}s "
                f"(recorded {a['forward_recorded_s']:.3f}s), backward {a['backward_s']:.3f}s")

    khash = kernel_source_hash()
    traffic = traffic_from_profiles(khash, args.config, args.dtype)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 / value,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": workload, "residual_precision": "f64",
                   "adaptive_penalty": "every 10 iterations"},
        "roofline": {
            "bound": "hbm",
            "kernel": "sweep: line prox + node averages + price update, fused "
                      "(k_sweep_tile for this FP32 iterate)",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg_bytes,
            "algorithmic_model": "S*(K+1)*T*(13L+6N): line arrays read and written, three "
                                 "re-read for the averages, node arrays",
            "ms_per_launch": prox_ms,
            "stored_bytes_per_launch": prox_bytes,
            "stored_model": "S*(K+1)*T*(8L+6N): the arrays this design keeps, read and "
                            "written once (both phases as one mean, no re-read)",
            "frac_stored": prox_bytes / (prox_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "frac_counters": (None if traffic is None
                              else traffic / (prox_ms * 1e-3) / 1e9 / PEAK_HBM_GBS),
        },
        "kernel_ms_per_launch": kernel_ms,
        "iteration_algorithmic_GBps": iter_bytes / (1e-3 / value * 1e3) / 1e9,
        "final_rms": [res["rms_primal"], res["rms_dual"]],
        "kernel_source_hash": khash,
    }
    out.update(extra)
    if args.cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args.config, args.cpu_sample_k, args.cpu_iters,
                                           args.cpu_medium_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
