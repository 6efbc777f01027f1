#!/usr/bin/env python3
"""Benchmark of the randomized-CSE hot path on one MI355X.

A step is one pass of the whole path over the default workload, 32
synthetic schemes of uneven shape in one batch (65536 processes, pools
proportional to rank, sharing rounds): load every scheme from device-resident
int8 tensors (validation and input analysis on the device), run all of them
in one batched launch (each unit reduces U, V or W^T by Algorithm 1 with the
strategies of Sec. 3.4, the pools sharing every 32 steps as in Sec. 3.5.2),
read every unit's results.  K passes are timed back to back, bracketed by
device synchronisation.  The same passes run plain (one launch per scheme,
one after another) for the batched-vs-plain comparison.

Prints one JSON line: substitution steps per second over all units, time to
the best addition count per scheme, the roofline position of the step-kernel
class with the most device time (HIP events around each of its launches),
the CPU oracle timed on the host cores over a sample of units, and, as extra
keys, the 4x4x4, 6x6x6 and serving workloads.  --workload 4x4x4 | 6x6x6 |
serve | driver prints that workload's own line instead.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CSE substitution steps/s and time-to-best additions; batched vs plain, 1 GPU"
# int32 VALU lane operations per second of MI355X: 256 CUs x 4 SIMDs x 32
# lanes per clock x 2.4 GHz = 78.6 T, the rate behind the published 157.3
# TFLOP/s fp32 vector peak (an FMA counts as two flops).  32-bit integer
# adds issue at that rate: the VALU microbenchmark (csrc/cse_calib.hip)
# measures 69.4 T lane-op/s, one wave64 v_add_u32 per 2.2 clocks per SIMD.
PEAK_ALU_OPS = 256 * 4 * 32 * 2.4e9


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    counter summary profiles/step_kernel_<workload>_hbm_counters.txt
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy), or None when there
    is none for this kernel or the kernel sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"step_kernel_{workload}_hbm_counters.txt")
    try:
        with open(path) as f:
            fields = dict(l.split(": ", 1) for l in f.read().splitlines() if ": " in l)
    except OSError:
        return None
    if fields.get("kernel", "").strip() != kernel:
        return None
    h = hashlib.sha256()
    for name in ("cse_kernels.hpp", "cse_step.hip", "cse_api.hip"):
        with open(os.path.join(ROOT, "paper_2512_13365_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if fields.get("kernel_sources_sha256_16", "").strip() != h.hexdigest()[:16]:
        return None
    return int(fields["traffic_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def calibrate():
    """Measured on-chip peaks: 32-bit integer VALU issue (a full-occupancy
    grid of independent v_add_u32 chains, 128 per wave and iteration) and LDS
    read bandwidth (conflict-free ds_read_b128), from the microbenchmarks in
    csrc/cse_calib.hip, timed with HIP events."""
    import ctypes
    path = os.path.join(ROOT, "paper_2512_13365_amd", "libcse_calib.so")
    L = ctypes.CDLL(path)
    L.cse_calib_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_float),
                                ctypes.POINTER(ctypes.c_double)]
    L.cse_calib_run.restype = ctypes.c_int
    ms, work = ctypes.c_float(), ctypes.c_double()
    # VALU: 8 workgroups of 4 waves per CU (32 waves, the most a CU holds).
    blocks, iters = 256 * 8, 20000
    rc = L.cse_calib_run(0, blocks, iters, ctypes.byref(ms), ctypes.byref(work))
    if rc:
        raise RuntimeError(f"VALU microbenchmark failed: HIP error {rc}")
    valu_instr_s = blocks * 4 * work.value / (ms.value * 1e-3)
    valu = {"lane_ops_per_s": valu_instr_s * 64, "wave_instructions_per_s": valu_instr_s, "ms": ms.value,
            "grid": f"{blocks} x 256 lanes, {iters} iterations of 128 independent v_add_u32 per wave"}
    # LDS: 2 workgroups of 64 KiB per CU.
    blocks, iters = 256 * 2, 100000
    rc = L.cse_calib_run(1, blocks, iters, ctypes.byref(ms), ctypes.byref(work))
    if rc:
        raise RuntimeError(f"LDS microbenchmark failed: HIP error {rc}")
    lds = {"bytes_per_s": work.value / (ms.value * 1e-3), "ms": ms.value,
           "grid": f"{blocks} x 256 lanes, {iters} iterations of 8 ds_read_b128 per lane"}
    return {"valu": valu, "lds": lds}


def time_to_best(res, tick_hz):
    """Per component: (best cost, seconds from job start until a unit with
    that cost finished)."""
    out = []
    for r in res:
        best = int(r["cost"].min())
        t = min(int(f) for c, f in zip(r["cost"], r["finish"]) if c == best)
        out.append((best, t / tick_hz))
    return out


def cpu_baseline(systems, kw, n_threads, min_seconds=10.0, max_reps=50):
    """The oracle on the full workload, repeated until about min_seconds of
    CPU time have passed (a run of a few tenths of a second alone is noisy).
    Returns (substitutions, seconds, repetitions)."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import cse_oracle
    cfg = cse_oracle.make_cfg(**kw)
    steps, reps = 0, 0
    t0 = time.perf_counter()
    while reps < max_reps and (reps == 0 or time.perf_counter() - t0 < min_seconds):
        for c, A in enumerate(systems):
            r = cse_oracle.run_pool(A, cfg, comp=c, n_threads=n_threads)
            steps += int(r["executed"].sum())
        reps += 1
    return steps, time.perf_counter() - t0, reps


def job_results(cse, ctx, job, n_proc, n_comp=3):
    return [cse.cse_get_unit_results(ctx, job, c, n_proc) for c in range(n_comp)]


def base_line(args, **kw):
    out = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic"}
    out.update(kw)
    return out


def timed_relaunch(cse, ctx, job, stream, torch, steps, warmup):
    for _ in range(warmup):
        cse.cse_relaunch(ctx, job, None, stream)
    cse.cse_wait(ctx, job)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        cse.cse_relaunch(ctx, job, None, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    cse.cse_wait(ctx, job)
    return ev0.elapsed_time(ev1) / 1e3


def run_plain44(args, cse, workloads, torch, ctx, stream):
    wl = workloads.plain_4x4x4()
    sc, rs = wl.schemes[0], wl.runs[0]
    kw = rs.as_kwargs()
    kw["count_path"] = COUNT_PATHS[args.count_path]
    if args.strategy:
        kw["weights"] = {args.strategy: 1}
    sid = cse.cse_scheme_load(ctx, *sc.systems)
    info = cse.cse_scheme_info(ctx, sid)
    log(f"[bench] workload {wl.name}: shapes {[A.shape for A in sc.systems]} n_proc {rs.n_proc}")
    job = cse.cse_launch(ctx, sid, cse.cse_run_cfg(**kw), stream)
    cse.cse_wait(ctx, job)
    gpu_s = timed_relaunch(cse, ctx, job, stream, torch, args.steps, args.warmup)
    log(f"[bench] timed {args.steps} steps: {gpu_s * 1e3:.3f} ms device")
    # Host copy of every unit's results and program (PCIe), timed apart.
    t0 = time.perf_counter()
    res = job_results(cse, ctx, job, rs.n_proc)
    for c in range(3):
        cse.cse_get_programs(ctx, job, c, rs.n_proc, max(1, info[c][2]))
    readback_s = time.perf_counter() - t0
    _, tick_hz = cse.cse_job_timing(ctx, job)
    subs = sum(int(r["executed"].sum()) for r in res)
    ops = sum(int(r["ops"].sum()) for r in res)
    ttb = time_to_best(res, tick_hz)
    per_step = gpu_s / args.steps
    launches = 1  # one step-kernel launch covers the three components of the job
    avg_launch = per_step / launches
    achieved = (ops / launches) / avg_launch
    out = base_line(
        args, value=subs * args.steps / gpu_s, unit="substitution steps/s", ms_per_step=per_step * 1e3,
        config={"workload": "plain-4x4x4-r49: U,V 49x16, W^T 16x49 ternary, p=0.30, row nnz in [1,8]; "
                            + (f"4096 processes, {args.strategy} only" if args.strategy
                               else "4096 processes gi/ga/wr 1:1:1") + "; seed 0; no sharing",
                "n_proc": rs.n_proc, "units": 3 * rs.n_proc, "substitutions_per_step": subs},
        time_to_best_ms={"U": ttb[0][1] * 1e3, "V": ttb[1][1] * 1e3, "Wt": ttb[2][1] * 1e3,
                         "scheme": max(t for _, t in ttb) * 1e3},
        best_additions={"U": ttb[0][0], "V": ttb[1][0], "Wt": ttb[2][0], "scheme": sum(b for b, _ in ttb),
                        "naive": sum(i[3] for i in info)},
        pcie_inclusive={"readback_ms": readback_s * 1e3,
                        "steps_per_s": subs / (per_step + readback_s),
                        "note": "job plus host copy of all unit results and programs"},
        roofline={"kernel": "step_kernel<1, false, false, false, 1>", "bound": "alu", "achieved": achieved / 1e12,
                  "peak": PEAK_ALU_OPS / 1e12, "unit": "T int32 lane-op/s", "frac": achieved / PEAK_ALU_OPS,
                  "traffic": measured_traffic("step_kernel<1, false, false, false, 1>", "plain_4x4x4"),
                  "traffic_unit": "HBM bytes per launch",
                  "algorithmic_ops_per_launch": ops / launches,
                  "avg_launch_ms": avg_launch * 1e3})
    cse.cse_job_release(ctx, job)
    cse.cse_scheme_free(ctx, sid)
    if not args.no_cpu_baseline:
        n_threads = min(16, os.cpu_count() or 1)
        log(f"[bench] cpu oracle on {n_threads} threads (full workload)")
        steps, dt, reps = cpu_baseline(sc.systems, {k: v for k, v in kw.items() if k != "count_path"},
                                       n_threads)
        out["cpu_baseline"] = {"value": steps / dt, "unit": "substitution steps/s", "cores": n_threads,
                               "kind": "oracle",
                               "sample": f"the full workload ({rs.n_proc} processes x 3 components) {reps} times: "
                                         f"{steps} substitutions in {dt:.2f} s"}
    return out


BATCH_NAME = ("batch-32-uneven: 32 schemes, (n,m,p) uniform in {2..7}^3, r = round((nmp)^0.93), U r x nm, "
              "V r x mp, W^T np x r, ternary p = 0.2; pools proportional to r summing to 65536 processes; paper "
              "weights, proc0 = g; sharing every 32 steps, 1% -> 10%; inputs resident in HBM, each pass loads "
              "(validates and analyses) all 32 schemes on the device, runs them and reads every unit's results")


def kernel_name(W, layout):
    gs, adj, tl = bool(layout & 1), bool(layout & 2), bool(layout & 4)
    nw = 1 << ((layout >> 3) & 3)
    b = lambda x: "true" if x else "false"
    return f"step_kernel<{W}, {b(gs)}, {b(adj)}, {b(tl)}, {nw}>"


def scheme_pass(cse, ctx, stream, dev, cfgs, batched, layouts=None):
    """One pass over the batch: load every scheme from its device tensors
    (and give its components the layouts chosen before timing, if any), run
    the jobs (one batched launch, or one plain launch after another), read
    every unit's results, release.  Returns per-pass figures."""
    import numpy as np
    t0 = time.perf_counter()
    out = {"subs": 0, "best": [], "ttb_s": [], "per_class_ops": {}, "classes": {}}
    pending = []

    def collect(j, sid, n, t_start):
        best_total, ttb = 0, 0.0
        _, hz = cse.cse_job_timing(ctx, j)
        for c in range(3):
            r = cse.cse_get_unit_results(ctx, j, c, n)
            out["subs"] += int(r["executed"].sum())
            b = int(r["cost"].min())
            best_total += b
            ttb = max(ttb, min(int(f) for cc, f in zip(r["cost"], r["finish"]) if cc == b) / hz)
            rows = cse.cse_scheme_info(ctx, sid)[c][0]
            key = ((rows + 63) // 64, cse.cse_scheme_layout(ctx, sid, c))
            out["per_class_ops"][key] = out["per_class_ops"].get(key, 0) + int(r["ops"].sum())
        out["best"].append(best_total)
        out["ttb_s"].append(t_start + ttb)

    def load(i, d):
        sid = cse.cse_scheme_load_device(ctx, *d, stream=stream)
        if layouts is not None:
            for c, lay in enumerate(layouts[i]):
                cse.cse_scheme_layout(ctx, sid, c, lay)
        return sid

    if batched:
        sids = [load(i, d) for i, d in enumerate(dev)]
        t_launch = time.perf_counter() - t0
        jobs = cse.cse_launch_batch(ctx, sids, cfgs, stream)
        for j in jobs:
            cse.cse_wait(ctx, j)
        out["kernel_times"] = cse.cse_kernel_times(ctx, jobs[0], reset=True)
        for j, sid, cfg in zip(jobs, sids, cfgs):
            collect(j, sid, cfg.n_proc, t_launch)
        for j in jobs:
            cse.cse_job_release(ctx, j)
        for sid in sids:
            cse.cse_scheme_free(ctx, sid)
    else:
        for i, (d, cfg) in enumerate(zip(dev, cfgs)):
            t_start = time.perf_counter() - t0
            sid = load(i, d)
            j = cse.cse_launch(ctx, sid, cfg, stream)
            cse.cse_wait(ctx, j)
            collect(j, sid, cfg.n_proc, t_start)
            cse.cse_job_release(ctx, j)
            cse.cse_scheme_free(ctx, sid)
    torch_sync()
    out["seconds"] = time.perf_counter() - t0
    return out


def torch_sync():
    import torch
    torch.cuda.synchronize()


def cpu_baseline_batch(wl, n_threads, budget_s=10.0, seed=7):
    """The oracle on a seeded uniform sample of the batch's units (scheme,
    component, process), each reduced from its input to the end without the
    sharing rounds (which need the whole pool); units are started until
    budget_s has passed, then the running ones finish."""
    import numpy as np
    from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor, wait
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import cse_oracle
    rng = np.random.default_rng(seed)
    offs = np.cumsum([0] + [3 * rs.n_proc for rs in wl.runs])
    cfgs = [cse_oracle.make_cfg(**dict(rs.as_kwargs(), share_every=0)) for rs in wl.runs]

    def one(u):
        i = int(np.searchsorted(offs, u, side="right") - 1)
        c, p = divmod(int(u - offs[i]), wl.runs[i].n_proc)
        r = cse_oracle.run_pool(wl.schemes[i].systems[c], cfgs[i], comp=c, procs=[p])
        return int(r["executed"][0])

    steps, units = 0, 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(n_threads) as ex:
        live = set()
        for u in rng.permutation(int(offs[-1])):
            if time.perf_counter() - t0 >= budget_s:
                break
            if len(live) >= n_threads:
                done, live = wait(live, return_when=FIRST_COMPLETED)
                for f in done:
                    steps += f.result()
                    units += 1
            live.add(ex.submit(one, u))
        for f in live:
            steps += f.result()
            units += 1
    return steps, time.perf_counter() - t0, units


def run_batch(args, cse, workloads, torch, ctx, stream):
    import numpy as np
    wl = workloads.batch_uneven()
    dev = [tuple(torch.from_numpy(A).to("cuda") for A in sc.systems) for sc in wl.schemes]
    cfgs = [cse.cse_run_cfg(**rs.as_kwargs()) for rs in wl.runs]
    torch.cuda.synchronize()
    log(f"[bench] workload batch-32: {len(wl.schemes)} schemes, {sum(rs.n_proc for rs in wl.runs)} processes")
    # Component layouts (state placement, gi form, waves per unit) chosen
    # once by the autotuner, before any timed pass; every pass loads the
    # schemes afresh and gives them these layouts.
    layouts, tuning = None, {"mode": "default"}
    if args.layouts == "autotune":
        t_tune = time.perf_counter()
        sids = [cse.cse_scheme_load_device(ctx, *d, stream=stream) for d in dev]
        default = [[cse.cse_scheme_layout(ctx, sid, c) for c in range(3)] for sid in sids]
        layouts = [cse.cse_autotune(ctx, sid, cfg, stream) for sid, cfg in zip(sids, cfgs)]
        for sid in sids:
            cse.cse_scheme_free(ctx, sid)
        torch.cuda.synchronize()
        changed = sum(a != b for d, t in zip(default, layouts) for a, b in zip(d, t))
        tuning = {"mode": "cse_autotune once per scheme before the timed passes",
                  "seconds": time.perf_counter() - t_tune, "components_changed": changed,
                  "components": 3 * len(sids)}
        log(f"[bench] autotune: {changed} of {3 * len(sids)} component layouts changed in {tuning['seconds']:.1f} s")
    cse.cse_ctx_set_timing(ctx, True)
    for w in range(args.warmup):
        p = scheme_pass(cse, ctx, stream, dev, cfgs, True, layouts)
        log(f"[bench] warmup {w}: {p['seconds'] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    passes = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        passes.append(scheme_pass(cse, ctx, stream, dev, cfgs, True, layouts))
        log(f"[bench] batched pass {k}: {passes[-1]['seconds'] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    cse.cse_ctx_set_timing(ctx, False)
    plain = []
    for k in range(args.plain_passes):
        plain.append(scheme_pass(cse, ctx, stream, dev, cfgs, False, layouts))
        log(f"[bench] plain pass {k}: {plain[-1]['seconds'] * 1e3:.1f} ms")
    subs = sum(p["subs"] for p in passes)
    sec = [p["seconds"] for p in passes]
    # Roofline of the kernel class with the most device time.
    cls_ns, cls_launch, cls_ops = {}, {}, {}
    for p in passes:
        for kt in p["kernel_times"]:
            key = (kt["row_words"], kt["layout"])
            cls_ns[key] = cls_ns.get(key, 0) + kt["device_ns"]
            cls_launch[key] = cls_launch.get(key, 0) + kt["launches"]
        for key, v in p["per_class_ops"].items():
            cls_ops[key] = cls_ops.get(key, 0) + v
    dom = max(cls_ns, key=cls_ns.get)
    avg_launch_s = cls_ns[dom] / 1e9 / cls_launch[dom]
    ops_per_launch = cls_ops.get(dom, 0) / cls_launch[dom]
    achieved = ops_per_launch / avg_launch_s
    first = passes[0]
    out = base_line(
        args, value=subs / total, unit="substitution steps/s", ms_per_step=total / args.steps * 1e3,
        config={"workload": BATCH_NAME, "schemes": len(wl.schemes), "n_proc_total": sum(rs.n_proc for rs in wl.runs),
                "substitutions_per_step": first["subs"], "inputs_sha256": workloads.workload_digest(wl),
                "layouts": tuning},
        ms_per_step_median=float(np.median(sec)) * 1e3,
        time_to_best_ms={"mean_over_schemes": float(np.mean(first["ttb_s"])) * 1e3,
                         "max_over_schemes": float(np.max(first["ttb_s"])) * 1e3},
        batched_vs_plain={
            "plain": None if not plain else {
                "passes": len(plain), "seconds_median": float(np.median([p["seconds"] for p in plain])),
                "steps_per_s": plain[0]["subs"] / float(np.median([p["seconds"] for p in plain])),
                "mean_time_to_best_ms": float(np.mean(plain[0]["ttb_s"])) * 1e3,
                "max_time_to_best_ms": float(np.max(plain[0]["ttb_s"])) * 1e3},
            "speedup": None if not plain else float(np.median([p["seconds"] for p in plain])) / float(np.median(sec)),
            "identical_results": None if not plain else all(p["best"] == first["best"] for p in passes + plain),
            "scheme_best_additions": first["best"]},
        roofline={"kernel": kernel_name(*dom), "bound": "alu", "achieved": achieved / 1e12,
                  "peak": PEAK_ALU_OPS / 1e12, "unit": "T int32 lane-op/s", "frac": achieved / PEAK_ALU_OPS,
                  "traffic": measured_traffic(kernel_name(*dom), "batch"), "traffic_unit": "HBM bytes per launch",
                  "algorithmic_ops_per_launch": ops_per_launch, "avg_launch_ms": avg_launch_s * 1e3,
                  "launches": cls_launch[dom],
                  "device_ms_per_class": {kernel_name(*k): v / 1e6 / args.steps for k, v in sorted(cls_ns.items())}})
    if not args.no_cpu_baseline:
        n_threads = min(16, os.cpu_count() or 1)
        log(f"[bench] cpu oracle on {n_threads} threads (sample of units)")
        steps, dt, units = cpu_baseline_batch(wl, n_threads)
        out["cpu_baseline"] = {"value": steps / dt, "unit": "substitution steps/s", "cores": n_threads,
                               "kind": "oracle",
                               "sample": f"{units} units drawn uniformly (seeded) from the batch's "
                                         f"{3 * sum(rs.n_proc for rs in wl.runs)} (scheme, component, process) "
                                         f"units, each reduced from its input to the end without sharing rounds: "
                                         f"{steps} substitutions in {dt:.2f} s"}
    return out


COUNT_PATHS = {"auto": 0, "popcount": 1, "mfma": 2}


def run_6x6x6(args, cse, workloads, torch, ctx, stream):
    wl = workloads.plain_6x6x6()
    sc, rs = wl.schemes[0], wl.runs[0]
    sid = cse.cse_scheme_load(ctx, *sc.systems)
    info = cse.cse_scheme_info(ctx, sid)
    cfg = cse.cse_run_cfg(**rs.as_kwargs(), count_path=COUNT_PATHS[args.count_path])
    tuning = None
    if args.autotune:
        t0 = time.perf_counter()
        layouts = cse.cse_autotune(ctx, sid, cfg, stream)
        tuning = {"seconds": time.perf_counter() - t0, "layouts": layouts}
        log(f"[bench] autotune: layouts {layouts} in {tuning['seconds']:.1f} s")
    job = cse.cse_launch(ctx, sid, cfg, stream)
    cse.cse_wait(ctx, job)
    gpu_s = timed_relaunch(cse, ctx, job, stream, torch, args.steps, args.warmup)
    res = job_results(cse, ctx, job, rs.n_proc)
    _, tick_hz = cse.cse_job_timing(ctx, job)
    subs = sum(int(r["executed"].sum()) for r in res)
    ops = sum(int(r["ops"].sum()) for r in res)
    ttb = time_to_best(res, tick_hz)
    cse.cse_job_release(ctx, job)
    cse.cse_scheme_free(ctx, sid)
    per_job = gpu_s / args.steps
    achieved = ops / per_job
    return base_line(
        args, value=subs * args.steps / gpu_s, unit="substitution steps/s",
        ms_per_step=per_job * 1e3,
        roofline={"kernel": "step_kernel<3, true, true, false, 4> (U, V) and step_kernel<1, false, false, false, 1> (W^T); "
                            "achieved over the whole job, sharing rounds included",
                  "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_ALU_OPS / 1e12,
                  "unit": "T int32 lane-op/s", "frac": achieved / PEAK_ALU_OPS, "traffic": None,
                  "algorithmic_ops_per_job": ops, "job_ms": per_job * 1e3},
        config={"workload": "plain-6x6x6-r160: U,V 160x36, W^T 36x160, p=0.15, row nnz in [1,12]; 16384 "
                            "processes, paper weights, proc0 = g; sharing every 32 steps, 1% -> 10%",
                "n_proc": rs.n_proc, "substitutions_per_step": subs, "count_path": args.count_path,
                "autotune": tuning},
        time_to_best_ms={"U": ttb[0][1] * 1e3, "V": ttb[1][1] * 1e3, "Wt": ttb[2][1] * 1e3,
                         "scheme": max(t for _, t in ttb) * 1e3},
        best_additions={"U": ttb[0][0], "V": ttb[1][0], "Wt": ttb[2][0], "scheme": sum(b for b, _ in ttb),
                        "naive": sum(i[3] for i in info)})


def run_driver(args, cse, workloads, torch, ctx, stream):
    """The tool's outer iterations on the 4x4x4 (or 6x6x6) systems until the
    best total is unchanged for `patience` iterations (Sec. 3.5.1-3.5.2,
    Sec. 4)."""
    if args.driver_scheme == "6x6x6":
        wl = workloads.plain_6x6x6()
        kw = wl.runs[0].as_kwargs()
        name = ("driver-6x6x6-r160: U,V 160x36, W^T 36x160 as plain-6x6x6; 16384 processes, paper weights, "
                "proc0 = g, sharing every 32 steps 1% -> 10% inside each iteration")
    else:
        wl = workloads.plain_4x4x4()
        kw = dict(seed=0, n_proc=4096, weights=dict(workloads.PAPER_WEIGHTS), proc0_greedy=True)
        name = "driver-4x4x4-r49: U,V 49x16, W^T 16x49 as plain-4x4x4; 4096 processes, paper weights, proc0 = g"
    n_proc = kw["n_proc"]
    sc = wl.schemes[0]
    sid = cse.cse_scheme_load(ctx, *sc.systems)
    info = cse.cse_scheme_info(ctx, sid)
    cfg = cse.cse_run_cfg(**kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    job, its = cse.cse_run_driver(ctx, sid, cfg, stream, reinit_pm=400, patience=args.patience,
                                  max_iterations=100)
    wall = time.perf_counter() - t0
    totals, ns = cse.cse_driver_totals(ctx, job, elapsed=True)
    best = [cse.cse_driver_best(ctx, job, c) for c in range(3)]
    res = job_results(cse, ctx, job, n_proc)
    subs = sum(int(r["executed"].sum()) for r in res)
    cse.cse_job_release(ctx, job)
    cse.cse_scheme_free(ctx, sid)
    first_best = totals.index(totals[-1])
    log(f"[bench] driver: {its} iterations in {wall:.2f} s, totals {totals}")
    return base_line(
        args, value=subs / wall, unit="substitution steps/s", ms_per_step=None,
        config={"workload": f"{name}; iterations until the best total is unchanged for {args.patience}, "
                            "best-prefix restarts of 40%",
                "n_proc": n_proc, "reinit_pm": 400, "patience": args.patience},
        driver={"iterations": its, "wall_s": wall, "ms_per_iteration": wall / its * 1e3,
                "substitutions": subs, "totals": totals,
                "time_to_best_ms": ns[first_best] / 1e6, "best_found_at_iteration": first_best,
                "first_iteration_total": totals[0], "final_total": totals[-1],
                "naive": sum(i[3] for i in info),
                "best_additions": {n: b["cost"] for n, b in zip(("U", "V", "Wt"), best)},
                "best_iteration": {n: b["iteration"] for n, b in zip(("U", "V", "Wt"), best)}})


def run_serve(args, cse, workloads, torch, ctx, stream):
    """Poisson stream of jobs: a continuous-batching server vs one plain
    launch per job in arrival order; latency = completion - arrival."""
    import numpy as np
    wl = workloads.serving_stream(n_jobs=args.jobs)
    sids = [cse.cse_scheme_load(ctx, *sc.systems) for sc in wl.schemes]
    cfgs = [cse.cse_run_cfg(**rs.as_kwargs()) for rs in wl.runs]
    arr = wl.arrivals_s
    out = {}
    # Served.
    srv = cse.cse_server_create(ctx, max_state_bytes=args.serve_budget_gib << 30, round_steps=32, stream=stream)
    ids = {}
    t0 = time.perf_counter()
    nxt = 0
    done_t = {}
    steps = 0
    while len(done_t) < len(cfgs):
        now = time.perf_counter() - t0
        while nxt < len(cfgs) and arr[nxt] <= now:
            ids[nxt] = cse.cse_server_submit(srv, sids[nxt], cfgs[nxt])
            nxt += 1
        running, queued = cse.cse_server_tick(srv)
        now = time.perf_counter() - t0
        for i, j in list(ids.items()):
            if i in done_t:
                continue
            st, _ = cse.cse_server_job_info(srv, j)
            if st == cse.CSE_JOB_DONE:
                done_t[i] = now
                steps += sum(int(cse.cse_get_unit_results(ctx, j, c, cfgs[i].n_proc)["executed"].sum())
                             for c in range(3))
                cse.cse_server_release(srv, j)
                if len(done_t) % 50 == 0:
                    log(f"[bench] served {len(done_t)}/{len(cfgs)}")
        if running == 0 and queued == 0 and nxt < len(cfgs):
            time.sleep(max(0.0, arr[nxt] - (time.perf_counter() - t0)))
    wall = time.perf_counter() - t0
    cse.cse_server_destroy(srv)
    lat = np.array([done_t[i] - arr[i] for i in range(len(cfgs))])
    out["served"] = {"p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
                     "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
                     "steps_per_s": steps / wall, "wall_s": wall, "substitutions": steps}
    log(f"[bench] served: p50 {out['served']['p50_latency_ms']:.1f} ms p99 {out['served']['p99_latency_ms']:.1f} ms")
    # Plain per-job launches in arrival order.
    t0 = time.perf_counter()
    lat = []
    steps = 0
    for i, (sid, cfg) in enumerate(zip(sids, cfgs)):
        now = time.perf_counter() - t0
        if arr[i] > now:
            time.sleep(arr[i] - now)
        j = cse.cse_launch(ctx, sid, cfg, stream)
        cse.cse_wait(ctx, j)
        lat.append(time.perf_counter() - t0 - arr[i])
        steps += sum(int(cse.cse_get_unit_results(ctx, j, c, cfg.n_proc)["executed"].sum()) for c in range(3))
        cse.cse_job_release(ctx, j)
        if (i + 1) % 50 == 0:
            log(f"[bench] plain {i + 1}/{len(cfgs)}")
    wall = time.perf_counter() - t0
    lat = np.array(lat)
    out["plain"] = {"p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
                    "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
                    "steps_per_s": steps / wall, "wall_s": wall, "substitutions": steps}
    for s in sids:
        cse.cse_scheme_free(ctx, s)
    return base_line(
        args, value=out["served"]["steps_per_s"], unit="substitution steps/s",
        ms_per_step=None,
        config={"workload": f"serve-poisson: {args.jobs} jobs, exponential gaps mean 50 ms; (n,m,p) in "
                            "{2..8}^3, r=round((nmp)^0.93), p=0.12; 2048 processes per job, paper weights, "
                            "step cap 4000, sharing 32 steps 1% -> 10%"},
        serving=out)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch", choices=["batch", "4x4x4", "6x6x6", "serve", "driver"])
    ap.add_argument("--plain-passes", type=int, default=2, help="batch: plain passes (one launch per scheme)")
    ap.add_argument("--no-extras", action="store_true",
                    help="batch: skip the 4x4x4, 6x6x6 and serving lines added as extra keys")
    ap.add_argument("--patience", type=int, default=10, help="driver: iterations without improvement to stop")
    ap.add_argument("--driver-scheme", default="4x4x4", choices=["4x4x4", "6x6x6"], help="driver: which systems")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--strategy", default=None, choices=["g", "ga", "wr", "gr", "gi", "mix", "gp"],
                    help="4x4x4 only: every process uses this strategy (per-strategy cost)")
    ap.add_argument("--autotune", action="store_true", help="6x6x6: pick component layouts with cse_autotune first")
    ap.add_argument("--layouts", default="default", choices=["default", "autotune"],
                    help="batch: the loader's component layouts, or those cse_autotune picks once before timing")
    ap.add_argument("--count-path", default="auto", choices=list(COUNT_PATHS),
                    help="4x4x4 / 6x6x6: how the input's pair counts are computed (same results)")
    ap.add_argument("--jobs", type=int, default=200, help="serving: number of jobs of the stream")
    ap.add_argument("--serve-budget-gib", type=int, default=96, help="serving: device state budget")
    ap.add_argument("--calibrate-only", action="store_true",
                    help="only run the VALU and LDS microbenchmarks and print their line")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (reference for HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the CSE processes of a pool are independent; across GPUs a pool "
              "would shard by process index with one small all-gather of sharing keys per round",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2512_13365_amd import cse, workloads

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_calibrate:
        n = args.copy_calibrate * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {args.copy_calibrate} MiB read + {args.copy_calibrate} MiB written")
        del src, dst
    if args.calibrate_only:
        print(json.dumps({"measured_peaks": calibrate()}), flush=True)
        return
    ctx = cse.cse_ctx_create(0)
    try:
        if args.workload == "batch":
            out = run_batch(args, cse, workloads, torch, ctx, stream)
            if not args.no_extras:
                # The other workloads, each timed on its own, as extra keys.
                sub = argparse.Namespace(**dict(vars(args), no_cpu_baseline=True, steps=min(args.steps, 10),
                                                warmup=1, strategy=None, autotune=False))
                keep = ("value", "unit", "ms_per_step", "config", "time_to_best_ms", "best_additions", "roofline",
                        "serving", "pcie_inclusive")
                for name, fn in (("plain_4x4x4", run_plain44), ("plain_6x6x6", run_6x6x6),
                                 ("serving", run_serve)):
                    log(f"[bench] extra: {name}")
                    r = fn(sub, cse, workloads, torch, ctx, stream)
                    out[name] = {k: v for k, v in r.items() if k in keep}
        elif args.workload == "4x4x4":
            out = run_plain44(args, cse, workloads, torch, ctx, stream)
        elif args.workload == "6x6x6":
            out = run_6x6x6(args, cse, workloads, torch, ctx, stream)
        elif args.workload == "driver":
            out = run_driver(args, cse, workloads, torch, ctx, stream)
        else:
            out = run_serve(args, cse, workloads, torch, ctx, stream)
        if "roofline" in out:
            # Peaks measured on this GPU beside the derived ones (context).
            out["roofline"]["measured_peaks"] = calibrate()
            out["roofline"]["frac_of_measured_valu"] = (
                out["roofline"]["achieved"] * 1e12 / out["roofline"]["measured_peaks"]["valu"]["lane_ops_per_s"])
    finally:
        cse.cse_ctx_destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
