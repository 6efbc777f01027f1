#!/usr/bin/env python3
"""Benchmark of the randomized-CSE hot path on one MI355X.

A step is one whole job: every process of every component of the workload
(U, V and W^T) reduced until no pair repeats (Algorithm 1 with the
strategies of Sec. 3.4).  The default workload is the synthetic 4x4x4
rank-49 system (U, V 49x16, W^T 16x49, 4096 processes, gi / ga / wr in equal
shares).  Inputs are resident in HBM before the timed region; the timed
region is K back-to-back relaunches of the job on one stream, bracketed by
device synchronisation, timed with HIP events on that stream.

Prints one JSON line: substitution steps per second (all units), time to
the best addition count, the roofline position of the step kernel, the CPU
oracle timed on the host cores, and batched vs plain launches of 32 uneven
schemes.  Other workloads (--workload 6x6x6 | batch | serve) print their own
line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CSE substitution steps/s and time-to-best additions; batched vs plain, 1 GPU"
# int32 VALU lane operations per second of MI355X: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz (the 157.3 TFLOP/s fp32 vector peak counts an FMA as two
# flops and packed fp32 as two lanes).
PEAK_ALU_OPS = 256 * 4 * 16 * 2.4e9


def measured_traffic():
    """HBM bytes per step-kernel launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy), or None when the
    kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "step_kernel_plain_4x4x4_hbm_counters.txt")
    try:
        with open(path) as f:
            fields = dict(l.split(": ", 1) for l in f.read().splitlines() if ": " in l)
    except OSError:
        return None
    h = hashlib.sha256()
    for name in ("cse_kernels.hpp", "cse_api.hip"):
        with open(os.path.join(ROOT, "paper_2512_13365_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if fields.get("kernel_sources_sha256_16", "").strip() != h.hexdigest()[:16]:
        return None
    return int(fields["traffic_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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
        roofline={"kernel": "step_kernel<1, false, false, false>", "bound": "alu", "achieved": achieved / 1e12,
                  "peak": PEAK_ALU_OPS / 1e12, "unit": "T int32 lane-op/s", "frac": achieved / PEAK_ALU_OPS,
                  "traffic": measured_traffic(), "traffic_unit": "HBM bytes per launch",
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


def batch_vs_plain(cse, workloads, torch, ctx, stream, reps=1, autotune=False):
    """32 uneven schemes: one batched launch vs 32 sequential plain launches,
    same pools and seeds (so the same results).  With autotune, every
    component first gets its fastest layout from cse_autotune (timed apart)."""
    wl = workloads.batch_uneven()
    sids = [cse.cse_scheme_load(ctx, *sc.systems) for sc in wl.schemes]
    cfgs = [cse.cse_run_cfg(**rs.as_kwargs()) for rs in wl.runs]
    n_procs = [rs.n_proc for rs in wl.runs]
    stats = {}
    tuning = None
    if autotune:
        t0 = time.perf_counter()
        chosen = [cse.cse_autotune(ctx, s, c, stream) for s, c in zip(sids, cfgs)]
        tuning = {"seconds": time.perf_counter() - t0,
                  "layouts": [[x for x in ch if x >= 0] for ch in chosen]}
        log(f"[bench] autotune: {tuning['seconds']:.1f} s")
    for mode in ("batched", "plain"):
        best_t = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == "batched":
                jobs = cse.cse_launch_batch(ctx, sids, cfgs, stream)
                for j in jobs:
                    cse.cse_wait(ctx, j)
                starts = [0.0] * len(jobs)
            else:
                jobs, starts = [], []
                for s, c in zip(sids, cfgs):
                    starts.append(time.perf_counter() - t0)
                    j = cse.cse_launch(ctx, s, c, stream)
                    cse.cse_wait(ctx, j)
                    jobs.append(j)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            steps, bests, ttbs = 0, [], []
            for j, n, st in zip(jobs, n_procs, starts):
                res = job_results(cse, ctx, j, n)
                _, hz = cse.cse_job_timing(ctx, j)
                steps += sum(int(r["executed"].sum()) for r in res)
                tb = time_to_best(res, hz)
                bests.append(sum(b for b, _ in tb))
                ttbs.append(st + max(t for _, t in tb))
            for j in jobs:
                cse.cse_job_release(ctx, j)
            if best_t is None or dt < best_t:
                best_t = dt
                stats[mode] = {"seconds": dt, "substitutions": steps, "steps_per_s": steps / dt,
                               "mean_time_to_best_ms": 1e3 * sum(ttbs) / len(ttbs),
                               "max_time_to_best_ms": 1e3 * max(ttbs), "best_additions": bests}
        log(f"[bench] batch-32 {mode}: {stats[mode]['seconds'] * 1e3:.1f} ms, "
            f"{stats[mode]['steps_per_s'] / 1e6:.1f} M steps/s")
    for s in sids:
        cse.cse_scheme_free(ctx, s)
    same = stats["batched"]["best_additions"] == stats["plain"]["best_additions"]
    return {"workload": "batch-32-uneven: (n,m,p) in {2..7}^3, r=round((nmp)^0.93), p=0.2; pools ~ r summing "
                        "to 65536; paper weights; sharing 32 steps 1% -> 10%",
            "batched": {k: v for k, v in stats["batched"].items() if k != "best_additions"},
            "plain": {k: v for k, v in stats["plain"].items() if k != "best_additions"},
            "speedup": stats["batched"]["steps_per_s"] / stats["plain"]["steps_per_s"],
            "scheme_best_additions": stats["batched"]["best_additions"], "identical_results": same,
            "autotune": tuning}


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
        roofline={"kernel": "step_kernel<3, true, true, false> (U, V) and step_kernel<1, false, false, false> (W^T); "
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
    ap.add_argument("--workload", default="4x4x4", choices=["4x4x4", "6x6x6", "batch", "serve", "driver"])
    ap.add_argument("--patience", type=int, default=10, help="driver: iterations without improvement to stop")
    ap.add_argument("--driver-scheme", default="4x4x4", choices=["4x4x4", "6x6x6"], help="driver: which systems")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--strategy", default=None, choices=["g", "ga", "wr", "gr", "gi", "mix", "gp"],
                    help="4x4x4 only: every process uses this strategy (per-strategy cost)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched vs plain section")
    ap.add_argument("--autotune", action="store_true",
                    help="batch / 6x6x6: pick component layouts with cse_autotune first")
    ap.add_argument("--count-path", default="auto", choices=list(COUNT_PATHS),
                    help="4x4x4 / 6x6x6: how the input's pair counts are computed (same results)")
    ap.add_argument("--jobs", type=int, default=200, help="serving: number of jobs of the stream")
    ap.add_argument("--serve-budget-gib", type=int, default=96, help="serving: device state budget")
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
    ctx = cse.cse_ctx_create(0)
    try:
        if args.workload == "4x4x4":
            out = run_plain44(args, cse, workloads, torch, ctx, stream)
            if not args.no_batch:
                out["batched_vs_plain"] = batch_vs_plain(cse, workloads, torch, ctx, stream)
        elif args.workload == "6x6x6":
            out = run_6x6x6(args, cse, workloads, torch, ctx, stream)
        elif args.workload == "driver":
            out = run_driver(args, cse, workloads, torch, ctx, stream)
        elif args.workload == "batch":
            bp = batch_vs_plain(cse, workloads, torch, ctx, stream, reps=2, autotune=args.autotune)
            out = base_line(args, value=bp["batched"]["steps_per_s"], unit="substitution steps/s",
                            ms_per_step=None, config={"workload": bp["workload"]}, batched_vs_plain=bp)
        else:
            out = run_serve(args, cse, workloads, torch, ctx, stream)
    finally:
        cse.cse_ctx_destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
