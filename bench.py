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
the best addition count, the roofline position of the step kernel, and the
CPU oracle timed on the host cores.
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_to_best(res, tick_hz):
    """Per component: (best cost, seconds from job start until a unit with
    that cost finished); scheme total = sum of bests, latest of the times."""
    out = []
    for r in res:
        best = int(r["cost"].min())
        t = min(int(f) for c, f in zip(r["cost"], r["finish"]) if c == best)
        out.append((best, t / tick_hz))
    return out


def cpu_baseline(systems, kw, n_threads):
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import cse_oracle
    cfg = cse_oracle.make_cfg(**kw)
    steps = 0
    t0 = time.perf_counter()
    for c, A in enumerate(systems):
        r = cse_oracle.run_pool(A, cfg, comp=c, n_threads=n_threads)
        steps += int(r["executed"].sum())
    dt = time.perf_counter() - t0
    return steps, dt


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (reference for HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the CSE processes need no collective, and this build "
              "runs on a single MI355X (see the sharding notes in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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
    wl = workloads.plain_4x4x4()
    sc, rs = wl.schemes[0], wl.runs[0]
    kw = rs.as_kwargs()
    ctx = cse.cse_ctx_create(0)
    sid = cse.cse_scheme_load(ctx, *sc.systems)
    info = cse.cse_scheme_info(ctx, sid)
    cfg = cse.cse_run_cfg(**kw)
    log(f"[bench] workload {wl.name}: shapes {[A.shape for A in sc.systems]} n_proc {rs.n_proc}")

    job = cse.cse_launch(ctx, sid, cfg, stream)
    cse.cse_wait(ctx, job)
    for _ in range(args.warmup):
        cse.cse_relaunch(ctx, job, None, stream)
    cse.cse_wait(ctx, job)
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps)")

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        cse.cse_relaunch(ctx, job, None, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    cse.cse_wait(ctx, job)
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    log(f"[bench] timed {args.steps} steps: {gpu_s * 1e3:.3f} ms device, {wall * 1e3:.3f} ms host")

    res = [cse.cse_get_unit_results(ctx, job, c, rs.n_proc) for c in range(3)]
    _, tick_hz = cse.cse_job_timing(ctx, job)
    subs = sum(int(r["executed"].sum()) for r in res)
    ops = sum(int(r["ops"].sum()) for r in res)
    ttb = time_to_best(res, tick_hz)
    per_step = gpu_s / args.steps
    launches = 1  # one step-kernel launch covers the three components of the job
    avg_launch = per_step / launches
    achieved = (ops / launches) / avg_launch

    out = {
        "metric": METRIC,
        "value": subs * args.steps / gpu_s,
        "unit": "substitution steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "plain-4x4x4-r49: U,V 49x16, W^T 16x49 ternary, p=0.30, row nnz in [1,8]; "
                        "4096 processes gi/ga/wr 1:1:1; seed 0; no sharing",
            "n_proc": rs.n_proc,
            "units": 3 * rs.n_proc,
            "substitutions_per_step": subs,
        },
        "time_to_best_ms": {
            "U": ttb[0][1] * 1e3, "V": ttb[1][1] * 1e3, "Wt": ttb[2][1] * 1e3,
            "scheme": max(t for _, t in ttb) * 1e3,
        },
        "best_additions": {"U": ttb[0][0], "V": ttb[1][0], "Wt": ttb[2][0],
                           "scheme": sum(b for b, _ in ttb),
                           "naive": sum(i[3] for i in info)},
        "roofline": {
            "kernel": "step_kernel<1, false>",
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_ALU_OPS / 1e12,
            "unit": "T int32 lane-op/s",
            "frac": achieved / PEAK_ALU_OPS,
            "traffic": None,
            "algorithmic_ops_per_launch": ops / launches,
            "avg_launch_ms": avg_launch * 1e3,
        },
    }

    if not args.no_cpu_baseline:
        n_threads = min(16, os.cpu_count() or 1)
        log(f"[bench] cpu oracle on {n_threads} threads (full workload)")
        steps, dt = cpu_baseline(sc.systems, kw, n_threads)
        out["cpu_baseline"] = {"value": steps / dt, "unit": "substitution steps/s", "cores": n_threads,
                               "kind": "oracle",
                               "sample": f"full workload: {rs.n_proc} processes x 3 components, "
                                         f"{steps} substitutions in {dt:.2f} s"}
    cse.cse_job_release(ctx, job)
    cse.cse_scheme_free(ctx, sid)
    cse.cse_ctx_destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
