#!/usr/bin/env python3
"""Benchmark of the batched AM trajectory optimizer on one MI355X.

One step = one pass of the whole hot path over one batch: the AM solve of
B = 1000 trajectories for K = 100 iterations (initial projection, then per
iteration xi1, trajectory evaluation, xi2, xi3/xi4 projections, multiplier
update) followed by the residual statistics, on synthetic inputs already in
HBM.  The metric is trajectory-AM-iterations per second (B*K per step).

Printed as one JSON line: throughput of the one-launch form, the plain form
(one launch per sub-step per iteration) beside it, the roofline of the
dominant kernel from HIP events around its launches, and the FP64 oracle
timed on the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3e12   # MI355X published FP32 vector peak [FLOP/s]
PEAK_HBM = 8.0e12             # MI355X HBM3E [B/s]


def flops_per_launch(q: int, nv: int, m: int, n: int, B: int, K: int) -> float:
    """Algorithmic floating-point operations of one fused solve (FMA = 2,
    add/mul/max/rsqrt/atan2/sincos = 1), counted from the iteration's
    arithmetic: 13 per (circle, obstacle, t) projection element, 10 per
    (circle, t), 38 + 38 nv per t (trajectory evaluation, heading step,
    velocity/acceleration projection, residual channels and the F^T
    reductions) and 34 nv^2 + 10 nv per trajectory (KKT applications,
    multiplier updates); the initial projection adds one projection pass."""
    per_iter = 13 * m * n * q + 10 * m * q + q * (38 + 38 * nv) + 34 * nv * nv + 10 * nv
    init = 13 * m * n * q + 10 * m * q + q * (30 + 34 * nv) + 16 * nv * nv
    return float(B) * (K * per_iter + init)


def bytes_per_launch(q: int, nv: int, m: int, n: int, B: int, K: int, esize: int = 4) -> float:
    """Algorithmic HBM bytes of one fused solve: state read and written once
    (5 nv coefficients, 5 nv multipliers), trajectory output 3q, obstacle
    table read once per block."""
    per_traj = (2 * 10 * nv + 3 * q) * esize
    return float(B) * per_traj + float((B + 3) // 4) * 2 * n * q * esize


def plain_bytes_per_iter(q: int, nv: int, m: int, n: int, B: int, esize: int = 4) -> float:
    """Algorithmic HBM bytes of one plain iteration: alpha, d written by the
    projection kernel and read by the target kernel (16 m n q per
    trajectory), plus the per-t channels (8 trajectory, 3 heading, 4 v/a,
    9 residual values written and read)."""
    return float(B) * (16 * m * n * q + 2 * (8 + 3 + 1 + 4 + 9) * q * esize)


def measured_traffic(workload: str):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE runs (scaled by the copy-kernel reference), or None
    when the kernel source has changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"fused_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def run_gpu(args):
    import torch

    from paper_2109_13030_amd import am, inputs

    cfg = inputs.CONFIGS[args.workload]
    pb, init = inputs.workload(args.workload)
    B, K = init["cx"].shape[0], cfg.iters
    m, n, q, nv = len(pb["r"]), len(pb["oa"]), pb["q"], pb["nv"]
    dtype = args.dtype
    torch.cuda.set_device(0)
    h = am.Handle.for_problem(pb, dtype)
    p = am.DeviceProblem(pb, dtype)
    stream = torch.cuda.current_stream()

    def make_states(count):
        return [am.DeviceState(init, m, n, q, dtype=dtype) for _ in range(count)]

    res_out = torch.empty((B, am.NRES), dtype=torch.float32 if dtype == "f32" else torch.float64, device="cuda")

    def timed(solver, steps, warmup):
        states = make_states(warmup + steps)
        for s in states[:warmup]:
            solver(s)
            am.residuals(h, p, s, out=res_out)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s, (e0, e1, e2) in zip(states[warmup:], ev):
            e0.record(stream)
            solver(s)
            e1.record(stream)
            am.residuals(h, p, s, out=res_out)
            e2.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        solve_ms = [a.elapsed_time(b) for a, b, _ in ev]
        step_ms = [a.elapsed_time(c) for a, _, c in ev]
        last = states[-1]
        return wall, solve_ms, step_ms, last

    fused = lambda s: am.solve(h, p, s, K)
    wall, solve_ms, step_ms, last = timed(fused, args.steps, args.warmup)
    res = am.residuals(h, p, last).cpu().numpy()
    ms_step = wall * 1e3 / args.steps
    value = B * K * args.steps / wall
    avg_kernel_s = float(np.mean(solve_ms)) * 1e-3
    flops = flops_per_launch(q, nv, m, n, B, K)
    achieved = flops / avg_kernel_s

    out = {
        "metric": "trajectory-AM-iterations/sec at batch 1000 vs plain; p99 replan latency",
        "value": value,
        "unit": "traj-AM-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: batch {B}, {m} circles (1.5x0.5 m robot), {n} moving "
                               f"elliptical obstacles, {q} timesteps, {nv} Bernstein coefficients, "
                               f"{K} AM iterations per solve + residuals",
                   "batch": B, "circles": m, "obstacles": n, "timesteps": q, "coefficients": nv,
                   "iterations": K},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR,
                     "traffic": measured_traffic(args.workload) if dtype == "f32" else None,
                     "kernel": "fused_kernel<float,11>", "kernel_ms": avg_kernel_s * 1e3,
                     "flop_per_launch": flops,
                     "hbm_bytes_per_launch": bytes_per_launch(q, nv, m, n, B, K)},
        "step_ms_events": float(np.mean(step_ms)),
        "final_residuals": {"fc_max_median": float(np.median(res[:, 0])),
                            "bc_max": float(res[:, 6].max()),
                            "nonfinite": int(res[:, 11].max())},
    }

    if not args.no_plain:
        ws = torch.empty(am.plain_workspace_size(h, B), dtype=torch.uint8, device="cuda")
        plain = lambda s: am.solve_plain(h, p, s, K, ws)
        psteps = max(2, min(args.steps, 10))
        pwall, psolve_ms, _, _ = timed(plain, psteps, 1)
        pvalue = B * K * psteps / pwall
        out["plain"] = {"value": pvalue, "ms_per_step": pwall * 1e3 / psteps,
                        "solve_ms_events": float(np.mean(psolve_ms)),
                        "launches_per_step": 6 * K + 7,
                        "fused_speedup": value / pvalue,
                        "hbm_bytes_per_iteration": plain_bytes_per_iter(q, nv, m, n, B)}
    return out, pb, init, K


def cpu_baseline(pb, init, K, seconds: float):
    """The FP64 oracle (tests' reference, untuned) on the host cores on a
    sample of the same workload's trajectories."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    orc = oracle.Oracle(pb)
    # calibrate on a few trajectories, then size the sample to ~`seconds`
    B = init["cx"].shape[0]
    probe = min(B, max(threads, 8))
    st = oracle.state_from(pb, {k: np.asarray(v)[:probe] for k, v in init.items()})
    t0 = time.perf_counter()
    orc.solve(st, K, nthreads=threads)
    dt = time.perf_counter() - t0
    per_traj = dt / probe
    sample = int(min(B, max(probe, seconds / max(per_traj, 1e-9))))
    st = oracle.state_from(pb, {k: np.asarray(v)[:sample] for k, v in init.items()})
    t0 = time.perf_counter()
    orc.solve(st, K, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": sample * K / dt, "unit": "traj-AM-iter/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sample} of {B} trajectories of the same workload, {K} iterations each, "
                      f"FP64, OpenMP over trajectories ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-ref", action="store_true",
                    help="run only a 512 MiB elementwise copy (y = x * 1), the size reference for "
                         "hardware byte counters, and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the batched AM solve has no cross-GPU step "
              "(trajectories are independent); run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.copy_ref:
        import torch
        x = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_ref_bytes_read": x.numel() * 4, "copy_ref_bytes_written": y.numel() * 4,
                          "launches": 3}))
        return
    out, pb, init, K = run_gpu(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pb, init, K, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
