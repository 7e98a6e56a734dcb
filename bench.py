#!/usr/bin/env python3
"""Benchmark of the batched AM trajectory optimizer on one MI355X.

One step = one pass of the whole hot path over one batch: the AM solve of
B = 1000 trajectories for K = 100 iterations (initial projection, then per
iteration xi1, trajectory evaluation, xi2, xi3/xi4 projections, multiplier
update) and the residual statistics of the final state, which the solve
forms itself, on synthetic inputs already in HBM.  The metric is
trajectory-AM-iterations per second (B*K per step).

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
N_CU, CLOCK_HZ = 256, 2.4e9   # compute units and peak engine clock


def flops_per_traj_iter(q: int, nv: int, m: int, n: int) -> float:
    """Algorithmic floating-point work of one trajectory-iteration of the
    method: ~60 per (circle, obstacle, t) element of the xi3/xi4 closed forms
    (offsets, scaled norm, angle, distance, target, residual and its share of
    the reduction) and ~4.4e4 for the dense steps at q = 100, nv = 11 (F^T g,
    the KKT applications, trajectory evaluation, heading step, F^T F xi)."""
    return 60.0 * m * n * q + 4.4e4


def flops_per_launch(q: int, nv: int, m: int, n: int, B: int, K: int) -> float:
    """Algorithmic flops of one solve: B K trajectory-iterations."""
    return float(B) * K * flops_per_traj_iter(q, nv, m, n)


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


# Files the fused kernel is compiled from; counters taken on an older build
# of any of them no longer describe the kernel.
FUSED_SOURCES = ["paper_2109_13030_amd/csrc/am_fused.hip", "paper_2109_13030_amd/csrc/am_device.h",
                 "paper_2109_13030_amd/csrc/am_internal.h", "paper_2109_13030_amd/csrc/am_poly.h",
                 "include/am.h"]


def kernel_sources_sha256(sources) -> str:
    """SHA-256 over the concatenated bytes of the given repository files."""
    import hashlib
    h = hashlib.sha256()
    for rel in sources:
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE runs (scaled by the copy-kernel reference), or None
    when the kernel source has changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"fused_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if kernel_sources_sha256(rec["sources"]) != rec["sources_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def measured_valu(workload: str):
    """VALU wave-instructions per launch of the fused kernel from the
    committed rocprofv3 SQ_INSTS_VALU run, or None when the kernel source has
    changed since."""
    path = os.path.join(ROOT, "profiles", f"fused_{workload}_valu.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if kernel_sources_sha256(rec["sources"]) != rec["sources_sha256"]:
        return None
    return rec["sq_insts_valu_per_launch"]


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
        return [am.DeviceState(init, m, n, q, dtype=dtype, residuals=True) for _ in range(count)]

    def timed(solver, steps, warmup):
        states = make_states(warmup + steps)
        for s in states[:warmup]:
            solver(s)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s, (e0, e1) in zip(states[warmup:], ev):
            e0.record(stream)
            solver(s)
            e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        solve_ms = [a.elapsed_time(b) for a, b in ev]
        last = states[-1]
        return wall, solve_ms, solve_ms, last

    # launch configuration (tile, register budget): the library's autotuner
    # times each once per shape (setup, not timed)
    (tile, waves), tile_ms = am.autotune(h, p, make_states(1)[0], K)
    fused = lambda s: am.solve(h, p, s, K)
    wall, solve_ms, step_ms, last = timed(fused, args.steps, args.warmup)
    res = last.t["res"].cpu().numpy()
    ms_step = wall * 1e3 / args.steps
    value = B * K * args.steps / wall
    avg_kernel_s = float(np.mean(solve_ms)) * 1e-3
    flops = flops_per_launch(q, nv, m, n, B, K)
    achieved = flops / avg_kernel_s
    valu = measured_valu(args.workload) if dtype == "f32" else None

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
                     "kernel": f"fused_kernel<{'float' if dtype == 'f32' else 'double'},{nv},"
                               f"{5 if m <= 5 and dtype == 'f32' else 8},{tile},{waves}>",
                     "kernel_ms": avg_kernel_s * 1e3, "tile": tile, "waves_per_simd": waves,
                     "autotune_ms": {f"tile{k[0]}_waves{k[1]}": round(v, 4) for k, v in tile_ms.items()},
                     "flop_per_launch": flops,
                     "flop_per_traj_iter": flops_per_traj_iter(q, nv, m, n),
                     "valu_insts_per_launch": valu,
                     "valu_issue_frac": (valu / (N_CU * CLOCK_HZ * avg_kernel_s)) if valu else None,
                     "hbm_bytes_per_launch": bytes_per_launch(q, nv, m, n, B, K)},
        "step_ms_events": float(np.mean(step_ms)),
        "step_ms_median": float(np.median(step_ms)),
        "solve_ms_median": float(np.median(solve_ms)),
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
    out["_final"] = last.numpy()
    return out, pb, init, K


def run_serving(rates, n_requests, modes=("continuous", "plain"), n_clients: int = 32,
                saturation: int = 64, budget: int = 4 << 30, seed: int = 5, max_rate=None, streams: int = 2):
    """Replanning workload c5 through the continuous-batching server: Poisson
    arrivals, per request B ~ U{256..2048}, n ~ U{5..30} moving obstacles,
    5 circles, 20 warm-started AM iterations.  Latency = completion seen by
    the server's scheduler - submission.  Modes: continuous batching (all
    admissible pending requests of one shape per launch, up to `streams`
    launches in flight: two measured best against one and four, at 2-3 kHz
    and in bursts), sequential (the same fused kernel, one request per launch, one
    launch at a time) and plain (one request at a time on the per-sub-step
    path).  max_rate[mode] skips the rates a mode cannot sustain.  Also a
    saturation run (all requests submitted at once) for capacity."""
    import torch

    from paper_2109_13030_amd import am, inputs

    torch.cuda.set_device(0)
    cfg = inputs.CONFIGS["c5"]
    K = cfg.iters
    clients = inputs.serving_clients(n_clients)
    mode_ids = {"continuous": am.SERVE_CONTINUOUS, "sequential": am.SERVE_SEQUENTIAL, "plain": am.SERVE_PLAIN}
    out = {"workload": "c5: Poisson replanning requests, B ~ U{256..2048}, n ~ U{5..30} moving obstacles, "
                       f"5 circles, {K} warm-started AM iterations per request, {n_clients} robots",
           "iterations": K, "budget_bytes": budget, "modes": {}}

    def one(mode, rate, count, rseed):
        # the scheduler polls for 20 ms after its last activity (longer than
        # the mean gap between arrivals at 50-200 Hz), so arrivals do not
        # wait for a thread wake-up
        rng = np.random.default_rng(rseed)
        # fresh samples per request, drawn before the server starts from a
        # pool of four sets per robot (drawing them inside the arrival loop
        # would limit the submission rate)
        pools = [[inputs.make_initial(inputs.replan_problem(c["problem"], 1), c["batch"],
                                      int(rng.integers(1 << 31)), cfg.sigma) for _ in range(4)] for c in clients]
        srv = am.Server(budget, streams=streams, max_per_launch=64, mode=mode_ids[mode], idle_spin_us=20000)
        steps = [0] * len(clients)
        # every robot's first (cold) request is served before the timed run;
        # requests name their shape and the server's KKT cache supplies the
        # handle (built on the first request of each shape)
        first = [srv.submit(None, c["problem"], i, c["batch"], K, c["init"])
                 for i, c in enumerate(clients)]
        for t in first:
            if not srv.wait(t, 120.0)[0]:
                raise RuntimeError("a serving request did not finish within 120 s")
        arr = inputs.poisson_arrivals(rate, count, rseed) if rate else np.zeros(count)
        work, tickets = 0, []
        t0 = time.perf_counter()
        t_note = t0
        for ta in arr:
            if time.perf_counter() - t_note > 60.0:
                t_note = time.perf_counter()
                print(f"serving {mode} {rate:g} Hz: {len(tickets)} of {count} requests submitted",
                      file=sys.stderr, flush=True)
            while True:
                now = time.perf_counter() - t0
                if now >= ta:
                    break
                time.sleep(min(ta - now, 2e-4))
            i = int(rng.integers(len(clients)))
            c = clients[i]
            steps[i] += 1
            pb = inputs.replan_problem(c["problem"], steps[i])
            init = pools[i][steps[i] % 4]
            tickets.append(srv.submit(None, pb, i, c["batch"], K, init))
            work += c["batch"] * K
        lat = []
        for t in tickets:
            done, l, _ = srv.wait(t, 120.0)
            if not done:
                raise RuntimeError("a serving request did not finish within 120 s")
            lat.append(l)
        lat = np.array(lat)
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        launches = st["launches"] - len(clients)
        return {"rate_hz": rate, "requests": count, "requests_per_launch": count / max(launches, 1),
                "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
                "max_ms": float(lat.max() * 1e3), "traj_iter_per_s": work / wall,
                "launches": launches, "memory_waits": st["memory_waits"],
                "peak_bytes": st["peak_bytes"]}

    for mode in modes:
        rows = []
        for r in rates:
            if max_rate and mode in max_rate and r > max_rate[mode]:
                continue
            count = n_requests(r) if callable(n_requests) else n_requests
            rows.append(one(mode, r, count, seed + int(r)))
            print(f"serving {mode} {r:g} Hz: p50 {rows[-1]['p50_ms']:.3f} ms p99 {rows[-1]['p99_ms']:.3f} ms",
                  file=sys.stderr, flush=True)
        if saturation:
            rows.append(one(mode, 0, saturation, seed))
        out["modes"][mode] = rows
    return out


def run_uneven(reps: int = 3, count: int | None = None):
    """Uneven multi-problem workload c3: 64 independent problems (B ~
    U{64..1024}, 3-5 circles, 2-20 obstacles, K = 100) solved (a) one problem
    at a time on the plain path, (b) one fused launch per problem, (c) all in
    one multi-problem launch, (d) that launch captured in a HIP graph and
    replayed.  Returns trajectory-iterations per second of each."""
    import torch

    from paper_2109_13030_amd import am, inputs

    torch.cuda.set_device(0)
    cfg = inputs.CONFIGS["c3"]
    K = cfg.iters
    probs = inputs.uneven_problems("c3", count=count)
    hs = [am.Handle.for_problem(pb, "f32") for pb, _ in probs]
    dps = [am.DeviceProblem(pb, "f32") for pb, _ in probs]
    mk = lambda: [am.DeviceState(init, len(pb["r"]), len(pb["oa"]), pb["q"], "f32") for pb, init in probs]
    work = sum(init["cx"].shape[0] for _, init in probs) * K
    stream = torch.cuda.current_stream()

    def timeit(fn, reps_):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps_):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps_ * 1e-3

    out = {"workload": f"c3: {len(probs)} problems, batch U{{64..1024}} (total {work // K}), 3-5 circles, "
                       f"2-20 moving obstacles, {K} iterations", "traj_iter_per_launch": work}
    sts = mk()
    wss = [torch.empty(am.plain_workspace_size(h, s_.B), dtype=torch.uint8, device="cuda") for h, s_ in zip(hs, sts)]
    t = timeit(lambda: [am.solve_plain(h, p, s_, K, w) for h, p, s_, w in zip(hs, dps, sts, wss)], 1)
    out["plain_per_problem"] = {"s": t, "traj_iter_per_s": work / t}
    del wss
    t = timeit(lambda: [am.solve(h, p, s_, K) for h, p, s_ in zip(hs, dps, sts)], reps)
    out["fused_per_problem"] = {"s": t, "traj_iter_per_s": work / t}
    ws = torch.empty(am.multi_workspace_size(len(probs)), dtype=torch.uint8, device="cuda")
    t = timeit(lambda: am.solve_multi(hs, dps, sts, K, ws), reps)
    out["one_launch"] = {"s": t, "traj_iter_per_s": work / t}
    best, times = am.autotune_multi(hs, dps, mk(), K, ws)
    out["autotune"] = {"best": {"tile": best[0], "waves_per_simd": best[1]},
                       "ms": {f"tile{k[0]}_waves{k[1]}": v for k, v in times.items()}}
    t = timeit(lambda: am.solve_multi(hs, dps, sts, K, ws), reps)
    out["one_launch_tuned"] = {"s": t, "traj_iter_per_s": work / t, "tile": best}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        am.solve_multi(hs, dps, sts, K, ws)
    t = timeit(g.replay, reps)
    out["one_launch_graph"] = {"s": t, "traj_iter_per_s": work / t, "tile": best}
    out["speedup_one_launch_vs_plain"] = out["one_launch"]["traj_iter_per_s"] / out["plain_per_problem"]["traj_iter_per_s"]
    # error of one tuned launch against the FP64 oracle on the first 4
    # trajectories of every 8th problem
    import oracle
    chk = mk()
    am.solve_multi(hs, dps, chk, K, ws)
    torch.cuda.synchronize()
    errs = []
    for (pb, init), s_ in list(zip(probs, chk))[::8]:
        pb, sub = inputs.as_stored(pb, {k: np.asarray(v)[:4] for k, v in init.items()}, "f32")
        o = oracle.Oracle(pb)
        ost = oracle.state_from(pb, sub)
        o.solve(ost, K)
        P, _, _ = oracle.basis(pb["q"], pb["nv"], pb["tf"])
        g = s_.numpy()
        e = np.zeros(4)
        for k in ("cx", "cy", "cpsi"):
            e = np.maximum(e, np.abs(g[k][:4] @ P.T - ost[k] @ P.T).max(axis=1))
        errs.extend(e.tolist())
    errs = np.array(errs)
    out["error_vs_oracle"] = {"trajectories": int(errs.size), "max_err": float(errs.max()),
                              "median_err": float(np.median(errs)), "within_1e-3": int((errs <= 1e-3).sum())}
    return out


def run_precision(sample: int = 24, steps: int = 3):
    """Precision workload c4 (B = 4096, 5 circles, 20 moving obstacles,
    K = 100): the one-launch FP32 solve, the plain FP32 path and the plain
    path with the BF16 split contraction, each timed and compared with the
    FP64 oracle (run on the FP32 input values) on a sample of trajectories
    (max |dx|, |dy| in m and |dpsi| in rad)."""
    import torch

    import oracle
    from paper_2109_13030_amd import am, inputs

    torch.cuda.set_device(0)
    pb, init = inputs.workload("c4")
    K = inputs.CONFIGS["c4"].iters
    B, m, n, q = init["cx"].shape[0], len(pb["r"]), len(pb["oa"]), pb["q"]
    idx = np.unique(np.linspace(0, B - 1, sample).astype(int))
    sub = {k: np.asarray(v)[idx] for k, v in init.items()}
    # FP64 oracle on the sample, on the values the FP32 arrays hold
    P, _, _ = oracle.basis(q, pb["nv"], pb["tf"])
    pb32, sub32 = inputs.as_stored(pb, sub, "f32")
    o = oracle.Oracle(pb32)
    ost = oracle.state_from(pb32, sub32)
    o.solve(ost, K)
    ox, oy, op = ost["cx"] @ P.T, ost["cy"] @ P.T, ost["cpsi"] @ P.T
    out = {"workload": f"c4: batch {B}, {m} circles, {n} moving obstacles, {q} timesteps, {K} iterations",
           "sample": int(len(idx))}
    p = am.DeviceProblem(pb, "f32")
    stream = torch.cuda.current_stream()
    for name, flags, plain in (("fused_fp32", 0, False), ("plain_fp32", 0, True),
                               ("plain_bf16x3", am.PLAIN_BF16X3, True)):
        h = am.Handle.for_problem(dict(pb, flags=flags), "f32")
        states = [am.DeviceState(init, m, n, q, "f32") for _ in range(steps + 1)]
        ws = torch.empty(am.plain_workspace_size(h, B), dtype=torch.uint8, device="cuda") if plain else None
        run = (lambda s_: am.solve_plain(h, p, s_, K, ws)) if plain else (lambda s_: am.solve(h, p, s_, K))
        run(states[0])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for s_ in states[1:]:
            run(s_)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3 / steps
        res = states[-1].numpy()
        gx, gy, gp = res["cx"][idx] @ P.T, res["cy"][idx] @ P.T, res["cpsi"][idx] @ P.T
        epos = np.maximum(np.abs(gx - ox).max(1), np.abs(gy - oy).max(1))
        epsi = np.abs(gp - op).max(1)
        out[name] = {"ms_per_solve": sec * 1e3, "traj_iter_per_s": B * K / sec,
                     "max_pos_err_m": float(epos.max()), "max_psi_err_rad": float(epsi.max()),
                     "within_1e-3": int(((epos <= 1e-3) & (epsi <= 1e-3)).sum())}
        del ws
    return out


def cpu_baseline(pb, init, K, seconds: float):
    """The FP64 oracle (the tests' reference, untuned; built -O3 -march=native
    from the same source) on the host cores: the workload's trajectories,
    as many of them as fit in about `seconds` with OpenMP over trajectories,
    one thread on 16 of them, and config c1 (B = 16, K = 50) in full.  The
    oracle runs on the values the FP32 device arrays hold, and its final
    state is returned for the error check."""
    import oracle
    from paper_2109_13030_amd import inputs
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    pb, init = inputs.as_stored(pb, init, "f32")
    orc = oracle.Oracle(pb, native=True)
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
    rec = {"value": sample * K / dt, "unit": "traj-AM-iter/s", "cores": threads, "kind": "oracle",
           "sample": f"first {sample} of {B} trajectories of the same workload, {K} iterations each, "
                     f"FP64, OpenMP over trajectories ({dt:.1f} s)", "build": oracle.NATIVE_FLAGS}
    # one thread on a few trajectories, and what the host is
    few = min(B, 16)
    st1 = oracle.state_from(pb, {k: np.asarray(v)[:few] for k, v in init.items()})
    t0 = time.perf_counter()
    orc.solve(st1, K, nthreads=1)
    rec["single_thread_value"] = few * K / (time.perf_counter() - t0)
    rec["single_thread_sample"] = f"first {few} trajectories, one thread"
    # config c1 in full (B = 16, 3 circles, 4 static obstacles, K = 50)
    pb1, init1 = inputs.workload("c1")
    K1 = inputs.CONFIGS["c1"].iters
    o1 = oracle.Oracle(pb1, native=True)
    for nth, key in ((threads, "c1_value"), (1, "c1_single_thread_value")):
        s1 = oracle.state_from(pb1, init1)
        t0 = time.perf_counter()
        o1.solve(s1, K1, nthreads=nth)
        rec[key] = init1["cx"].shape[0] * K1 / (time.perf_counter() - t0)
    rec["cpu_model"] = cpu_model()
    rec["nproc"] = os.cpu_count()
    return rec, st


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def error_vs_oracle(pb, gpu: dict, orc_state: dict):
    """Max |dx|, |dy| [m] and |dpsi| [rad] of the GPU's final trajectories
    against the FP64 oracle's on the oracle's sample (the oracle run on the
    FP32 input values the GPU received)."""
    import oracle
    P, _, _ = oracle.basis(int(pb["q"]), int(pb["nv"]), float(pb["tf"]))
    S = orc_state["cx"].shape[0]
    ex = np.abs(gpu["cx"][:S] @ P.T - orc_state["cx"] @ P.T).max(1)
    ey = np.abs(gpu["cy"][:S] @ P.T - orc_state["cy"] @ P.T).max(1)
    ep = np.abs(gpu["cpsi"][:S] @ P.T - orc_state["cpsi"] @ P.T).max(1)
    e = np.maximum(np.maximum(ex, ey), ep)
    return {"trajectories": int(S), "max_pos_err_m": float(max(ex.max(), ey.max())),
            "max_psi_err_rad": float(ep.max()), "median_err": float(np.median(e)),
            "within_1e-3": int((e <= 1e-3).sum())}


def fixed_cost(workload: str = "c2", solves: int = 35):
    """Time per fused solve with solves issued back to back (as the
    benchmark's steps are) for K = 0, 1, 2 and the workload's K, without and
    with the residual statistics: the difference between K and 0 is the
    iterations' cost, the K = 0 time the set-up, first projection,
    write-back and the gap between launches."""
    import torch

    from paper_2109_13030_amd import am, inputs
    torch.cuda.set_device(0)
    cfg = inputs.CONFIGS[workload]
    pb, init = inputs.workload(workload)
    h = am.Handle.for_problem(pb, "f32")
    p = am.DeviceProblem(pb, "f32")
    m, n, q = len(pb["r"]), len(pb["oa"]), pb["q"]
    am.autotune(h, p, am.DeviceState(init, m, n, q, "f32"), cfg.iters)
    rows = []
    for res in (False, True):
        for K in (0, 1, 2, cfg.iters):
            sts = [am.DeviceState(init, m, n, q, "f32", residuals=res) for _ in range(solves + 5)]
            for st in sts[:5]:
                am.solve(h, p, st, K)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for st in sts[5:]:
                am.solve(h, p, st, K)
            e1.record()
            torch.cuda.synchronize()
            rows.append({"residuals": res, "K": K, "us_per_solve": e0.elapsed_time(e1) / solves * 1e3})
            print(f"residuals={res} K={K}: {rows[-1]['us_per_solve']:.2f} us", file=sys.stderr, flush=True)
    return {"workload": workload, "batch": int(init["cx"].shape[0]), "solves_back_to_back": solves,
            "launch": {"tile": h.tile, "waves_per_simd": h.waves}, "rows": rows}


def copy_by_size(launches=200):
    """Bandwidth of a plain elementwise copy (half the bytes read, half
    written) for the byte counts one launch of the plain path's elementwise
    kernels moves (their algorithmic bytes at c2 and c4), launched back to
    back like the plain path's kernels: what an elementwise launch of that
    size reaches on this GPU."""
    import torch
    out = []
    for label, moved in (("c2 k_targets", 30.0e6), ("c2 k_project", 44.8e6),
                         ("c4 k_targets", 204.8e6), ("c4 k_project", 347.4e6)):
        n = int(moved / 8)
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            torch.mul(x, 1.0, out=y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(launches):
            torch.mul(x, 1.0, out=y)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / launches * 1e3
        out.append({"size_of": label, "bytes_moved": 8 * n, "us_per_launch": us,
                    "TBps": 8 * n / (us * 1e-6) / 1e12})
        print(f"copy {label}: {us:.2f} us, {out[-1]['TBps']:.2f} TB/s", file=sys.stderr, flush=True)
        del x, y
    return {"copy_by_size": out, "launches_each": launches}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serve", action="store_true",
                    help="run only the replanning (serving) workload at 50/100/200 Hz and print its JSON")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="length of each Poisson run of --serve (requests = rate x seconds)")
    ap.add_argument("--serve-requests", type=int, default=0,
                    help="with --serve: requests per arrival rate (default: rate x --serve-seconds)")
    ap.add_argument("--uneven", action="store_true", help="run only the 64-problem uneven workload (c3)")
    ap.add_argument("--precision", action="store_true",
                    help="run only the precision workload (c4): FP32 vs BF16-split contraction, errors vs oracle")
    ap.add_argument("--no-serve", action="store_true", help="skip the short serving measurement")
    ap.add_argument("--mpc", action="store_true",
                    help="run only the closed-loop MPC benchmark on synthetic crowds (batch 1, 200, 1000)")
    ap.add_argument("--mpc-episodes", type=int, default=20)
    ap.add_argument("--mpc-iters", type=int, default=10, help="AM iterations per control period")
    ap.add_argument("--copy-ref", action="store_true",
                    help="run only a 512 MiB elementwise copy (y = x * 1), the size reference for "
                         "hardware byte counters, and exit")
    ap.add_argument("--fixed-cost", action="store_true",
                    help="run only the per-solve times of back-to-back fused solves for K = 0, 1, 2 and the "
                         "workload's K, with and without residual statistics, and exit")
    ap.add_argument("--copy-sizes", action="store_true",
                    help="run only elementwise copies (y = x * 1) that move as many bytes as one launch of "
                         "the plain path's projection and target kernels at c2 and c4, and exit")
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
        torch.mul(x, 1.0, out=y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(2):
            torch.mul(x, 1.0, out=y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 2
        print(json.dumps({"copy_ref_bytes_read": x.numel() * 4, "copy_ref_bytes_written": y.numel() * 4,
                          "launches": 3, "copy_ms": ms, "copy_GBps": 2 * x.numel() * 4 / (ms * 1e-3) / 1e9}))
        return
    if args.copy_sizes:
        print(json.dumps(copy_by_size()), flush=True)
        return
    if args.fixed_cost:
        print(json.dumps(fixed_cost(args.workload)), flush=True)
        return
    if args.uneven:
        print(json.dumps(run_uneven()), flush=True)
        return
    if args.precision:
        print(json.dumps(run_precision()), flush=True)
        return
    if args.mpc:
        import torch

        from paper_2109_13030_amd import mpc
        torch.cuda.set_device(0)
        res = mpc.benchmark(episodes=args.mpc_episodes, iters=args.mpc_iters,
                            progress=lambda s: print(s, file=sys.stderr, flush=True))
        print(json.dumps({"workload": "closed-loop MPC, 30-person synthetic crowds (static, same-direction "
                                      "flow up to 0.3 m/s, opposite flow up to 1.0 m/s), 1.5x0.5 m robot "
                                      f"tracking a straight line at 1 m/s, 40 ms period, {args.mpc_iters} "
                                      "warm-started iterations, 10 s horizon, nearest 10 people per period",
                          "episodes": args.mpc_episodes, "iterations": args.mpc_iters, "results": res}),
              flush=True)
        return
    if args.serve:
        count = (lambda r: args.serve_requests) if args.serve_requests else (lambda r: int(r * args.serve_seconds))
        rates = (50.0, 100.0, 200.0, 1000.0, 2000.0, 3000.0)
        sv = run_serving(rates, count, modes=("continuous", "sequential", "plain"), saturation=256,
                         max_rate={"plain": 200.0})
        # continuous batching held to one launch in flight: requests that
        # arrive during a launch share the next one
        one = run_serving(rates, count, modes=("continuous",), saturation=256, streams=1)
        sv["modes"]["continuous_one_stream"] = one["modes"]["continuous"]
        print(json.dumps(sv), flush=True)
        return
    out, pb, init, K = run_gpu(args)
    if not args.no_serve:
        sv = run_serving((200.0, 2000.0), lambda r: 300 if r < 1000 else 2000,
                         modes=("continuous", "sequential", "plain"), saturation=64, max_rate={"plain": 200.0})
        out["serving"] = sv
        cont = sv["modes"]["continuous"][0]
        out["p99_replan_latency_ms"] = cont["p99_ms"]
    final = out.pop("_final")
    if not args.no_cpu_baseline:
        out["cpu_baseline"], orc_state = cpu_baseline(pb, init, K, args.cpu_seconds)
        out["error_vs_oracle"] = error_vs_oracle(pb, final, orc_state)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
