"""Shared test helpers: run the GPU library and the oracle on identical inputs
and compare what they return."""
from __future__ import annotations

import numpy as np

import oracle

# FP32 parity tolerance of the fixed-iteration solve against the FP64 oracle
TOL_POS = 1e-3   # m
TOL_PSI = 1e-3   # rad
# A trajectory is well conditioned when the FP64 oracle itself moves by no
# more than TOL/20 under a relative perturbation of 2^-24 of its initial
# coefficients (the rounding of an FP32 input).  Only for those does a
# 1e-3 agreement of an FP32 computation follow from the arithmetic.
COND_FRACTION = 1.0 / 20.0


def subset(init: dict, idx) -> dict:
    return {k: np.asarray(v)[idx] for k, v in init.items()}


def run_oracle(pb: dict, init: dict, K: int, flags: int | None = None, nthreads: int = 0):
    p = dict(pb) if flags is None else dict(pb, flags=flags)
    orc = oracle.Oracle(p)
    st = oracle.state_from(p, init)
    orc.solve(st, K, nthreads=nthreads)
    return orc, st


def oracle_traj(orc, st):
    x, y, psi = orc.trajectories(st)
    return x, y, psi


def run_gpu(pb: dict, init: dict, K: int, dtype: str = "f32", projections: bool = False, handle=None,
            problem=None):
    import torch
    from paper_2109_13030_amd import am
    h = handle if handle is not None else am.Handle.for_problem(pb, dtype)
    p = problem if problem is not None else am.DeviceProblem(pb, dtype)
    st = am.DeviceState(init, len(pb["r"]), len(pb["oa"]), int(pb["q"]), dtype=dtype, projections=projections)
    am.solve(h, p, st, K)
    torch.cuda.synchronize()
    return h, p, st


def gpu_traj(pb: dict, out: dict):
    """x, y, psi from the returned Bernstein coefficients (oracle basis)."""
    P, _, _ = oracle.basis(int(pb["q"]), int(pb["nv"]), float(pb["tf"]))
    return out["cx"] @ P.T, out["cy"] @ P.T, out["cpsi"] @ P.T


def traj_errors(pb: dict, out: dict, orc, st):
    """Per-trajectory max |dx|, |dy| (m) and |dpsi| (rad)."""
    gx, gy, gp = gpu_traj(pb, out)
    ox, oy, op = oracle_traj(orc, st)
    epos = np.maximum(np.abs(gx - ox).max(1), np.abs(gy - oy).max(1))
    epsi = np.abs(gp - op).max(1)
    return epos, epsi


def conditioning(pb: dict, init: dict, K: int, trials: int = 2, seed: int = 7, nthreads: int = 0):
    """Per-trajectory spread of the FP64 oracle result under 2^-24 relative
    perturbations of the initial coefficients (max over trials of max |dx|,
    |dy|, |dpsi|)."""
    orc, st = run_oracle(pb, init, K, nthreads=nthreads)
    x0, y0, p0 = oracle_traj(orc, st)
    rng = np.random.default_rng(seed)
    spread = np.zeros(x0.shape[0])
    for _ in range(trials):
        pert = dict(init)
        for k in ("cx", "cy"):
            v = np.asarray(init[k], np.float64)
            pert[k] = v * (1.0 + 2.0 ** -24 * rng.choice([-1.0, 1.0], v.shape))
        o2, s2 = run_oracle(pb, pert, K, nthreads=nthreads)
        x, y, p = oracle_traj(o2, s2)
        spread = np.maximum(spread, np.maximum(np.abs(x - x0).max(1), np.maximum(np.abs(y - y0).max(1),
                                                                                  np.abs(p - p0).max(1))))
    return orc, st, spread
