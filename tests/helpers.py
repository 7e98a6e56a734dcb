"""Shared test helpers: run the GPU library and the oracle on identical inputs
and compare what they return."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2109_13030_amd import inputs

# FP32 parity tolerance of the fixed-iteration solve against the FP64 oracle
TOL_POS = 1e-3   # m
TOL_PSI = 1e-3   # rad


def as_stored(pb: dict, init: dict, dtype: str):
    """The problem and initial state as the device arrays of `dtype` hold
    them (inputs.as_stored).  The oracle of an FP32 test runs on these
    values, so that a parity test measures the arithmetic of the path and
    not the quantisation of its inputs."""
    return inputs.as_stored(pb, init, dtype)


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
