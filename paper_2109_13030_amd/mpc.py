"""Closed-loop model-predictive control on top of the batched AM solver.

The paper runs its batch optimizer inside an MPC loop (Sec. IV,
implementation details): every control period the batch is re-solved for a
few iterations from fresh samples around a straight line, with the Lagrange
multipliers of every sample warm-started from the previous period, and the
best trajectory of the batch is executed.  Its benchmarks are a crowd of 30
people around a robot that tracks a straight line at 1 m/s: a static crowd,
a crowd walking the same way (up to 0.3 m/s) and a crowd walking towards the
robot (up to 1.0 m/s); the metrics are success rate (no collision), tracking
error with respect to the straight line and the acceleration used.

The paper's scenes are not available; `crowd_scene` draws seeded stand-ins
of the same kind.  Everything on the GPU goes through the C-ABI (`am`): the
solve, the residuals and the best-trajectory selection.  The host side only
simulates the plant: it advances the robot along the selected trajectory,
moves the people and checks the true robot rectangle against them.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import am, inputs

KINDS = ("static", "same_direction", "opposite_direction")


@dataclass
class Crowd:
    """People as discs moving at constant velocity (static ones have zero
    velocity); positions at time 0."""
    kind: str
    pos: np.ndarray        # [n, 2]
    vel: np.ndarray        # [n, 2]
    radius: float
    start: np.ndarray      # robot start (x, y)
    speed: float           # desired speed along +x
    length: float          # robot rectangle (body axis along the heading)
    width: float


def crowd_scene(kind: str, seed: int, n: int = 30, radius: float = 0.3, speed: float = 1.0,
                length: float = 1.5, width: float = 0.5, lane_half_width: float = 4.0,
                extent: float = 36.0) -> Crowd:
    """Seeded stand-in for the paper's crowd benchmarks: n people in a
    corridor |y| <= lane_half_width ahead of the robot (x in [4, extent]),
    at least 2 radii apart.  `same_direction`: velocities along +x with
    speed ~U[0.1, 0.3] m/s; `opposite_direction`: along -x with speed
    ~U[0.3, 1.0] m/s; small lateral components ~U[-0.05, 0.05] m/s."""
    if kind not in KINDS:
        raise ValueError(f"kind must be one of {KINDS}")
    rng = np.random.default_rng(seed)
    pos = []
    while len(pos) < n:
        p = np.array([rng.uniform(4.0, extent), rng.uniform(-lane_half_width, lane_half_width)])
        if all(np.hypot(*(p - o)) >= 2.2 * radius for o in pos):
            pos.append(p)
    pos = np.array(pos)
    vel = np.zeros((n, 2))
    if kind == "same_direction":
        vel[:, 0] = rng.uniform(0.1, 0.3, n)
    elif kind == "opposite_direction":
        vel[:, 0] = -rng.uniform(0.3, 1.0, n)
    if kind != "static":
        vel[:, 1] = rng.uniform(-0.05, 0.05, n)
    return Crowd(kind, pos, vel, radius, np.array([0.0, 0.0]), speed, length, width)


# ------------------------------------------------------------------ plant side

def bernstein_rows(nv: int, tf: float, tau: float):
    """Bernstein basis of degree nv-1 on [0, tf] and its first two time
    derivatives at time tau (each a length-nv vector)."""
    N = nv - 1
    s = min(max(tau / tf, 0.0), 1.0)

    def b(k, deg):
        if k < 0 or k > deg:
            return 0.0
        return math.comb(deg, k) * s ** k * (1.0 - s) ** (deg - k)

    P = np.array([b(i, N) for i in range(nv)])
    Pd = np.array([N * (b(i - 1, N - 1) - b(i, N - 1)) for i in range(nv)]) / tf
    Pdd = np.array([N * (N - 1) * (b(i - 2, N - 2) - 2 * b(i - 1, N - 2) + b(i, N - 2))
                    for i in range(nv)]) / tf ** 2
    return P, Pd, Pdd


def rect_disc_distance(p, psi: float, length: float, width: float, c, r: float) -> float:
    """Signed distance between a rectangle (centre p, heading psi) and a disc
    (centre c, radius r): negative when they overlap."""
    d = np.asarray(c, float) - np.asarray(p, float)
    cs, sn = math.cos(psi), math.sin(psi)
    lx, ly = cs * d[0] + sn * d[1], -sn * d[0] + cs * d[1]
    hx, hy = length / 2.0, width / 2.0
    ox, oy = abs(lx) - hx, abs(ly) - hy
    outside = math.hypot(max(ox, 0.0), max(oy, 0.0))
    inside = min(max(ox, oy), 0.0)
    return outside + inside - r


@dataclass
class EpisodeResult:
    success: bool
    collided: bool
    reached: bool
    steps: int
    tracking_error_mean: float
    accel_mean: float
    min_clearance: float
    replan_ms_mean: float
    replan_ms_p99: float
    feasible_fraction: float


class MPC:
    """Receding-horizon controller: one handle (KKT family) for the robot
    and crowd size, device state for `batch` samples kept between periods
    (its multipliers are the warm start)."""

    def __init__(self, batch: int, iters: int = 10, horizon: float = 10.0, q: int = 100, nv: int = 11,
                 circles: int = 5, length: float = 1.5, width: float = 0.5, n_obs: int = 10,
                 vmax: float = 1.5, amax: float = 1.5, rho: float = 1.0, sigma: float = 0.5,
                 fc_tol: float = 0.02, buffer: float = 0.05, reuse_previous: bool = True,
                 dt: float = 0.04, seed: int = 0, dtype: str = "f32"):
        import torch
        self.torch = torch
        self.dtype = dtype
        self.history = []   # per period: (selected index, its coefficients)
        self.B, self.K, self.tf, self.q, self.nv = int(batch), int(iters), float(horizon), int(q), int(nv)
        self.m, self.n = int(circles), int(n_obs)
        self.length, self.width = float(length), float(width)
        self.r = inputs.circle_offsets(self.m, self.length)
        # circles that cover the rectangle: radius to the corners of each
        # circle's L/m x W slice
        self.rc = math.hypot(self.length / (2 * self.m), self.width / 2.0)
        self.vmax, self.amax, self.rho, self.sigma, self.fc_tol = vmax, amax, rho, sigma, fc_tol
        self.buffer, self.reuse, self.dt = float(buffer), bool(reuse_previous), float(dt)
        self.rng = np.random.default_rng(seed)
        self.h = am.Handle(self.q, self.nv, self.tf, self.r, self.n, self.rho, dtype=dtype)
        self.state = None
        self.prev = None
        self.res = torch.empty((self.B, am.NRES), dtype=torch.float32 if dtype == "f32" else torch.float64,
                               device="cuda")
        # coefficients of a trajectory delayed by one period, by least squares
        # on the grid: c' = pinv(P) P(t + dt) c
        grid = inputs.time_grid(self.q, self.tf)
        P = np.stack([bernstein_rows(self.nv, self.tf, t)[0] for t in grid])
        Ps = np.stack([bernstein_rows(self.nv, self.tf, t + self.dt)[0] for t in grid])
        self.shift = np.linalg.pinv(P) @ Ps

    def end_point(self, crowd: Crowd, t_end: float):
        """End of the plan: the desired point at t_end, moved sideways in
        0.25 m steps to the nearest spot whose body-length disc is clear of
        every person predicted at t_end (the boundary conditions are hard
        constraints, so the end point itself must be free)."""
        x = crowd.start[0] + crowd.speed * t_end
        people = crowd.pos + crowd.vel * t_end
        need = crowd.radius + self.buffer + 0.5 * math.hypot(self.length, self.width) + 0.1
        for dy in sorted(np.arange(-12, 13) * 0.25, key=abs):
            y = crowd.start[1] + dy
            if np.all(np.hypot(people[:, 0] - x, people[:, 1] - y) >= need):
                return x, y
        return x, crowd.start[1]

    def nearest_people(self, crowd: Crowd, now: float, p0, t) -> np.ndarray:
        """The n_obs people that come closest, over the horizon, to the
        segment from the robot to the end of the desired line (the others
        stay out of the problem; n_obs fixes the KKT family)."""
        a = np.asarray(p0, float)
        b = crowd.start + np.array([crowd.speed * (now + self.tf), 0.0])
        ab = b - a
        L2 = max(float(ab @ ab), 1e-12)
        px = crowd.pos[:, 0:1] + crowd.vel[:, 0:1] * t[None, :]
        py = crowd.pos[:, 1:2] + crowd.vel[:, 1:2] * t[None, :]
        s = np.clip(((px - a[0]) * ab[0] + (py - a[1]) * ab[1]) / L2, 0.0, 1.0)
        d = np.hypot(px - (a[0] + s * ab[0]), py - (a[1] + s * ab[1])).min(axis=1)
        return np.argsort(d, kind="stable")[: self.n]

    def problem(self, crowd: Crowd, now: float, p0, v0, a0, psi0, dpsi0, ddpsi0) -> dict:
        t = inputs.time_grid(self.q, self.tf) + now
        sel = self.nearest_people(crowd, now, p0, t)
        ox = crowd.pos[sel, :1] + crowd.vel[sel, :1] * t[None, :]
        oy = crowd.pos[sel, 1:] + crowd.vel[sel, 1:] * t[None, :]
        goal_x, goal_y = self.end_point(crowd, now + self.tf)
        return dict(q=self.q, nv=self.nv, tf=self.tf, r=self.r, ox=ox, oy=oy,
                    oa=np.full(self.n, crowd.radius + self.buffer), ob=np.full(self.n, crowd.radius + self.buffer),
                    rc=self.rc,
                    bx=np.array([p0[0], v0[0], a0[0], goal_x, crowd.speed, 0.0]),
                    by=np.array([p0[1], v0[1], a0[1], goal_y, 0.0, 0.0]),
                    bpsi=np.array([psi0, dpsi0, ddpsi0, 0.0, 0.0, 0.0]),
                    vmax=self.vmax, amax=self.amax, rho=self.rho, rho_psi=self.rho, flags=0)

    def samples(self, pb: dict) -> dict:
        """Initial coefficients: Gaussian samples around the straight line
        between the two position boundary values (Sec. IV); a batch of one
        takes the straight line itself.  With `reuse_previous`, sample 0 is
        the previous period's selected trajectory delayed by one period."""
        B, nv = self.B, self.nv
        sig = self.sigma if B > 1 else 0.0
        init = inputs.make_initial(pb, B, int(self.rng.integers(1 << 31)), sig)
        init = {k: init[k] for k in ("cx", "cc", "cy", "cs", "cpsi")}
        if self.reuse and self.prev is not None:
            for k in init:
                init[k][0] = self.shift @ self.prev[k]
        return init

    def solve_select(self, pb: dict, init: dict):
        """The batch solve of one period on the GPU, from the given samples
        and the multipliers kept from the previous period, then the residuals
        and the best-trajectory selection; returns (index, its coefficients,
        its max |f_c|)."""
        p = am.DeviceProblem(pb, self.dtype)
        if self.state is None:
            self.state = am.DeviceState(init, self.m, self.n, self.q, self.dtype, outputs=False)
        else:
            self.state.load_coefficients(init)   # multipliers stay: warm start
        am.solve(self.h, p, self.state, self.K)
        am.residuals(self.h, p, self.state, out=self.res)
        idx, cost, fc = am.select_best(self.h, self.res, self.fc_tol)
        if idx < 0:
            raise RuntimeError("every trajectory of the batch is non-finite")
        coef = {k: self.state.t[k][idx].double().cpu().numpy() for k in ("cx", "cc", "cy", "cs", "cpsi")}
        return idx, coef, fc

    def plan(self, pb: dict):
        """One replanning period: solve, select; returns (coefficients of the
        best trajectory (x, y, psi), whether it met the collision tolerance,
        milliseconds from upload to selection)."""
        t0 = time.perf_counter()
        init = self.samples(pb)
        idx, coef, fc = self.solve_select(pb, init)
        self.prev = coef
        self.history.append((idx, coef))
        ms = (time.perf_counter() - t0) * 1e3
        return coef, fc <= self.fc_tol, ms

    def run(self, crowd: Crowd, duration: float = 25.0) -> EpisodeResult:
        """Closed loop until the robot has covered the course or `duration`
        seconds have passed; the robot follows the selected trajectory for
        one control period dt, the people move on, collisions are checked at
        every period with the true rectangle and discs."""
        self.state = None
        self.prev = None
        self.history = []
        dt = self.dt
        p = crowd.start.astype(float).copy()
        v = np.array([crowd.speed, 0.0])
        a = np.zeros(2)
        psi = dpsi = ddpsi = 0.0
        course = crowd.start[0] + crowd.speed * duration * 0.8
        track, accel, clear, ms, feas = [], [], [], [], []
        collided = reached = False
        steps = 0
        now = 0.0
        while now < duration:
            pb = self.problem(crowd, now, p, v, a, psi, dpsi, ddpsi)
            coef, ok, t_ms = self.plan(pb)
            ms.append(t_ms)
            feas.append(ok)
            P, Pd, Pdd = bernstein_rows(self.nv, self.tf, dt)
            p = np.array([coef["cx"] @ P, coef["cy"] @ P])
            v = np.array([coef["cx"] @ Pd, coef["cy"] @ Pd])
            a = np.array([coef["cx"] @ Pdd, coef["cy"] @ Pdd])
            psi, dpsi, ddpsi = coef["cpsi"] @ P, coef["cpsi"] @ Pd, coef["cpsi"] @ Pdd
            now += dt
            steps += 1
            people = crowd.pos + crowd.vel * now
            dmin = min(rect_disc_distance(p, psi, crowd.length, crowd.width, c, crowd.radius) for c in people)
            clear.append(dmin)
            des = crowd.start + np.array([crowd.speed * now, 0.0])
            track.append(float(np.hypot(*(p - des))))
            accel.append(float(np.hypot(*a)))
            if dmin < 0.0:
                collided = True
                break
            if p[0] >= course:
                reached = True
                break
        ms_arr = np.array(ms)
        return EpisodeResult(success=reached and not collided, collided=collided, reached=reached, steps=steps,
                             tracking_error_mean=float(np.mean(track)), accel_mean=float(np.mean(accel)),
                             min_clearance=float(np.min(clear)), replan_ms_mean=float(ms_arr.mean()),
                             replan_ms_p99=float(np.percentile(ms_arr, 99)),
                             feasible_fraction=float(np.mean(feas)))


def benchmark(batches=(1, 200, 1000), episodes: int = 20, iters: int = 10, seed: int = 7,
              duration: float = 25.0, progress=None):
    """Success rate, tracking error and acceleration per crowd kind and batch
    size (the shape of the paper's batch-size comparison), on seeded scenes.
    `progress(text)` is called after every (batch, kind) cell."""
    out = {}
    for B in batches:
        ctl = MPC(B, iters=iters, seed=seed)
        rows = {}
        for kind in KINDS:
            t0 = time.perf_counter()
            res = [ctl.run(crowd_scene(kind, seed * 1000 + e), duration=duration) for e in range(episodes)]
            rows[kind] = {
                "success_rate": float(np.mean([r.success for r in res])),
                "collision_rate": float(np.mean([r.collided for r in res])),
                "tracking_error_m": float(np.mean([r.tracking_error_mean for r in res])),
                "accel_mps2": float(np.mean([r.accel_mean for r in res])),
                "min_clearance_m": float(np.min([r.min_clearance for r in res])),
                "replan_ms_mean": float(np.mean([r.replan_ms_mean for r in res])),
                "replan_ms_p99": float(np.max([r.replan_ms_p99 for r in res])),
                "feasible_fraction": float(np.mean([r.feasible_fraction for r in res])),
            }
            if progress:
                progress(f"batch {B} {kind}: success {rows[kind]['success_rate']:.2f} "
                         f"({time.perf_counter() - t0:.1f} s)")
        out[str(B)] = rows
    return out
