"""Seeded synthetic workloads for the batched AM trajectory optimizer.

This module only draws numbers: obstacle tables, robot geometry, boundary
conditions and initial Bernstein control points.  It holds none of the
method's arithmetic and is the one module shared by the GPU path and the
oracle-based tests, so that both see identical inputs.

Workloads follow the paper's setting (Sec. II-B, Sec. IV): a rectangular
holonomic robot covered by ``m`` overlapping circles, ``n`` axis-aligned
elliptical obstacles (static or moving at constant velocity), a 30 s horizon
(the paper gives about 30 s, Sec. II-B), boundary conditions shared by the whole batch, and
initial trajectories drawn once from a Gaussian around a straight line
(Sec. IV, implementation details).  The paper's crowd scenes are not
available; these seeded draws stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BOX = (0.0, 10.0)          # square workspace [m]
START = (1.0, 1.0)
GOAL = (9.0, 9.0)
SEED_BASE = 13030


@dataclass(frozen=True)
class Config:
    """One workload.  Sizes per problem; ``batch``/``n_obs``/``circles`` may be
    ranges (lo, hi) for the uneven and serving workloads."""
    name: str
    batch: object
    circles: object
    n_obs: object
    length: float
    width: float
    r_circle: float
    dynamic: bool
    iters: int
    dtype: str = "f32"
    q: int = 100
    nv: int = 11
    tf: float = 30.0
    sigma: float = 0.5
    vmax: float = 1.5
    amax: float = 1.5
    rho: float = 1.0
    problems: int = 1
    extra: dict = field(default_factory=dict)


CONFIGS = {
    # small FP64 case the oracle finishes in seconds
    "c1": Config("c1", batch=16, circles=3, n_obs=4, length=1.2, width=0.6, r_circle=0.3,
                 dynamic=False, iters=50, dtype="f64"),
    # the headline workload: B = 1000, 5 circles, 10 moving obstacles, 100 iterations
    "c2": Config("c2", batch=1000, circles=5, n_obs=10, length=1.5, width=0.5, r_circle=0.25,
                 dynamic=True, iters=100),
    # 64 independent problems of uneven size in one launch
    "c3": Config("c3", batch=(64, 1024), circles=(3, 5), n_obs=(2, 20), length=1.5, width=0.5,
                 r_circle=0.25, dynamic=True, iters=100, problems=64),
    # large batch, 20 moving obstacles
    "c4": Config("c4", batch=4096, circles=5, n_obs=20, length=1.5, width=0.5, r_circle=0.25,
                 dynamic=True, iters=100),
    # replanning requests: sizes per request, 20 warm-started iterations
    "c5": Config("c5", batch=(256, 2048), circles=5, n_obs=(5, 30), length=1.5, width=0.5,
                 r_circle=0.25, dynamic=True, iters=20,
                 extra=dict(rates_hz=(50.0, 100.0, 200.0))),
}


def time_grid(q: int, tf: float) -> np.ndarray:
    """t_k = k*tf/(q-1), k = 0..q-1 (both ends on the grid)."""
    return np.arange(q, dtype=np.float64) * (tf / (q - 1))


def circle_offsets(m: int, length: float) -> np.ndarray:
    """Evenly spaced circle centres along the body axis: (i - (m-1)/2) * L/m."""
    return (np.arange(m, dtype=np.float64) - (m - 1) / 2.0) * (length / m)


def draw_obstacles(rng: np.random.Generator, n: int, q: int, tf: float, dynamic: bool,
                   keep_clear: float, start=START, goal=GOAL):
    """n axis-aligned ellipses with semi-axes ~U[0.3, 0.8] m.  Moving obstacles
    have velocities ~U[-1, 1] m/s per axis and their centre at tf/2 drawn
    uniformly in the box, so they cross it mid-horizon; static ones sit
    uniformly in the box.  An obstacle whose ellipse, grown by ``keep_clear``,
    holds the start at t=0 or the goal at t=tf is redrawn."""
    t = time_grid(q, tf)
    ox = np.zeros((n, q))
    oy = np.zeros((n, q))
    oa = np.zeros(n)
    ob = np.zeros(n)
    for j in range(n):
        while True:
            a, b = rng.uniform(0.3, 0.8, 2)
            cx, cy = rng.uniform(BOX[0], BOX[1], 2)
            if dynamic:
                vx, vy = rng.uniform(-1.0, 1.0, 2)
                xs = cx + vx * (t - tf / 2.0)
                ys = cy + vy * (t - tf / 2.0)
            else:
                xs = np.full(q, cx)
                ys = np.full(q, cy)
            ga, gb = a + keep_clear, b + keep_clear
            s0 = ((xs[0] - start[0]) / ga) ** 2 + ((ys[0] - start[1]) / gb) ** 2
            s1 = ((xs[-1] - goal[0]) / ga) ** 2 + ((ys[-1] - goal[1]) / gb) ** 2
            if s0 > 1.0 and s1 > 1.0:
                break
        ox[j], oy[j], oa[j], ob[j] = xs, ys, a, b
    return ox, oy, oa, ob


def make_problem(cfg: Config, seed: int, m: int | None = None, n: int | None = None,
                 flags: int = 0) -> dict:
    """Problem dict shared by the whole batch (keys as in the oracle and the
    C-ABI problem description)."""
    rng = np.random.default_rng(seed)
    m = int(cfg.circles if m is None else m)
    n = int(cfg.n_obs if n is None else n)
    r = circle_offsets(m, cfg.length)
    keep = cfg.r_circle + cfg.length / 2.0
    ox, oy, oa, ob = draw_obstacles(rng, n, cfg.q, cfg.tf, cfg.dynamic, keep)
    return dict(q=cfg.q, nv=cfg.nv, tf=cfg.tf, r=r, ox=ox, oy=oy, oa=oa, ob=ob,
                rc=cfg.r_circle,
                bx=np.array([START[0], 0.0, 0.0, GOAL[0], 0.0, 0.0]),
                by=np.array([START[1], 0.0, 0.0, GOAL[1], 0.0, 0.0]),
                bpsi=np.zeros(6), vmax=cfg.vmax, amax=cfg.amax, rho=cfg.rho,
                rho_psi=cfg.rho, flags=int(flags))


def straight_line_points(p0: float, pf: float, nv: int) -> np.ndarray:
    """Bernstein control points of a rest-to-rest straight segment: the first
    three equal p0, the last three equal pf (zero end velocity and
    acceleration) and the interior ones are evenly spaced between them."""
    s = np.clip((np.arange(nv) - 2.0) / (nv - 5.0), 0.0, 1.0)
    return p0 + (pf - p0) * s


def make_initial(pb: dict, B: int, seed: int, sigma: float = 0.5) -> dict:
    """Initial state for B trajectories: straight-line control points plus
    N(0, sigma^2) noise on the interior points (indices 3 .. nv-4), which keeps
    the boundary conditions; constant heading psi0; zero multipliers and
    slack coefficients."""
    rng = np.random.default_rng(seed)
    nv = int(pb["nv"])
    cx = np.tile(straight_line_points(pb["bx"][0], pb["bx"][3], nv), (B, 1))
    cy = np.tile(straight_line_points(pb["by"][0], pb["by"][3], nv), (B, 1))
    inner = slice(3, nv - 3)
    k = nv - 6
    cx[:, inner] += rng.normal(0.0, sigma, (B, k))
    cy[:, inner] += rng.normal(0.0, sigma, (B, k))
    cpsi = np.full((B, nv), float(pb["bpsi"][0]))
    z = np.zeros((B, nv))
    return dict(cx=cx, cy=cy, cpsi=cpsi, cc=z.copy(), cs=z.copy(),
                lam=np.zeros((B, 4 * nv)), lampsi=np.zeros((B, nv)))


def config_seed(name: str) -> int:
    return SEED_BASE + int(name[1:])


def workload(name: str, batch: int | None = None, seed: int | None = None):
    """(problem, initial state) of a single-problem config."""
    cfg = CONFIGS[name]
    s = config_seed(name) if seed is None else seed
    ss = np.random.SeedSequence(s)
    kp, ki = ss.spawn(2)
    pb = make_problem(cfg, int(kp.generate_state(1)[0]))
    B = int(cfg.batch if batch is None else batch)
    init = make_initial(pb, B, int(ki.generate_state(1)[0]), cfg.sigma)
    return pb, init


def uneven_problems(name: str = "c3", count: int | None = None, seed: int | None = None,
                    batch_cap: int | None = None):
    """List of (problem, initial state) for the uneven multi-problem workload:
    batch ~ U{lo..hi}, circles ~ U{lo..hi}, obstacles ~ U{lo..hi} per problem."""
    cfg = CONFIGS[name]
    s = config_seed(name) if seed is None else seed
    count = cfg.problems if count is None else count
    out = []
    for child in np.random.SeedSequence(s).spawn(count):
        rng = np.random.default_rng(child)
        B = int(rng.integers(cfg.batch[0], cfg.batch[1] + 1))
        if batch_cap is not None:
            B = min(B, batch_cap)
        m = int(rng.integers(cfg.circles[0], cfg.circles[1] + 1)) if isinstance(cfg.circles, tuple) else cfg.circles
        n = int(rng.integers(cfg.n_obs[0], cfg.n_obs[1] + 1))
        pb = make_problem(cfg, int(rng.integers(1 << 62)), m=m, n=n)
        init = make_initial(pb, B, int(rng.integers(1 << 62)), cfg.sigma)
        out.append((pb, init))
    return out


# ---------------------------------------------------------------- replanning workload

def serving_clients(count: int, seed: int | None = None):
    """Robots of the replanning workload: each has its own scene (5 circles,
    n ~ U{5..30} moving obstacles) and sample count B ~ U{256..2048}."""
    cfg = CONFIGS["c5"]
    s = config_seed("c5") if seed is None else seed
    out = []
    for child in np.random.SeedSequence(s).spawn(count):
        rng = np.random.default_rng(child)
        B = int(rng.integers(cfg.batch[0], cfg.batch[1] + 1))
        n = int(rng.integers(cfg.n_obs[0], cfg.n_obs[1] + 1))
        pb = make_problem(cfg, int(rng.integers(1 << 62)), m=cfg.circles, n=n)
        init = make_initial(pb, B, int(rng.integers(1 << 62)), cfg.sigma)
        out.append(dict(problem=pb, init=init, batch=B, n=n))
    return out


def replan_problem(pb: dict, step: int, period: float = 0.04) -> dict:
    """The scene `step` control periods later: every obstacle advanced along
    its constant velocity (the horizon slides with the controller)."""
    q, tf = int(pb["q"]), float(pb["tf"])
    dt = tf / (q - 1)
    ox, oy = np.asarray(pb["ox"]), np.asarray(pb["oy"])
    if ox.shape[0] == 0 or q < 2:
        return dict(pb)
    vx = (ox[:, 1] - ox[:, 0]) / dt
    vy = (oy[:, 1] - oy[:, 0]) / dt
    shift = step * period
    return dict(pb, ox=ox + vx[:, None] * shift, oy=oy + vy[:, None] * shift)


def as_stored(pb: dict, init: dict, dtype: str):
    """The problem and initial state as device arrays of `dtype` hold them:
    for FP32 the obstacle table and the initial coefficients and
    multipliers rounded once to float32 (the problem's scalars travel as
    doubles through the C-ABI and are unchanged)."""
    if dtype != "f32":
        return pb, init
    r32 = lambda v: np.asarray(np.asarray(v, np.float64), np.float32).astype(np.float64)
    pb = dict(pb, **{k: r32(pb[k]) for k in ("ox", "oy", "oa", "ob")})
    init = {k: r32(v) for k, v in init.items()}
    return pb, init


def poisson_arrivals(rate_hz: float, count: int, seed: int = 0) -> np.ndarray:
    """Arrival times [s] of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, count))
