"""Closed-loop MPC on the batched solver: host-side plant pieces on the CPU
(Bernstein evaluation between grid points, rectangle-disc geometry, scene
draws) and a short closed loop on the GPU."""
import math

import numpy as np
import pytest

import oracle
from paper_2109_13030_amd import mpc


@pytest.mark.parametrize("nv,tf", [(11, 10.0), (8, 3.0)])
def test_bernstein_rows_match_the_oracle_basis_on_the_grid(nv, tf):
    q = 17
    P, Pd, Pdd = oracle.basis(q, nv, tf)
    for k in range(q):
        a, b, c = mpc.bernstein_rows(nv, tf, k * tf / (q - 1))
        np.testing.assert_allclose(a, P[k], rtol=0, atol=1e-12)
        np.testing.assert_allclose(b, Pd[k], rtol=0, atol=1e-11)
        np.testing.assert_allclose(c, Pdd[k], rtol=0, atol=1e-10)


def test_bernstein_rows_between_grid_points_are_a_polynomial():
    """A degree-10 polynomial given by its Bernstein coefficients: value and
    derivatives at an off-grid time agree with numpy's polynomial algebra."""
    rng = np.random.default_rng(1)
    nv, tf = 11, 7.0
    coef = rng.normal(size=nv)
    N = nv - 1
    # power-basis coefficients in s = t / tf
    poly = np.polynomial.Polynomial([0.0])
    for i in range(nv):
        poly += coef[i] * math.comb(N, i) * np.polynomial.Polynomial([0, 1]) ** i * np.polynomial.Polynomial([1, -1]) ** (N - i)
    t = 2.345
    P, Pd, Pdd = mpc.bernstein_rows(nv, tf, t)
    assert coef @ P == pytest.approx(poly(t / tf), abs=1e-12)
    assert coef @ Pd == pytest.approx(poly.deriv(1)(t / tf) / tf, abs=1e-11)
    assert coef @ Pdd == pytest.approx(poly.deriv(2)(t / tf) / tf ** 2, abs=1e-10)


def test_rect_disc_distance_closed_forms():
    L, W, r = 1.5, 0.5, 0.3
    # along the body axis, across it, at the corner's diagonal, and inside
    assert mpc.rect_disc_distance((0, 0), 0.0, L, W, (2.0, 0.0), r) == pytest.approx(2.0 - L / 2 - r)
    assert mpc.rect_disc_distance((0, 0), 0.0, L, W, (0.0, 1.0), r) == pytest.approx(1.0 - W / 2 - r)
    assert mpc.rect_disc_distance((0, 0), math.pi / 2, L, W, (0.0, 2.0), r) == pytest.approx(2.0 - L / 2 - r)
    assert mpc.rect_disc_distance((1, 1), 0.0, L, W, (1 + L / 2 + 3, 1 + W / 2 + 4), r) == pytest.approx(5.0 - r)
    assert mpc.rect_disc_distance((0, 0), 0.3, L, W, (0.0, 0.0), r) == pytest.approx(-W / 2 - r)
    # brute force over the rectangle's boundary and interior
    rng = np.random.default_rng(2)
    for _ in range(50):
        p, psi, c = rng.uniform(-2, 2, 2), rng.uniform(-math.pi, math.pi), rng.uniform(-3, 3, 2)
        u = np.linspace(-L / 2, L / 2, 301)
        v = np.linspace(-W / 2, W / 2, 101)
        X, Y = np.meshgrid(u, v)
        gx = p[0] + math.cos(psi) * X - math.sin(psi) * Y
        gy = p[1] + math.sin(psi) * X + math.cos(psi) * Y
        dmin = np.hypot(gx - c[0], gy - c[1]).min()
        dist = mpc.rect_disc_distance(p, psi, L, W, c, r) + r   # centre to rectangle
        if dist > 0:
            assert dist == pytest.approx(dmin, abs=5e-3)
        else:
            assert dmin < 5e-3


@pytest.mark.parametrize("kind", mpc.KINDS)
def test_crowd_scene_draws(kind):
    a, b = mpc.crowd_scene(kind, 11), mpc.crowd_scene(kind, 11)
    np.testing.assert_array_equal(a.pos, b.pos)
    np.testing.assert_array_equal(a.vel, b.vel)
    assert a.pos.shape == (30, 2)
    d = np.hypot(*(a.pos[:, None, :] - a.pos[None, :, :]).transpose(2, 0, 1))
    assert (d + np.eye(30) * 10 >= 2.2 * a.radius - 1e-12).all()
    if kind == "static":
        assert not a.vel.any()
    elif kind == "same_direction":
        assert (a.vel[:, 0] > 0).all() and (a.vel[:, 0] <= 0.3).all()
    else:
        assert (a.vel[:, 0] < 0).all() and (a.vel[:, 0] >= -1.0).all()


@pytest.mark.gpu
def test_short_closed_loop_is_finite_and_deterministic():
    """A 1 s closed loop (25 periods of 40 ms, 64 samples, 5 iterations) in
    the opposite-flow crowd: finite metrics, the robot advances, and a rerun
    with the same seeds gives the same result."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    crowd = mpc.crowd_scene("opposite_direction", 5)
    r1 = mpc.MPC(64, iters=5, seed=3).run(crowd, duration=1.0)
    r2 = mpc.MPC(64, iters=5, seed=3).run(crowd, duration=1.0)
    assert r1.steps == 25 and not r1.collided
    assert np.isfinite([r1.tracking_error_mean, r1.accel_mean, r1.min_clearance]).all()
    assert r1.tracking_error_mean < 1.0
    for f in ("success", "collided", "reached", "steps", "tracking_error_mean", "accel_mean", "min_clearance",
              "feasible_fraction"):
        assert getattr(r1, f) == getattr(r2, f), f


@pytest.mark.gpu
def test_fp64_closed_loop_matches_an_oracle_driven_loop():
    """Five control periods of the FP64 closed loop (8 samples, 6 warm-started
    iterations per period) against the same loop with the FP64 oracle as the
    solver (its state, and so its multipliers, kept between periods, Sec. IV)
    and the selection rule written out in numpy: every period selects the
    same sample, with coefficients within 1e-8."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle

    def best_rule(res, tol):
        fin = res[:, 11] == 0
        ok = fin & (res[:, 0] <= tol)
        pool = np.flatnonzero(ok) if ok.any() else np.flatnonzero(fin)
        key = res[pool, 7] if ok.any() else res[pool, 0]
        return int(pool[np.lexsort((pool, key))[0]])

    class OracleMPC(mpc.MPC):
        def solve_select(self, pb, init):
            orc = oracle.Oracle(pb)
            st = oracle.state_from(pb, init)
            if self.state is not None:                       # warm start
                st["lam"][:], st["lampsi"][:] = self.state["lam"], self.state["lampsi"]
            orc.solve(st, self.K)
            self.state = st
            res = orc.residuals(st)
            idx = best_rule(res, self.fc_tol)
            return idx, {k: st[k][idx].copy() for k in ("cx", "cc", "cy", "cs", "cpsi")}, res[idx, 0]

    crowd = mpc.crowd_scene("opposite_direction", 5)
    kw = dict(iters=6, seed=3, dtype="f64")
    gpu = mpc.MPC(8, **kw)
    gpu.run(crowd, duration=0.2)
    ref = OracleMPC(8, **kw)
    ref.run(crowd, duration=0.2)
    assert len(gpu.history) == len(ref.history) == 5
    for (ig, cg), (io, co) in zip(gpu.history, ref.history):
        assert ig == io
        for k in cg:
            np.testing.assert_allclose(cg[k], co[k], atol=1e-8, rtol=0, err_msg=k)
