"""Seeded workload generators (CPU): determinism, sizes of every config, and
the properties the input recipe promises."""
import numpy as np
import pytest

import oracle
from paper_2109_13030_amd import inputs


@pytest.mark.parametrize("name", ["c1", "c2", "c4"])
def test_workloads_are_deterministic_and_sized(name):
    cfg = inputs.CONFIGS[name]
    pb, init = inputs.workload(name, batch=32)
    pb2, init2 = inputs.workload(name, batch=32)
    for k in ("ox", "oy", "oa", "ob", "r"):
        np.testing.assert_array_equal(pb[k], pb2[k])
    for k in init:
        np.testing.assert_array_equal(init[k], init2[k])
    assert pb["ox"].shape == (cfg.n_obs, cfg.q) and len(pb["r"]) == cfg.circles
    assert init["cx"].shape == (32, cfg.nv) and init["lam"].shape == (32, 4 * cfg.nv)
    assert ((pb["oa"] >= 0.3) & (pb["oa"] <= 0.8)).all() and ((pb["ob"] >= 0.3) & (pb["ob"] <= 0.8)).all()
    # different seeds differ
    pb3, _ = inputs.workload(name, batch=32, seed=1)
    assert not np.array_equal(pb3["ox"], pb["ox"])


def test_obstacles_leave_start_and_goal_free():
    cfg = inputs.CONFIGS["c2"]
    keep = cfg.r_circle + cfg.length / 2.0
    for seed in range(20):
        pb = inputs.make_problem(cfg, seed)
        ga, gb = pb["oa"] + keep, pb["ob"] + keep
        s0 = ((pb["ox"][:, 0] - inputs.START[0]) / ga) ** 2 + ((pb["oy"][:, 0] - inputs.START[1]) / gb) ** 2
        s1 = ((pb["ox"][:, -1] - inputs.GOAL[0]) / ga) ** 2 + ((pb["oy"][:, -1] - inputs.GOAL[1]) / gb) ** 2
        assert (s0 > 1).all() and (s1 > 1).all()


def test_moving_obstacles_have_constant_velocity_within_bounds():
    pb, _ = inputs.workload("c2")
    dt = pb["tf"] / (pb["q"] - 1)
    vx = np.diff(pb["ox"], axis=1) / dt
    vy = np.diff(pb["oy"], axis=1) / dt
    np.testing.assert_allclose(vx, np.broadcast_to(vx[:, :1], vx.shape), atol=1e-9)
    np.testing.assert_allclose(vy, np.broadcast_to(vy[:, :1], vy.shape), atol=1e-9)
    assert (np.abs(vx) <= 1.0).all() and (np.abs(vy) <= 1.0).all()


def test_initial_samples_meet_the_boundary_conditions():
    """The noise sits on interior control points only, so position,
    velocity and acceleration at both ends are those of the straight
    rest-to-rest segment."""
    pb, init = inputs.workload("c2", batch=50)
    P, Pd, Pdd = oracle.basis(pb["q"], pb["nv"], pb["tf"])
    for c, b in ((init["cx"], pb["bx"]), (init["cy"], pb["by"])):
        np.testing.assert_allclose(c @ P[0], b[0], atol=1e-12)
        np.testing.assert_allclose(c @ P[-1], b[3], atol=1e-12)
        np.testing.assert_allclose(c @ Pd[[0, -1]].T, 0.0, atol=1e-12)
        np.testing.assert_allclose(c @ Pdd[[0, -1]].T, 0.0, atol=1e-12)
    assert np.std(init["cx"][:, 5]) > 0.3   # noise present in the interior


def test_uneven_and_serving_draws_respect_their_ranges():
    probs = inputs.uneven_problems("c3", count=16)
    for pb, init in probs:
        assert 64 <= init["cx"].shape[0] <= 1024
        assert 3 <= len(pb["r"]) <= 5 and 2 <= len(pb["oa"]) <= 20
    for c in inputs.serving_clients(16):
        assert 256 <= c["batch"] <= 2048 and 5 <= c["n"] <= 30
        assert c["init"]["cx"].shape[0] == c["batch"]


def test_replan_problem_advances_obstacles():
    pb, _ = inputs.workload("c2")
    nxt = inputs.replan_problem(pb, 3, period=0.04)
    dt = pb["tf"] / (pb["q"] - 1)
    v = (pb["ox"][:, 1] - pb["ox"][:, 0]) / dt
    np.testing.assert_allclose(nxt["ox"] - pb["ox"], (v * 0.12)[:, None] * np.ones(pb["q"]), atol=1e-9)


def test_poisson_arrivals_rate():
    t = inputs.poisson_arrivals(200.0, 20000, seed=1)
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 200.0) < 5.0
