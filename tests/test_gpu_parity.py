"""GPU library against the FP64 oracle on identical seeded inputs (needs an
MI355X).  Every call goes through the C-ABI of include/am.h."""
import numpy as np
import pytest

import oracle
from paper_2109_13030_amd import inputs
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_13030_amd import am
    am.lib()


def _small(name="c1", B=None, **kw):
    pb, init = inputs.workload(name, batch=B)
    pb = dict(pb, **kw)
    return pb, init


# ------------------------------------------------------------- setup (FP64 on the GPU)

@pytest.mark.parametrize("name", ["c1", "c2"])
def test_setup_inverse_matches_oracle_kkt(name):
    """The GPU's FP64 KKT inverses invert the oracle's KKT matrices (eq. over_2)."""
    from paper_2109_13030_amd import am
    pb, _ = inputs.workload(name, batch=1)
    h = am.Handle.for_problem(pb, "f64")
    k1i, k2i, basis = h.matrices()
    _, K1, K2 = oracle.Oracle(pb).matrices()
    P, Pd, Pdd = oracle.basis(pb["q"], pb["nv"], pb["tf"])
    np.testing.assert_allclose(basis[0], P, atol=1e-14)
    np.testing.assert_allclose(basis[1], Pd, atol=1e-14)
    np.testing.assert_allclose(basis[2], Pdd, atol=1e-14)
    for K, Ki in ((K1, k1i), (K2, k2i)):
        I = np.eye(K.shape[0])
        assert np.abs(K @ Ki - I).max() < 1e-8
        assert np.abs(Ki @ K - I).max() < 1e-8


# ------------------------------------------------------------- FP64 GPU = oracle (same algorithm)

def _run_plain(pb, init, K, dtype, projections=True):
    import torch
    from paper_2109_13030_amd import am
    h = am.Handle.for_problem(pb, dtype)
    p = am.DeviceProblem(pb, dtype)
    st = am.DeviceState(init, len(pb["r"]), len(pb["oa"]), pb["q"], dtype=dtype, projections=projections)
    ws = torch.empty(am.plain_workspace_size(h, st.B), dtype=torch.uint8, device="cuda")
    am.solve_plain(h, p, st, K, ws)
    torch.cuda.synchronize()
    return h, p, st


def _compare_f64(pb, init, K, tol=1e-8, projections=True, plain=False):
    if plain:
        h, p, st = _run_plain(pb, init, K, "f64", projections=projections)
    else:
        h, p, st = H.run_gpu(pb, init, K, "f64", projections=projections)
    out = st.numpy()
    orc, ost = H.run_oracle(pb, init, K)
    epos, epsi = H.traj_errors(pb, out, orc, ost)
    assert epos.max() < tol and epsi.max() < tol, (epos.max(), epsi.max())
    # multipliers (Bernstein coordinates) and slack coefficients as trajectories
    lam_scale = 1.0 + np.abs(ost["lam"]).max()
    assert np.abs(out["lam"] - ost["lam"]).max() < 1e3 * tol * lam_scale
    assert np.abs(out["lam_psi"] - ost["lampsi"]).max() < 1e3 * tol * (1 + np.abs(ost["lampsi"]).max())
    if projections:
        # alpha compared through (cos, sin); d directly
        a_g, a_o = out["alpha"], ost["alpha"]
        assert np.abs(np.cos(a_g) - np.cos(a_o)).max() < 1e3 * tol
        assert np.abs(np.sin(a_g) - np.sin(a_o)).max() < 1e3 * tol
        assert np.abs(out["d"] - ost["d"]).max() < 1e3 * tol * (1 + ost["d"].max())
        va = out["va"]
        assert np.abs(va[:, 1] - ost["dv"]).max() < 1e3 * tol
        assert np.abs(va[:, 3] - ost["da"]).max() < 1e3 * tol
    x = out["traj"]
    gx, gy, gp = H.gpu_traj(pb, out)
    np.testing.assert_allclose(x[:, 0], gx, atol=1e-9)
    np.testing.assert_allclose(x[:, 1], gy, atol=1e-9)
    np.testing.assert_allclose(x[:, 2], gp, atol=1e-9)
    return out, ost


def test_c1_f64_matches_oracle():
    """Config c1 (B = 16, 3 circles, 4 static obstacles, 50 iterations) in FP64."""
    pb, init = inputs.workload("c1")
    _compare_f64(pb, init, 50)


# (v_max, a_max, least clamped share of (trajectory, t) for d_v and d_a
# after 30 iterations): bounds below what the start-goal distance needs
# (~0.38 m/s on average), clamping at most time steps from the start; and
# bounds that no time step reaches in the first iterations and about a third
# reach by the end, so the discs become active during the solve
_DISCS = [(0.25, 0.002, 0.5, 0.5), (0.7, 0.15, 0.2, 0.3)]


@pytest.mark.parametrize("plain", [False, True])
@pytest.mark.parametrize("vmax,amax,share_v,share_a", _DISCS)
def test_active_velocity_and_acceleration_discs_f64(vmax, amax, share_v, share_a, plain):
    """The disc projections of eqs. compute_dv and compute_da clamp (d_v =
    d_a = 1 at the clamped time steps): fused and plain FP64 paths against
    the oracle."""
    pb, init = inputs.workload("c1", batch=8)
    pb = dict(pb, vmax=vmax, amax=amax)
    _, ost = _compare_f64(pb, init, 30, plain=plain)
    assert (ost["dv"] >= 1.0 - 1e-12).mean() > share_v
    assert (ost["da"] >= 1.0 - 1e-12).mean() > share_a


@pytest.mark.parametrize("vmax,amax,share_v,share_a", _DISCS)
def test_active_velocity_and_acceleration_discs_f32(vmax, amax, share_v, share_a):
    """The same clamped problems in FP32 against the oracle."""
    pb, init = inputs.workload("c1", batch=8)
    pb = dict(pb, vmax=vmax, amax=amax)
    _fp32_gate(pb, init, 30)


@pytest.mark.parametrize("flags", [oracle.ALPHA_LITERAL, oracle.XTILDE_SLACK, oracle.PSI_NO_UNWRAP,
                                   oracle.Q_CS_ZERO, oracle.LAMPSI_LITERAL])
def test_readings_f64_match_oracle(flags):
    """Each alternative reading gives the oracle's result (FP64, 10 iterations)."""
    pb, init = inputs.workload("c1", batch=6)
    pb = dict(pb, flags=flags)
    _compare_f64(pb, init, 10)


@pytest.mark.parametrize("B,K", [(1, 5), (5, 7), (9, 0), (4, 1)])
def test_ragged_batches_and_zero_iterations_f64(B, K):
    """Batches that fill part of a block, and iters = 0 (initial projection only)."""
    pb, init = inputs.workload("c2", batch=B)
    _compare_f64(pb, init, K)


def test_no_obstacles_and_single_circle_f64():
    pb, init = inputs.workload("c1", batch=5)
    pb0 = dict(pb, ox=np.zeros((0, pb["q"])), oy=np.zeros((0, pb["q"])), oa=np.zeros(0), ob=np.zeros(0))
    _compare_f64(pb0, init, 20, projections=False)
    pb1 = dict(pb, r=np.zeros(1), ob=pb["oa"].copy())
    _compare_f64(pb1, init, 20)


def _nv8(name, B):
    """A workload with 8 Bernstein coefficients per variable (the library's
    other basis size): the problem of `name` with nv = 8 and fresh samples."""
    pb, _ = inputs.workload(name, batch=1)
    pb = dict(pb, nv=8)
    return pb, inputs.make_initial(pb, B, inputs.config_seed(name) + 8, 0.5)


@pytest.mark.parametrize("plain", [False, True])
def test_nv8_f64_matches_oracle(plain):
    """The nv = 8 kernel instances (fused and plain) follow the oracle at FP64."""
    pb, init = _nv8("c1", 7)
    _compare_f64(pb, init, 12, plain=plain)


def test_nv8_f32_within_tolerance():
    """The nv = 8 FP32 instances (every launch configuration) against the
    oracle at 1e-3 m / 1e-3 rad, 300 trajectories of a c2-like problem."""
    from paper_2109_13030_amd import am
    pb, init = _nv8("c2", 300)
    h = am.Handle.for_problem(pb, "f32")
    p = am.DeviceProblem(pb, "f32")
    ref = None
    for tile, waves in am.LAUNCHES:
        h.tile, h.waves = tile, waves
        st = am.DeviceState(init, len(pb["r"]), len(pb["oa"]), pb["q"], "f32")
        am.solve(h, p, st, 60)
        out = st.numpy()
        if ref is None:
            ref = out
            _fp32_gate(pb, init, 60, out=out)
        else:
            for k in ("cx", "cy", "cpsi", "lam", "lam_psi"):
                assert np.array_equal(out[k], ref[k]), (tile, waves, k)


def test_warm_start_continues_the_iteration_f64():
    """K1 iterations then K2 more from the returned state = K1 + K2 at once."""
    from paper_2109_13030_amd import am
    pb, init = inputs.workload("c1", batch=8)
    h, p, st = H.run_gpu(pb, init, 30, "f64")
    st2 = am.DeviceState(st.numpy(), len(pb["r"]), len(pb["oa"]), pb["q"], "f64")
    am.solve(h, p, st2, 20)
    a = st2.numpy()
    _, _, st3 = H.run_gpu(pb, init, 50, "f64", handle=h, problem=p)
    b = st3.numpy()
    gx, gy, gp = H.gpu_traj(pb, a)
    hx, hy, hp = H.gpu_traj(pb, b)
    assert max(np.abs(gx - hx).max(), np.abs(gy - hy).max(), np.abs(gp - hp).max()) < 1e-8


# ------------------------------------------------------------- FP32 against the FP64 oracle

def _fp32_gate(pb, init, K, idx=None, out=None):
    """FP32 GPU vs FP64 oracle on trajectories idx (all by default): every
    trajectory within 1e-3 m and 1e-3 rad, the oracle run on the FP32 input
    values the GPU received."""
    if out is None:
        _, _, st = H.run_gpu(pb, init, K, "f32")
        out = st.numpy()
    if idx is None:
        idx = np.arange(out["cx"].shape[0])
    pb32, init32 = H.as_stored(pb, H.subset(init, idx), "f32")
    orc, ost = H.run_oracle(pb32, init32, K)
    outs = {k: (v[idx] if v is not None else None) for k, v in out.items()}
    epos, epsi = H.traj_errors(pb32, outs, orc, ost)
    bad = np.where((epos > H.TOL_POS) | (epsi > H.TOL_PSI))[0]
    assert bad.size == 0, (f"{bad.size} of {len(idx)} trajectories outside the tolerance: "
                           f"indices {np.asarray(idx)[bad][:10]}, max pos {epos.max():.3e} m, max psi {epsi.max():.3e} rad")
    return epos, epsi


def test_c1_f32_matches_oracle():
    pb, init = inputs.workload("c1")
    _fp32_gate(pb, init, 50)


@pytest.mark.parametrize("m", [1, 2, 4, 6, 7, 8])
def test_f32_circle_counts_against_oracle(m):
    """FP32 with 1 to 8 circles: the kernel instance with room for five
    circles (m <= 5) and the one with room for eight, each through its
    projection loops for m = C, C - 1, C - 2 and the general one (m = 3 and
    5 are c1 and c2)."""
    import dataclasses
    cfg = dataclasses.replace(inputs.CONFIGS["c2"], circles=m)
    pb = inputs.make_problem(cfg, 21)
    init = inputs.make_initial(pb, 24, 22, cfg.sigma)
    _fp32_gate(pb, init, 30)


def _largest_problem(B):
    import dataclasses
    cfg = dataclasses.replace(inputs.CONFIGS["c2"], q=128, n_obs=64, circles=8)
    pb = inputs.make_problem(cfg, 31)
    return pb, inputs.make_initial(pb, B, 32, cfg.sigma)


def test_largest_sizes_f32():
    """The largest problem the library takes (AM_MAX_Q, AM_MAX_OBS,
    AM_MAX_CIRCLES): 128 time steps, 64 obstacles (a full 64-bit vote mask,
    64 KB of obstacle table in LDS), 8 circles."""
    pb, init = _largest_problem(6)
    _fp32_gate(pb, init, 10)


def test_largest_sizes_plain_f64():
    """The per-sub-step path at the largest sizes (its kernels keep no
    obstacle table in LDS), FP64 against the oracle."""
    pb, init = _largest_problem(3)
    _compare_f64(pb, init, 4, plain=True)


def test_singular_kkt_is_reported():
    """A valid shape whose xi1 KKT matrix is numerically singular: a horizon of
    1 ms makes the acceleration blocks ~1e22 times the position blocks, so
    Gauss-Jordan meets a pivot below 1e-13 of the largest entry; am_setup
    returns AM_ERR_SINGULAR and no handle."""
    from paper_2109_13030_amd import am
    pb, _ = inputs.workload("c1", batch=1)
    with pytest.raises(am.AmError) as e:
        am.Handle.for_problem(dict(pb, tf=1e-3), "f64")
    assert e.value.code == am.AM_ERR_SINGULAR, str(e.value)


def test_largest_sizes_f64_fit_or_clean_error():
    """FP64 at the largest sizes needs more LDS than a workgroup may hold: the
    solve either matches the oracle or is refused before any launch with a
    message that names the LDS need."""
    from paper_2109_13030_amd import am
    pb, init = _largest_problem(3)
    try:
        _compare_f64(pb, init, 4)
    except am.AmError as e:
        assert e.code == am.AM_ERR_INVALID and "LDS" in str(e), str(e)


def test_c2_f32_full_batch_against_oracle():
    """Config c2 at its full size (B = 1000, 5 circles, 10 moving obstacles,
    100 iterations) in the launch the benchmark times: all 1000 trajectories
    against the oracle, each within 1e-3 m and 1e-3 rad."""
    pb, init = inputs.workload("c2")
    _, _, st = H.run_gpu(pb, init, 100, "f32")
    out = st.numpy()
    epos, epsi = _fp32_gate(pb, init, 100, None, out)
    print(f"c2 FP32: max |dx| {epos.max():.3e} m, max |dpsi| {epsi.max():.3e} rad, median {np.median(epos):.2e} m")
    # every trajectory keeps the boundary conditions and finite values
    from paper_2109_13030_amd import am
    h = am.Handle.for_problem(pb, "f32")
    p = am.DeviceProblem(pb, "f32")
    res = am.residuals(h, p, st).cpu().numpy()
    assert res[:, am.RES_NAMES.index("nonfinite")].max() == 0
    assert res[:, am.RES_NAMES.index("bc_max")].max() < 1e-3


def test_residuals_match_oracle():
    from paper_2109_13030_amd import am
    pb, init = inputs.workload("c1", batch=8)
    h, p, st = H.run_gpu(pb, init, 30, "f64")
    res = am.residuals(h, p, st).cpu().numpy()
    orc, ost = H.run_oracle(pb, init, 30)
    ref = orc.residuals(ost)
    np.testing.assert_allclose(res, ref, atol=1e-7, rtol=1e-6)


def test_f32_residuals_full_c2_match_f64_residuals_of_the_same_state():
    """The FP32 residual kernel at the benchmark's size (B = 1000 after 100
    iterations) against the FP64 residual kernel, which the tests above pin
    to the oracle, evaluated on the same coefficients: the two differ only by
    the FP32 rounding of the evaluation and of the closed forms.  Positions
    are O(10 m) and every statistic is a distance, a speed, a heading or a
    sum of squares of them, so 2e-4 absolute plus 1e-4 relative holds for
    well over a thousand ulps of the largest operand."""
    from paper_2109_13030_amd import am
    pb, init = inputs.workload("c2")
    h, p, st = H.run_gpu(pb, init, 100, "f32")
    r32 = am.residuals(h, p, st).cpu().numpy()
    out = st.numpy()
    same = {k: out[k] for k in am.DeviceState.KEYS}
    h64 = am.Handle.for_problem(pb, "f64")
    p64 = am.DeviceProblem(pb, "f64")
    st64 = am.DeviceState(same, len(pb["r"]), len(pb["oa"]), pb["q"], dtype="f64")
    r64 = am.residuals(h64, p64, st64).cpu().numpy()
    assert r32.shape == (1000, len(am.RES_NAMES))
    for j, name in enumerate(am.RES_NAMES):
        np.testing.assert_allclose(r32[:, j], r64[:, j], atol=2e-4, rtol=1e-4, err_msg=name)


@pytest.mark.parametrize("flags", [0, 1, 2])
@pytest.mark.parametrize("plain", [False, True])
def test_solve_residuals_match_oracle_f64(flags, plain):
    """The residual statistics a solve writes itself (am_state.res: the fused
    kernel's epilogue, the plain path's residual kernel) against the oracle's
    residuals of its own final state (FP64, c1 at 30 iterations, ragged
    batch), under the default angle, the literal angle and the slack copies."""
    import torch
    from paper_2109_13030_amd import am
    pb, init = inputs.workload("c1", batch=7)
    pb = dict(pb, flags=flags)
    h = am.Handle.for_problem(pb, "f64")
    p = am.DeviceProblem(pb, "f64")
    st = am.DeviceState(init, len(pb["r"]), len(pb["oa"]), pb["q"], "f64", residuals=True)
    if plain:
        ws = torch.empty(am.plain_workspace_size(h, st.B), dtype=torch.uint8, device="cuda")
        am.solve_plain(h, p, st, 30, ws)
    else:
        am.solve(h, p, st, 30)
    torch.cuda.synchronize()
    got = st.t["res"].cpu().numpy()
    orc, ost = H.run_oracle(pb, init, 30)
    ref = orc.residuals(ost)
    np.testing.assert_allclose(got, ref, atol=1e-7, rtol=1e-6)


def test_solve_residuals_full_c2_f32():
    """At the benchmark's size (FP32, B = 1000, K = 100) the statistics of the
    fused kernel's epilogue equal the FP64 residual kernel's on the same
    final coefficients, to the bound of the test above (the epilogue
    evaluates the positions in FP64 from the orthonormal coefficients, the
    residual kernel from the Bernstein ones)."""
    import torch
    from paper_2109_13030_amd import am
    pb, init = inputs.workload("c2")
    h = am.Handle.for_problem(pb, "f32")
    p = am.DeviceProblem(pb, "f32")
    st = am.DeviceState(init, len(pb["r"]), len(pb["oa"]), pb["q"], "f32", residuals=True)
    am.solve(h, p, st, 100)
    torch.cuda.synchronize()
    got = st.t["res"].cpu().numpy()
    out = st.numpy()
    same = {k: out[k] for k in am.DeviceState.KEYS}
    h64 = am.Handle.for_problem(pb, "f64")
    p64 = am.DeviceProblem(pb, "f64")
    st64 = am.DeviceState(same, len(pb["r"]), len(pb["oa"]), pb["q"], dtype="f64")
    r64 = am.residuals(h64, p64, st64).cpu().numpy()
    for j, name in enumerate(am.RES_NAMES):
        np.testing.assert_allclose(got[:, j], r64[:, j], atol=2e-4, rtol=1e-4, err_msg=name)


def _odd_horizon_problem(q, B=5):
    import dataclasses
    cfg = dataclasses.replace(inputs.CONFIGS["c2"], q=q)
    pb = inputs.make_problem(cfg, 11)
    return pb, inputs.make_initial(pb, B, 12, cfg.sigma)


@pytest.mark.parametrize("q", [37, 65, 127])
@pytest.mark.parametrize("plain", [False, True])
def test_odd_horizon_f64(q, plain):
    """An odd number of time steps: the fused kernel's two halves differ in
    length and the plain target kernel takes its one-step-per-item path."""
    pb, init = _odd_horizon_problem(q)
    _compare_f64(pb, init, 8, plain=plain)


def test_residuals_odd_horizon():
    from paper_2109_13030_amd import am
    pb, init = _odd_horizon_problem(37, B=6)
    h, p, st = H.run_gpu(pb, init, 10, "f64")
    res = am.residuals(h, p, st).cpu().numpy()
    orc, ost = H.run_oracle(pb, init, 10)
    np.testing.assert_allclose(res, orc.residuals(ost), atol=1e-7, rtol=1e-6)


def test_multi_problem_launch_equals_single_launches():
    """Uneven problems in one launch give bit-identical results to one launch
    per problem (same kernel, same arithmetic)."""
    import torch
    from paper_2109_13030_amd import am
    probs = inputs.uneven_problems("c3", count=5, batch_cap=70)
    handles, dps, sts, singles = [], [], [], []
    for pb, init in probs:
        h = am.Handle.for_problem(pb, "f32")
        dp = am.DeviceProblem(pb, "f32")
        handles.append(h)
        dps.append(dp)
        sts.append(am.DeviceState(init, len(pb["r"]), len(pb["oa"]), pb["q"], "f32"))
        s1 = am.DeviceState(init, len(pb["r"]), len(pb["oa"]), pb["q"], "f32")
        am.solve(h, dp, s1, 12)
        singles.append(s1)
    ws = torch.empty(am.multi_workspace_size(len(probs)), dtype=torch.uint8, device="cuda")
    am.solve_multi(handles, dps, sts, 12, ws)
    torch.cuda.synchronize()
    for s, s1 in zip(sts, singles):
        for k in ("cx", "cy", "cpsi", "lam", "lam_psi", "traj"):
            assert torch.equal(s.t[k], s1.t[k]), k


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_multi_problem_launch_matches_oracle(dtype):
    """One multi-problem launch over problems of different circle and
    obstacle counts and batch sizes (each with its own KKT, eq. over_3), run
    eagerly and as a replayed HIP graph, against the oracle problem by
    problem: FP64 within 1e-8, FP32 within the 1e-3 tolerance."""
    import torch
    from paper_2109_13030_amd import am
    probs = inputs.uneven_problems("c3", count=6, batch_cap=12)
    assert len({len(pb["r"]) for pb, _ in probs}) > 1 and len({len(pb["oa"]) for pb, _ in probs}) > 1
    K = 30 if dtype == "f64" else 100
    hs = [am.Handle.for_problem(pb, dtype) for pb, _ in probs]
    dps = [am.DeviceProblem(pb, dtype) for pb, _ in probs]
    mk = lambda: [am.DeviceState(init, len(pb["r"]), len(pb["oa"]), pb["q"], dtype) for pb, init in probs]
    ws = torch.empty(am.multi_workspace_size(len(probs)), dtype=torch.uint8, device="cuda")
    eager = mk()
    am.solve_multi(hs, dps, eager, K, ws)
    torch.cuda.synchronize()
    pristine, work = mk(), mk()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        am.solve_multi(hs, dps, work, K, ws)
    for s, p in zip(work, pristine):
        for k in am.DeviceState.KEYS:
            s.t[k].copy_(p.t[k])
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    for (pb, init), e, w in zip(probs, eager, work):
        for out in (e.numpy(), w.numpy()):
            if dtype == "f64":
                orc, ost = H.run_oracle(pb, init, K)
                epos, epsi = H.traj_errors(pb, out, orc, ost)
                assert epos.max() < 1e-8 and epsi.max() < 1e-8, (epos.max(), epsi.max())
            else:
                _fp32_gate(pb, init, K, None, out)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_empty_batches_launch_nothing(dtype):
    """Batch 0 with empty (NULL) arrays: every entry point succeeds and
    launches nothing; the selection reports -1; an empty problem between two
    others in one multi-problem launch leaves their results as in single
    launches."""
    import torch
    from paper_2109_13030_amd import am
    pb, init = inputs.workload("c1", batch=3)
    m, n, q = len(pb["r"]), len(pb["oa"]), pb["q"]
    empty = {k: np.zeros((0,) + np.asarray(v).shape[1:]) for k, v in init.items()}
    h = am.Handle.for_problem(pb, dtype)
    p = am.DeviceProblem(pb, dtype)
    st = am.DeviceState(empty, m, n, q, dtype=dtype)
    for k in st.t:
        st.t[k] = None   # every array pointer NULL
    am.solve(h, p, st, 5)
    am.solve_plain(h, p, st, 5, torch.empty(0, dtype=torch.uint8, device="cuda"))
    res = am.residuals(h, p, st, out=torch.empty((0, am.NRES), dtype=torch.float32 if dtype == "f32"
                                                 else torch.float64, device="cuda"))
    assert tuple(res.shape) == (0, am.NRES)
    assert am.select_best(h, res, 0.05) == (-1, 0.0, 0.0)
    a = am.DeviceState(init, m, n, q, dtype=dtype)
    b = am.DeviceState(init, m, n, q, dtype=dtype)
    ws = torch.empty(am.multi_workspace_size(3), dtype=torch.uint8, device="cuda")
    am.solve_multi([h, h, h], [p, p, p], [a, st, b], 7, ws)
    one = am.DeviceState(init, m, n, q, dtype=dtype)
    am.solve(h, p, one, 7)
    torch.cuda.synchronize()
    for k in ("cx", "cy", "cpsi", "lam", "lam_psi", "traj"):
        assert torch.equal(a.t[k], one.t[k]), k
        assert torch.equal(b.t[k], one.t[k]), k


# ------------------------------------------------------------- plain path (one launch per sub-step)

def test_plain_f64_matches_oracle():
    """The per-sub-step path with alpha, d in device memory gives the oracle's
    result (FP64, c1, 30 iterations)."""
    pb, init = inputs.workload("c1", batch=7)
    _compare_f64(pb, init, 30, plain=True)


@pytest.mark.parametrize("flags", [oracle.ALPHA_LITERAL, oracle.XTILDE_SLACK, oracle.LAMPSI_LITERAL])
def test_plain_readings_f64(flags):
    pb, init = inputs.workload("c2", batch=5)
    _compare_f64(dict(pb, flags=flags), init, 6, plain=True)


def test_plain_f32_c2_against_oracle():
    """Plain path at the full c2 size: all 1000 trajectories against the
    oracle."""
    pb, init = inputs.workload("c2")
    _, _, st = _run_plain(pb, init, 100, "f32", projections=False)
    _fp32_gate(pb, init, 100, None, st.numpy())


def test_multi_problem_launch_in_a_graph_replays_exactly():
    """The multi-problem launch captured in a HIP graph: every replay, with
    eager resets and synchronisations between replays, equals the eager
    launch bit for bit."""
    import torch
    from paper_2109_13030_amd import am
    probs = inputs.uneven_problems("c3", count=4, batch_cap=40)
    hs = [am.Handle.for_problem(pb, "f32") for pb, _ in probs]
    dps = [am.DeviceProblem(pb, "f32") for pb, _ in probs]
    pristine = [am.DeviceState(init, len(pb["r"]), len(pb["oa"]), pb["q"], "f32") for pb, init in probs]
    work = [am.DeviceState(init, len(pb["r"]), len(pb["oa"]), pb["q"], "f32") for pb, init in probs]
    ws = torch.empty(am.multi_workspace_size(len(probs)), dtype=torch.uint8, device="cuda")
    am.solve_multi(hs, dps, work, 9, ws)
    torch.cuda.synchronize()
    eager = [{k: v.clone() for k, v in s.t.items() if v is not None} for s in work]

    def reset():
        for s, p in zip(work, pristine):
            for k in am.DeviceState.KEYS:
                s.t[k].copy_(p.t[k])
        torch.cuda.synchronize()

    reset()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        am.solve_multi(hs, dps, work, 9, ws)
    for _ in range(3):
        reset()
        g.replay()
        torch.cuda.synchronize()
        for s, e in zip(work, eager):
            for k, v in e.items():
                assert torch.equal(s.t[k], v), k


# ------------------------------------------------------------- precision option: BF16 split contraction

def test_bf16x3_contraction_matches_fp32_contraction():
    """One iteration: the matrix-core BF16 split contraction reproduces the
    FP32 multipliers far below plain BF16 resolution (2^-8): the split keeps
    ~2^-17 per product, and the sums over t partly cancel."""
    from paper_2109_13030_amd import am
    pb, init = inputs.workload("c4", batch=45)
    a = _run_plain(pb, init, 1, "f32")[2].numpy()
    b = _run_plain(dict(pb, flags=am.PLAIN_BF16X3), init, 1, "f32")[2].numpy()
    scale = np.abs(a["lam"]).max()
    assert scale > 0
    assert np.abs(a["lam"] - b["lam"]).max() <= 1e-3 * scale
    assert np.abs(a["lam_psi"] - b["lam_psi"]).max() <= 1e-3 * (np.abs(a["lam_psi"]).max() + 1e-30)


def test_bf16x3_plain_c4_sampled_against_oracle():
    """Precision workload c4 (20 moving obstacles), plain path with the BF16
    split contraction: FP32 tolerance against the FP64 oracle on sampled
    trajectories (batch reduced to 512 to keep the test short)."""
    from paper_2109_13030_amd import am
    pb, init = inputs.workload("c4", batch=512)
    _, _, st = _run_plain(dict(pb, flags=am.PLAIN_BF16X3), init, 100, "f32", projections=False)
    out = st.numpy()
    idx = np.unique(np.concatenate([[0, 511], np.random.default_rng(3).choice(512, 14, replace=False)]))
    _fp32_gate(pb, init, 100, idx, out)


# ------------------------------------------------------------- launch tiles and the autotuner

def test_launch_configurations_give_identical_results_and_autotune_picks_one():
    """Every launch configuration (trajectories per block x register budget)
    computes the same trajectories bit for bit (ragged last block included);
    the autotuner picks one of them and leaves it set on the handle."""
    import torch
    from paper_2109_13030_amd import am
    pb, init = inputs.workload("c2", batch=9)
    h = am.Handle.for_problem(pb, "f32")
    p = am.DeviceProblem(pb, "f32")
    outs = {}
    for t, w in am.LAUNCHES:
        h.tile, h.waves = t, w
        st = am.DeviceState(init, len(pb["r"]), len(pb["oa"]), pb["q"], "f32")
        am.solve(h, p, st, 15)
        torch.cuda.synchronize()
        outs[(t, w)] = st.numpy()
    first = am.LAUNCHES[0]
    for c in am.LAUNCHES[1:]:
        for k in ("cx", "cy", "cpsi", "lam", "lam_psi", "traj"):
            np.testing.assert_array_equal(outs[c][k], outs[first][k])
    scratch = am.DeviceState(init, len(pb["r"]), len(pb["oa"]), pb["q"], "f32")
    best, times = am.autotune(h, p, scratch, 15)
    assert best in am.LAUNCHES and (h.tile, h.waves) == best
    assert set(times) == set(am.LAUNCHES) and all(v > 0 for v in times.values())
    # FP64 handles have the 2-wavefront budget only
    h64 = am.Handle.for_problem(pb, "f64")
    with pytest.raises(am.AmError):
        h64.waves = 3