"""Replanning server (continuous batching) through the C-ABI (needs an
MI355X): results are the same alone and in the mix, warm starts continue the
iteration, admission respects the device-memory budget."""
import numpy as np
import pytest

from paper_2109_13030_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def am():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_13030_amd import am as amod
    amod.lib()
    return amod


def _clients(count, cap=300):
    cl = inputs.serving_clients(count, seed=77)
    for c in cl:
        c["batch"] = min(c["batch"], cap)
        c["init"] = {k: v[:c["batch"]] for k, v in c["init"].items()}
    return cl


def _handles(am, clients):
    return [am.Handle.for_problem(c["problem"], "f32") for c in clients]


def test_same_result_alone_and_in_the_mix(am):
    """A request's trajectories are bit-identical whether it runs alone or in
    one launch with others.  The mix is made to share a launch: one stream,
    and a long request occupies it while the eight arrive, so the scheduler
    admits all eight together once the stream frees (launches < requests)."""
    clients = _clients(8)
    hs = _handles(am, clients)
    K = 12
    s1 = am.Server(1 << 28, streams=4, max_per_launch=16)
    t = s1.submit(hs[3], clients[3]["problem"], 0, clients[3]["batch"], K, clients[3]["init"])
    done, _, alone = s1.wait(t, 60.0, traj=True)
    assert done
    s1.close()
    s2 = am.Server(1 << 28, streams=1, max_per_launch=16, idle_spin_us=5000)
    blocker = _clients(9)[8]
    hb = _handles(am, [blocker])[0]
    tb = s2.submit(hb, blocker["problem"], 100, blocker["batch"], 20000, blocker["init"])
    tickets = [s2.submit(h, c["problem"], i, c["batch"], K, c["init"]) for i, (h, c) in enumerate(zip(hs, clients))]
    outs = [s2.wait(tk, 60.0, traj=True) for tk in tickets]
    assert s2.wait(tb, 60.0)[0]
    assert all(o[0] for o in outs)
    np.testing.assert_array_equal(outs[3][2], alone)
    st = s2.stats()
    assert st["completed"] == len(clients) + 1
    assert st["launches"] < st["completed"], st
    s2.close()
    # and equal to the direct batch solve
    import torch
    c = clients[3]
    p = am.DeviceProblem(c["problem"], "f32")
    ds = am.DeviceState(c["init"], 5, c["n"], c["problem"]["q"], "f32")
    am.solve(hs[3], p, ds, K)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ds.t["traj"].cpu().numpy(), alone)


def test_requests_of_two_shapes_in_one_queue(am):
    """Requests of two time-step counts queued together while a long request
    holds the only stream: each launch holds one shape (a launch mixing them
    would be refused), every request completes, and each result equals its
    direct solve."""
    import dataclasses

    import torch
    cfg = dataclasses.replace(inputs.CONFIGS["c5"], q=64)
    short = []
    for k in range(3):
        pb = inputs.make_problem(cfg, 500 + k, m=5, n=6 + k)
        short.append(dict(problem=pb, init=inputs.make_initial(pb, 40, 600 + k), batch=40, n=6 + k))
    mixed = [c for pair in zip(_clients(3, cap=40), short) for c in pair]
    hs = _handles(am, mixed)
    K = 9
    s = am.Server(1 << 28, streams=1, max_per_launch=16, idle_spin_us=5000)
    blocker = _clients(9)[8]
    hb = _handles(am, [blocker])[0]   # the server uses the handle until the request completes
    tb = s.submit(hb, blocker["problem"], 100, blocker["batch"], 20000, blocker["init"])
    tickets = [s.submit(h, c["problem"], i, c["batch"], K, c["init"]) for i, (h, c) in enumerate(zip(hs, mixed))]
    outs = [s.wait(tk, 60.0, traj=True) for tk in tickets]
    assert s.wait(tb, 60.0)[0]
    st = s.stats()
    s.close()
    assert all(o[0] for o in outs)
    assert st["launches"] >= 3, st   # the blocker, then at least one launch per shape
    for h, c, (_, _, traj) in zip(hs, mixed, outs):
        p = am.DeviceProblem(c["problem"], "f32")
        ds = am.DeviceState(c["init"], 5, c["n"], c["problem"]["q"], "f32")
        am.solve(h, p, ds, K)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ds.t["traj"].cpu().numpy(), traj)


def test_served_requests_match_the_oracle(am):
    """FP64 server: a mix of requests and a warm-started second request of
    one client, each against the FP64 oracle at 1e-8; the oracle's second
    solve starts from fresh samples and the multipliers of its own first
    solve (the warm start of Sec. IV)."""
    import oracle
    clients = _clients(3, cap=24)
    hs = [am.Handle.for_problem(c["problem"], "f64") for c in clients]
    K = 12
    s = am.Server(1 << 28, streams=2, max_per_launch=8, dtype="f64")
    tickets = [s.submit(h, c["problem"], i, c["batch"], K, c["init"]) for i, (h, c) in enumerate(zip(hs, clients))]
    outs = [s.wait(tk, 60.0, traj=True) for tk in tickets]
    c0 = clients[0]
    pb2 = inputs.replan_problem(c0["problem"], 1)
    init2 = inputs.make_initial(pb2, c0["batch"], 99)
    t2 = s.submit(hs[0], pb2, 0, c0["batch"], K, init2)
    warm = s.wait(t2, 60.0, traj=True)
    s.close()
    assert all(o[0] for o in outs) and warm[0]
    first = None
    for c, (_, _, traj) in zip(clients, outs):
        orc = oracle.Oracle(c["problem"])
        ost = oracle.state_from(c["problem"], c["init"])
        orc.solve(ost, K)
        x, y, p = orc.trajectories(ost)
        np.testing.assert_allclose(traj[:, 0], x, atol=1e-8, rtol=0)
        np.testing.assert_allclose(traj[:, 1], y, atol=1e-8, rtol=0)
        np.testing.assert_allclose(traj[:, 2], p, atol=1e-8, rtol=0)
        if first is None:
            first = ost
    orc = oracle.Oracle(pb2)
    ost = oracle.state_from(pb2, dict(init2, lam=first["lam"], lampsi=first["lampsi"]))
    orc.solve(ost, K)
    x, y, p = orc.trajectories(ost)
    np.testing.assert_allclose(warm[2][:, 0], x, atol=1e-8, rtol=0)
    np.testing.assert_allclose(warm[2][:, 1], y, atol=1e-8, rtol=0)
    np.testing.assert_allclose(warm[2][:, 2], p, atol=1e-8, rtol=0)


def test_all_nonfinite_request_reports_nonfinite(am):
    """A request whose every trajectory is NaN: am_server_best returns
    AM_ERR_NONFINITE; a finite request served beside it is unaffected."""
    clients = _clients(2, cap=32)
    hs = _handles(am, clients)
    bad = {k: np.full_like(np.asarray(v, np.float64), np.nan) for k, v in clients[0]["init"].items()}
    s = am.Server(1 << 28, streams=2, max_per_launch=8, select_best=True, fc_tol=0.05)
    t0 = s.submit(hs[0], clients[0]["problem"], 0, clients[0]["batch"], 5, bad)
    t1 = s.submit(hs[1], clients[1]["problem"], 1, clients[1]["batch"], 5, clients[1]["init"])
    assert s.wait(t0, 60.0)[0] and s.wait(t1, 60.0)[0]
    with pytest.raises(am.AmError) as e:
        s.best(t0)
    assert e.value.code == am.AM_ERR_NONFINITE
    assert s.best(t1)[0] >= 0
    s.close()


def test_warm_start_reuses_the_multipliers(am):
    """A client's next request starts from fresh samples and the multipliers of
    its previous result (the paper's MPC warm start of lambda): equal, bit for
    bit, to two direct solves chained through lambda."""
    import torch
    c = _clients(1)[0]
    h = _handles(am, [c])[0]
    pb2 = inputs.replan_problem(c["problem"], 1)
    init2 = inputs.make_initial(pb2, c["batch"], 99)
    s = am.Server(1 << 28, streams=2, max_per_launch=4)
    t1 = s.submit(h, c["problem"], 5, c["batch"], 8, c["init"])
    assert s.wait(t1, 60.0)[0]
    t2 = s.submit(h, pb2, 5, c["batch"], 8, init2)
    done, lat, warm = s.wait(t2, 60.0, traj=True)
    assert done and lat > 0
    s.close()
    p1 = am.DeviceProblem(c["problem"], "f32")
    d1 = am.DeviceState(c["init"], 5, c["n"], c["problem"]["q"], "f32")
    am.solve(h, p1, d1, 8)
    torch.cuda.synchronize()
    lam = d1.t["lam"].cpu().numpy().astype(np.float64)
    lamp = d1.t["lam_psi"].cpu().numpy().astype(np.float64)
    p2 = am.DeviceProblem(pb2, "f32")
    d2 = am.DeviceState(dict(init2, lam=lam, lam_psi=lamp), 5, c["n"], c["problem"]["q"], "f32")
    am.solve(h, p2, d2, 8)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(warm, d2.t["traj"].cpu().numpy())


def test_budget_admission_and_overlap(am):
    """With room for only a few requests at a time every request still
    completes; the budget is never exceeded and requests waited for memory."""
    clients = _clients(10, cap=256)
    hs = _handles(am, clients)
    q, nv = clients[0]["problem"]["q"], 11
    per = 256 * (10 * nv + 3 * q) * 4 + 2 * 30 * q * 4 + 1024
    budget = 3 * per
    s = am.Server(budget, streams=4, max_per_launch=8)
    tickets = [s.submit(h, c["problem"], i, c["batch"], 10, c["init"]) for i, (h, c) in enumerate(zip(hs, clients))]
    assert all(s.wait(t, 120.0)[0] for t in tickets)
    # a second round: warm blocks of idle clients are dropped to make room
    tickets = [s.submit(h, c["problem"], i, c["batch"], 10, c["init"]) for i, (h, c) in enumerate(zip(hs, clients))]
    assert all(s.wait(t, 120.0)[0] for t in tickets)
    st = s.stats()
    assert st["completed"] == 20
    assert st["peak_bytes"] <= budget
    assert st["memory_waits"] > 0
    s.close()


@pytest.mark.parametrize("mode", [1, 2])
def test_sequential_and_plain_modes_agree(am, mode):
    clients = _clients(3, cap=200)
    hs = _handles(am, clients)
    K = 10
    res = {}
    for md in (0, mode):
        s = am.Server(1 << 28, streams=2, max_per_launch=8, mode=md)
        tks = [s.submit(h, c["problem"], i, c["batch"], K, c["init"]) for i, (h, c) in enumerate(zip(hs, clients))]
        res[md] = [s.wait(t, 120.0, traj=True)[2] for t in tks]
        s.close()
    for a, b in zip(res[0], res[mode]):
        assert np.abs(a - b).max() < 1e-3


def test_oversized_request_rejected(am):
    c = _clients(1)[0]
    h = _handles(am, [c])[0]
    s = am.Server(4096, streams=1, max_per_launch=1)
    with pytest.raises(am.AmError) as e:
        s.submit(h, c["problem"], 0, c["batch"], 5, c["init"])
    assert e.value.code == am.AM_ERR_INVALID
    s.close()


def _best_rule(res, tol):
    """The selection rule of am_select_best, written out over numpy rows."""
    fin = res[:, 11] == 0
    ok = fin & (res[:, 0] <= tol)
    if ok.any():
        idx = np.flatnonzero(ok)
        return int(idx[np.lexsort((idx, res[idx, 7]))[0]])
    if fin.any():
        idx = np.flatnonzero(fin)
        return int(idx[np.lexsort((idx, res[idx, 0]))[0]])
    return -1


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_select_best_rule_on_planted_rows(am, dtype):
    """am_select_best on hand-made residual rows: least cost among rows under
    the collision tolerance, ties to the lower index, fallback to the least
    max |f_c|, -1 when every row is non-finite."""
    import torch
    c = _clients(1)[0]
    h = am.Handle.for_problem(c["problem"], dtype)
    ft = np.float32 if dtype == "f32" else np.float64
    rng = np.random.default_rng(3)
    for B, case in ((1, "one"), (37, "ties"), (700, "fallback"), (5000, "random"), (64, "nonfinite")):
        res = np.zeros((B, am.NRES), ft)
        res[:, 0] = rng.uniform(0.0, 0.2, B).astype(ft)
        res[:, 7] = np.round(rng.uniform(1.0, 5.0, B), 1).astype(ft)   # many equal costs
        if case == "fallback":
            res[:, 0] += 0.5
        if case == "nonfinite":
            res[:, 11] = 1.0
        if case == "ties":
            res[:, 0] = 0.01
            res[:, 7] = 2.0
            res[5:, 7] = 1.5
        t = torch.as_tensor(res, device="cuda")
        idx, cost, fc = am.select_best(h, t, 0.05)
        want = _best_rule(res, ft(0.05))
        assert idx == want, case
        if case == "ties":
            assert idx == 5
        if want >= 0:
            assert cost == res[want, 7] and fc == res[want, 0]


def test_server_reports_the_best_trajectory(am):
    """With select_best the server returns, per request, the trajectory that
    the selection rule picks from the residuals its solve wrote: the same
    index, cost and residual as the rule applied to the residuals of the
    direct batch solve."""
    import torch
    clients = _clients(4)
    hs = _handles(am, clients)
    K = 10
    s = am.Server(1 << 28, streams=2, max_per_launch=8, select_best=True, fc_tol=0.05)
    tickets = [s.submit(h, c["problem"], i, c["batch"], K, c["init"]) for i, (h, c) in enumerate(zip(hs, clients))]
    for tk in tickets:
        assert s.wait(tk, 60.0)[0]
    got = [s.best(tk) for tk in tickets]
    s.close()
    for (h, c), (idx, cost, fc) in zip(zip(hs, clients), got):
        p = am.DeviceProblem(c["problem"], "f32")
        ds = am.DeviceState(c["init"], 5, c["n"], c["problem"]["q"], "f32", residuals=True)
        am.solve(h, p, ds, K)
        torch.cuda.synchronize()
        r = ds.t["res"].cpu().numpy()
        want = _best_rule(r, np.float32(0.05))
        assert idx == want
        assert cost == pytest.approx(float(r[want, 7]), rel=0, abs=0)
        assert fc == pytest.approx(float(r[want, 0]), rel=0, abs=0)


def test_server_kkt_cache_by_shape(am):
    """Requests that name a shape instead of a handle get a handle from the
    server's KKT cache (one per distinct shape); results equal the direct
    solve with a handle built for the same shape."""
    import torch
    clients = _clients(6)
    K = 8
    s = am.Server(1 << 28, streams=2, max_per_launch=8)
    tickets = [s.submit(None, c["problem"], i, c["batch"], K, c["init"]) for i, c in enumerate(clients)]
    outs = [s.wait(tk, 60.0, traj=True) for tk in tickets]
    s.close()
    assert all(o[0] for o in outs)
    for c, (_, _, traj) in zip(clients, outs):
        h = am.Handle.for_problem(c["problem"], "f32")
        p = am.DeviceProblem(c["problem"], "f32")
        ds = am.DeviceState(c["init"], 5, c["n"], c["problem"]["q"], "f32")
        am.solve(h, p, ds, K)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ds.t["traj"].cpu().numpy(), traj)


def test_inputs_beyond_the_pinned_arena(am):
    """More queued input than the server's pinned host arena holds (64 MiB):
    the requests that do not fit go through the launch slot's staging, and
    every result still equals its direct solve (first, middle and last
    request checked)."""
    import torch
    c = inputs.serving_clients(1, seed=91)[0]
    B = 2048
    pb = c["problem"]
    init = inputs.make_initial(pb, B, 91, 0.5)
    h = am.Handle.for_problem(pb, "f32")
    per = (2 * len(pb["oa"]) * pb["q"] + 2 * len(pb["oa"]) + 5 * B * pb["nv"]) * 4
    count = (64 << 20) // per + 12
    K = 2
    srv = am.Server(1 << 31, streams=1, max_per_launch=64, idle_spin_us=2000)
    # a long request holds the only stream while the rest queue up, so their
    # inputs are all staged before any of them launches
    blocker = srv.submit(h, pb, 100000, 256, 40000, {k: v[:256] for k, v in init.items()})
    tickets = [srv.submit(h, pb, i, B, K, init) for i in range(count)]
    assert srv.wait(blocker, 120.0)[0]
    outs = {}
    for i, t in enumerate(tickets):
        done, _, tr = srv.wait(t, 120.0, traj=i in (0, count // 2, count - 1))
        assert done
        if tr is not None:
            outs[i] = tr
    assert srv.stats()["completed"] == count + 1
    srv.close()
    p = am.DeviceProblem(pb, "f32")
    ds = am.DeviceState(init, len(pb["r"]), len(pb["oa"]), pb["q"], "f32")
    am.solve(h, p, ds, K)
    torch.cuda.synchronize()
    ref = ds.t["traj"].cpu().numpy()
    for i, tr in outs.items():
        np.testing.assert_array_equal(tr, ref, err_msg=f"request {i}")
