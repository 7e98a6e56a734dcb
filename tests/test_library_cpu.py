"""The C-ABI library without a GPU: it loads, exports every function that
include/am.h declares, and rejects bad arguments on the host before any HIP
call."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "am.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(am_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def amlib():
    from paper_2109_13030_amd import am
    return am


def test_header_and_binding_agree(amlib):
    assert header_functions() == sorted(amlib.EXPORTS)


def test_library_exports_every_declared_symbol(amlib):
    L = amlib.lib()
    for name in header_functions():
        assert hasattr(L, name), name
    out = os.popen(f"nm -D --defined-only {amlib.LIB_PATH}").read()
    for name in header_functions():
        assert re.search(rf"\bT {name}\b", out), name


def _shape(amlib, **kw):
    r = np.array([-0.4, 0.0, 0.4])
    s = amlib.Shape()
    s.q, s.nv, s.tf, s.m = kw.get("q", 100), kw.get("nv", 11), kw.get("tf", 30.0), kw.get("m", 3)
    s.r_off = r.ctypes.data_as(ct.POINTER(ct.c_double)) if kw.get("r", True) else None
    s.n_obs, s.rho, s.rho_psi = kw.get("n", 4), kw.get("rho", 1.0), kw.get("rho_psi", 1.0)
    s.dtype, s.flags = kw.get("dtype", 0), kw.get("flags", 0)
    return s, r


@pytest.mark.parametrize("bad", [dict(q=2), dict(q=129), dict(nv=9), dict(tf=0.0), dict(tf=float("nan")),
                                 dict(m=0), dict(m=9), dict(r=False), dict(n=-1), dict(n=65), dict(rho=0.0),
                                 dict(rho_psi=-1.0), dict(dtype=3), dict(flags=64), dict(q=10, nv=11)])
def test_setup_rejects_bad_shapes(amlib, bad):
    L = amlib.lib()
    s, _keep = _shape(amlib, **bad)
    h = ct.c_void_p()
    rc = L.am_setup(ct.byref(s), ct.byref(h))
    assert rc == amlib.AM_ERR_INVALID
    assert not h.value
    assert len(L.am_last_error()) > 0


def test_null_arguments_rejected(amlib):
    L = amlib.lib()
    assert L.am_setup(None, None) == amlib.AM_ERR_INVALID
    p, st = amlib.Problem(), amlib.State()
    assert L.am_solve_batch(None, ct.byref(p), 1, 1, ct.byref(st), None) == amlib.AM_ERR_INVALID
    assert L.am_residuals(None, ct.byref(p), 1, ct.byref(st), None, None) == amlib.AM_ERR_INVALID
    assert L.am_solve_batch_plain(None, ct.byref(p), 1, 1, ct.byref(st), None, 0, None) == amlib.AM_ERR_INVALID
    v = ct.c_size_t()
    assert L.am_multi_workspace_size(-1, ct.byref(v)) == amlib.AM_ERR_INVALID
    assert L.am_multi_workspace_size(3, ct.byref(v)) == amlib.AM_OK and v.value >= 3 * 400
    assert L.am_solve_multi(0, None, None, None, None, None, None, 0, None) == amlib.AM_OK
    assert L.am_solve_multi(2, None, None, None, None, None, None, 0, None) == amlib.AM_ERR_INVALID
    i = ct.c_int32()
    assert L.am_set_tile(None, 2) == amlib.AM_ERR_INVALID
    assert L.am_set_waves(None, 2) == amlib.AM_ERR_INVALID
    assert L.am_get_waves(None, ct.byref(i)) == amlib.AM_ERR_INVALID
    assert L.am_autotune(None, None, 1, 1, None, None, None, None, None) == amlib.AM_ERR_INVALID
    assert L.am_autotune_multi(0, None, None, None, None, None, None, 0, None, None, None, None) == amlib.AM_ERR_INVALID
    assert L.am_select_best(None, 1, None, 0.1, None, None, None) == amlib.AM_ERR_INVALID
    assert L.am_server_best(None, 0, ct.byref(i), None, None) == amlib.AM_ERR_INVALID
    L.am_destroy(None)


@pytest.mark.parametrize("bad", [dict(hbm_budget=0), dict(streams=0), dict(streams=17), dict(max_per_launch=0),
                                 dict(max_per_launch=257), dict(mode=3), dict(dtype=2), dict(idle_spin_us=-1),
                                 dict(idle_spin_us=1000001)])
def test_server_rejects_bad_config(amlib, bad):
    L = amlib.lib()
    c = amlib.ServerConfig()
    c.hbm_budget, c.streams, c.max_per_launch, c.mode, c.dtype = 1 << 26, 2, 8, 0, 0
    for k, v in bad.items():
        setattr(c, k, v)
    s = ct.c_void_p()
    assert L.am_server_create(ct.byref(c), ct.byref(s)) == amlib.AM_ERR_INVALID
    assert not s.value
    assert len(L.am_last_error()) > 0
    assert L.am_server_submit(None, None, None) == amlib.AM_ERR_INVALID
    L.am_server_destroy(None)
