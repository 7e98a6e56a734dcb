"""Thin Python binding of the C-ABI in include/am.h (ctypes).

Argument marshalling only: every step of the iteration runs in the HIP
library ``libam_hip.so``.  PyTorch provides device memory and streams.  The
library must have been built (``python -m paper_2109_13030_amd.build``);
nothing here falls back to another implementation.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libam_hip.so")

AM_OK, AM_ERR_INVALID, AM_ERR_HIP, AM_ERR_SINGULAR, AM_ERR_NONFINITE, AM_ERR_NOMEM = 0, -1, -2, -4, -5, -6
AM_F32, AM_F64 = 0, 1
ALPHA_LITERAL, XTILDE_SLACK, PSI_NO_UNWRAP, LAMPSI_LITERAL, Q_CS_ZERO = 1, 2, 4, 8, 16
PLAIN_BF16X3 = 32
NRES = 12
RES_NAMES = ("fc_max", "fc_rms", "fv_max", "fa_max", "slack_max", "heading_max",
             "bc_max", "cost", "clear_level", "v_excess", "a_excess", "nonfinite")

# every function the header declares
EXPORTS = ("am_setup", "am_destroy", "am_last_error", "am_solve_batch", "am_plain_workspace_size",
           "am_solve_batch_plain", "am_multi_workspace_size", "am_solve_multi", "am_residuals",
           "am_setup_matrices", "am_server_create", "am_server_submit", "am_server_wait",
           "am_server_stats", "am_server_destroy", "am_set_tile", "am_get_tile", "am_autotune",
           "am_autotune_multi", "am_select_best", "am_server_best", "am_set_waves", "am_get_waves",
           "am_solve_multi_static")
STATIC_MAX_PROBLEMS = 128   # AM_STATIC_MAX_PROBLEMS
TILES = (1, 2, 4)
WAVES = (2, 3)
LAUNCHES = tuple((t, w) for w in WAVES for t in TILES)   # order of the autotuner's times
SERVE_CONTINUOUS, SERVE_SEQUENTIAL, SERVE_PLAIN = 0, 1, 2


class AmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class Shape(ct.Structure):
    _fields_ = [("q", ct.c_int32), ("nv", ct.c_int32), ("tf", ct.c_double), ("m", ct.c_int32),
                ("r_off", ct.POINTER(ct.c_double)), ("n_obs", ct.c_int32), ("rho", ct.c_double),
                ("rho_psi", ct.c_double), ("dtype", ct.c_int32), ("flags", ct.c_uint32)]


class Problem(ct.Structure):
    _fields_ = [("obs_x", ct.c_void_p), ("obs_y", ct.c_void_p), ("obs_a", ct.c_void_p),
                ("obs_b", ct.c_void_p), ("r_circle", ct.c_double), ("bc_x", ct.c_double * 6),
                ("bc_y", ct.c_double * 6), ("bc_psi", ct.c_double * 6), ("v_max", ct.c_double),
                ("a_max", ct.c_double)]


class State(ct.Structure):
    _fields_ = [(k, ct.c_void_p) for k in ("cx", "cc", "cy", "cs", "cpsi", "lam", "lam_psi",
                                           "alpha", "d", "va", "traj", "res")]


class ServerConfig(ct.Structure):
    _fields_ = [("hbm_budget", ct.c_size_t), ("streams", ct.c_int32), ("max_per_launch", ct.c_int32),
                ("mode", ct.c_int32), ("dtype", ct.c_int32), ("select_best", ct.c_int32),
                ("fc_tol", ct.c_double), ("idle_spin_us", ct.c_int32)]


class Request(ct.Structure):
    _fields_ = [("handle", ct.c_void_p), ("shape", ct.POINTER(Shape)), ("client", ct.c_int32),
                ("batch", ct.c_int32), ("iters", ct.c_int32),
                ("obs_x", ct.POINTER(ct.c_double)), ("obs_y", ct.POINTER(ct.c_double)),
                ("obs_a", ct.POINTER(ct.c_double)), ("obs_b", ct.POINTER(ct.c_double)),
                ("r_circle", ct.c_double), ("bc_x", ct.c_double * 6), ("bc_y", ct.c_double * 6),
                ("bc_psi", ct.c_double * 6), ("v_max", ct.c_double), ("a_max", ct.c_double),
                ("init", ct.POINTER(ct.c_double))]


_lib = None


def lib():
    """Loads libam_hip.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2109_13030_amd.build`")
        L = ct.CDLL(LIB_PATH)
        vp, i32, sz = ct.c_void_p, ct.c_int32, ct.c_size_t
        L.am_setup.argtypes = [ct.POINTER(Shape), ct.POINTER(vp)]
        L.am_destroy.argtypes = [vp]
        L.am_destroy.restype = None
        L.am_last_error.restype = ct.c_char_p
        L.am_solve_batch.argtypes = [vp, ct.POINTER(Problem), i32, i32, ct.POINTER(State), vp]
        L.am_plain_workspace_size.argtypes = [vp, i32, ct.POINTER(sz)]
        L.am_solve_batch_plain.argtypes = [vp, ct.POINTER(Problem), i32, i32, ct.POINTER(State), vp, sz, vp]
        L.am_multi_workspace_size.argtypes = [i32, ct.POINTER(sz)]
        L.am_solve_multi.argtypes = [i32, ct.POINTER(vp), ct.POINTER(Problem), ct.POINTER(i32),
                                     ct.POINTER(i32), ct.POINTER(State), vp, sz, vp]
        L.am_residuals.argtypes = [vp, ct.POINTER(Problem), i32, ct.POINTER(State), vp, vp]
        L.am_setup_matrices.argtypes = [vp, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double),
                                        ct.POINTER(ct.c_double)]
        L.am_server_create.argtypes = [ct.POINTER(ServerConfig), ct.POINTER(vp)]
        L.am_server_submit.argtypes = [vp, ct.POINTER(Request), ct.POINTER(ct.c_int64)]
        L.am_server_wait.argtypes = [vp, ct.c_int64, ct.c_double, ct.POINTER(i32), ct.POINTER(ct.c_double), vp]
        L.am_server_stats.argtypes = [vp, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64), ct.POINTER(sz),
                                      ct.POINTER(ct.c_int64)]
        L.am_server_destroy.argtypes = [vp]
        L.am_server_destroy.restype = None
        L.am_set_tile.argtypes = [vp, i32]
        L.am_get_tile.argtypes = [vp, ct.POINTER(i32)]
        L.am_set_waves.argtypes = [vp, i32]
        L.am_get_waves.argtypes = [vp, ct.POINTER(i32)]
        L.am_autotune.argtypes = [vp, ct.POINTER(Problem), i32, i32, ct.POINTER(State), vp, ct.POINTER(i32),
                                  ct.POINTER(i32), ct.POINTER(ct.c_float)]
        L.am_solve_multi_static.argtypes = [i32, ct.POINTER(vp), ct.POINTER(Problem), ct.POINTER(i32),
                                            ct.POINTER(i32), ct.POINTER(State), vp]
        L.am_autotune_multi.argtypes = [i32, ct.POINTER(vp), ct.POINTER(Problem), ct.POINTER(i32), ct.POINTER(i32),
                                        ct.POINTER(State), vp, sz, vp, ct.POINTER(i32), ct.POINTER(i32),
                                        ct.POINTER(ct.c_float)]
        L.am_select_best.argtypes = [vp, i32, vp, ct.c_double, vp, vp, vp]
        L.am_server_best.argtypes = [vp, ct.c_int64, ct.POINTER(i32), ct.POINTER(ct.c_double),
                                     ct.POINTER(ct.c_double)]
        _lib = L
    return _lib


def check(rc: int):
    if rc != AM_OK:
        raise AmError(rc, lib().am_last_error().decode())


def _torch():
    import torch
    return torch


def _dt(dtype: str):
    torch = _torch()
    return torch.float64 if dtype == "f64" else torch.float32


def _ptr(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else ct.c_void_p(0)


def _stream_ptr(stream):
    if stream is None:
        return ct.c_void_p(_torch().cuda.current_stream().cuda_stream)
    return ct.c_void_p(stream.cuda_stream)


class Handle:
    """am_setup for one problem shape (KKT family member)."""

    def __init__(self, q: int, nv: int, tf: float, r_off, n_obs: int, rho: float, rho_psi: float | None = None,
                 dtype: str = "f32", flags: int = 0):
        self.r_off = np.ascontiguousarray(np.asarray(r_off, dtype=np.float64))
        s = Shape()
        s.q, s.nv, s.tf, s.m = int(q), int(nv), float(tf), len(self.r_off)
        s.r_off = self.r_off.ctypes.data_as(ct.POINTER(ct.c_double))
        s.n_obs, s.rho = int(n_obs), float(rho)
        s.rho_psi = float(rho if rho_psi is None else rho_psi)
        s.dtype = AM_F64 if dtype == "f64" else AM_F32
        s.flags = int(flags)
        self.dtype, self.q, self.nv, self.m, self.n = dtype, int(q), int(nv), len(self.r_off), int(n_obs)
        self.flags = int(flags)
        h = ct.c_void_p()
        check(lib().am_setup(ct.byref(s), ct.byref(h)))
        self._h = h

    @classmethod
    def for_problem(cls, pb: dict, dtype: str = "f32"):
        return cls(pb["q"], pb["nv"], pb["tf"], pb["r"], len(pb["oa"]), pb["rho"], pb.get("rho_psi", pb["rho"]),
                   dtype=dtype, flags=int(pb.get("flags", 0)))

    @property
    def ptr(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().am_destroy(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def tile(self) -> int:
        v = ct.c_int32()
        check(lib().am_get_tile(self._h, ct.byref(v)))
        return v.value

    @tile.setter
    def tile(self, t: int):
        check(lib().am_set_tile(self._h, int(t)))

    @property
    def waves(self) -> int:
        v = ct.c_int32()
        check(lib().am_get_waves(self._h, ct.byref(v)))
        return v.value

    @waves.setter
    def waves(self, w: int):
        check(lib().am_set_waves(self._h, int(w)))

    def matrices(self):
        """(KKT1^-1, KKT2^-1, basis[3, q, nv]) in Bernstein coordinates, FP64."""
        nv, q = self.nv, self.q
        k1 = np.zeros((2 * nv + 6, 2 * nv + 6))
        k2 = np.zeros((nv + 6, nv + 6))
        bs = np.zeros((3, q, nv))
        dp = ct.POINTER(ct.c_double)
        check(lib().am_setup_matrices(self._h, k1.ctypes.data_as(dp), k2.ctypes.data_as(dp), bs.ctypes.data_as(dp)))
        return k1, k2, bs


class DeviceProblem:
    """Obstacle table of one problem in device memory plus the scalar data."""

    def __init__(self, pb: dict, dtype: str = "f32", device="cuda"):
        torch = _torch()
        dt = _dt(dtype)
        n, q = len(pb["oa"]), int(pb["q"])
        self.ox = torch.as_tensor(np.asarray(pb["ox"], np.float64).reshape(n, q), dtype=dt, device=device).contiguous()
        self.oy = torch.as_tensor(np.asarray(pb["oy"], np.float64).reshape(n, q), dtype=dt, device=device).contiguous()
        self.oa = torch.as_tensor(np.asarray(pb["oa"], np.float64), dtype=dt, device=device).contiguous()
        self.ob = torch.as_tensor(np.asarray(pb["ob"], np.float64), dtype=dt, device=device).contiguous()
        p = Problem()
        p.obs_x, p.obs_y, p.obs_a, p.obs_b = (_ptr(t) if n > 0 else ct.c_void_p(0)
                                              for t in (self.ox, self.oy, self.oa, self.ob))
        p.r_circle = float(pb["rc"])
        p.bc_x[:] = [float(v) for v in pb["bx"]]
        p.bc_y[:] = [float(v) for v in pb["by"]]
        p.bc_psi[:] = [float(v) for v in pb["bpsi"]]
        p.v_max, p.a_max = float(pb["vmax"]), float(pb["amax"])
        self.c = p


class DeviceState:
    """Per-batch state as device tensors (row-major, time fastest)."""

    KEYS = ("cx", "cc", "cy", "cs", "cpsi", "lam", "lam_psi")

    def __init__(self, init: dict, m: int, n: int, q: int, dtype: str = "f32", device="cuda",
                 outputs: bool = True, projections: bool = False, residuals: bool = False):
        torch = _torch()
        dt = _dt(dtype)
        B, nv = np.asarray(init["cx"]).shape
        self.B, self.nv, self.q, self.m, self.n = B, nv, q, m, n
        src = dict(init)
        src.setdefault("cc", np.zeros((B, nv)))
        src.setdefault("cs", np.zeros((B, nv)))
        src.setdefault("lam", np.zeros((B, 4 * nv)))
        if "lam_psi" not in src:
            src["lam_psi"] = src.get("lampsi", np.zeros((B, nv)))
        self.t = {}
        for k in self.KEYS:
            self.t[k] = torch.as_tensor(np.asarray(src[k], np.float64), dtype=dt, device=device).contiguous()
        self.t["traj"] = torch.zeros((B, 3, q), dtype=dt, device=device) if outputs else None
        self.t["va"] = torch.zeros((B, 4, q), dtype=dt, device=device) if projections else None
        self.t["alpha"] = torch.zeros((B, m * n, q), dtype=dt, device=device) if projections else None
        self.t["d"] = torch.zeros((B, m * n, q), dtype=dt, device=device) if projections else None
        self.t["res"] = torch.zeros((B, NRES), dtype=dt, device=device) if residuals else None

    @property
    def c(self) -> State:
        s = State()
        for k in ("cx", "cc", "cy", "cs", "cpsi", "lam", "lam_psi", "alpha", "d", "va", "traj", "res"):
            setattr(s, k, _ptr(self.t.get(k)))
        return s

    def load_coefficients(self, init: dict):
        """Overwrites the coefficients (cx, cc, cy, cs, cpsi; missing ones = 0)
        in place and keeps the multipliers (a warm start)."""
        torch = _torch()
        for k in ("cx", "cc", "cy", "cs", "cpsi"):
            v = init.get(k)
            src = np.zeros((self.B, self.nv)) if v is None else np.asarray(v, np.float64).reshape(self.B, self.nv)
            self.t[k].copy_(torch.as_tensor(src, dtype=self.t[k].dtype))

    def numpy(self) -> dict:
        return {k: (v.detach().cpu().numpy().astype(np.float64) if v is not None else None) for k, v in self.t.items()}


def solve(h: Handle, p: DeviceProblem, st: DeviceState, iters: int, stream=None):
    check(lib().am_solve_batch(h.ptr, ct.byref(p.c), st.B, int(iters), ct.byref(st.c), _stream_ptr(stream)))


def plain_workspace_size(h: Handle, batch: int) -> int:
    v = ct.c_size_t()
    check(lib().am_plain_workspace_size(h.ptr, int(batch), ct.byref(v)))
    return v.value


def solve_plain(h: Handle, p: DeviceProblem, st: DeviceState, iters: int, workspace, stream=None):
    check(lib().am_solve_batch_plain(h.ptr, ct.byref(p.c), st.B, int(iters), ct.byref(st.c),
                                     _ptr(workspace), workspace.numel() * workspace.element_size(),
                                     _stream_ptr(stream)))


def multi_workspace_size(nprob: int) -> int:
    v = ct.c_size_t()
    check(lib().am_multi_workspace_size(int(nprob), ct.byref(v)))
    return v.value


def solve_multi(handles, problems, states, iters, workspace, stream=None):
    k = len(handles)
    H = (ct.c_void_p * k)(*[h.ptr.value for h in handles])
    P = (Problem * k)(*[p.c for p in problems])
    Bs = (ct.c_int32 * k)(*[s.B for s in states])
    Ks = (ct.c_int32 * k)(*([int(iters)] * k if np.isscalar(iters) else [int(v) for v in iters]))
    S = (State * k)(*[s.c for s in states])
    check(lib().am_solve_multi(k, H, P, Bs, Ks, S, _ptr(workspace), workspace.numel() * workspace.element_size(),
                               _stream_ptr(stream)))


def solve_multi_static(handles, problems, states, iters, stream=None):
    """am_solve_multi with the problem table in the library's static device
    array (no workspace, nothing allocated)."""
    k = len(handles)
    H = (ct.c_void_p * max(k, 1))(*[h.ptr.value for h in handles])
    P = (Problem * max(k, 1))(*[p.c for p in problems])
    Bs = (ct.c_int32 * max(k, 1))(*[s.B for s in states])
    Ks = (ct.c_int32 * max(k, 1))(*([int(iters)] * k if np.isscalar(iters) else [int(v) for v in iters]))
    S = (State * max(k, 1))(*[s.c for s in states])
    check(lib().am_solve_multi_static(k, H, P, Bs, Ks, S, _stream_ptr(stream)))


def autotune(h: Handle, p: DeviceProblem, scratch: DeviceState, iters: int, stream=None):
    """Picks the fastest launch configuration for this batch (overwrites
    scratch); returns ((tile, waves), {(tile, waves): ms})."""
    bt, bw = ct.c_int32(), ct.c_int32()
    times = (ct.c_float * len(LAUNCHES))()
    check(lib().am_autotune(h.ptr, ct.byref(p.c), scratch.B, int(iters), ct.byref(scratch.c), _stream_ptr(stream),
                            ct.byref(bt), ct.byref(bw), times))
    return (bt.value, bw.value), {c: v for c, v in zip(LAUNCHES, list(times)) if v >= 0}


def autotune_multi(handles, problems, scratch_states, iters, workspace, stream=None):
    k = len(handles)
    H = (ct.c_void_p * k)(*[h.ptr.value for h in handles])
    P = (Problem * k)(*[p.c for p in problems])
    Bs = (ct.c_int32 * k)(*[s.B for s in scratch_states])
    Ks = (ct.c_int32 * k)(*([int(iters)] * k))
    S = (State * k)(*[s.c for s in scratch_states])
    bt, bw = ct.c_int32(), ct.c_int32()
    times = (ct.c_float * len(LAUNCHES))()
    check(lib().am_autotune_multi(k, H, P, Bs, Ks, S, _ptr(workspace), workspace.numel() * workspace.element_size(),
                                  _stream_ptr(stream), ct.byref(bt), ct.byref(bw), times))
    return (bt.value, bw.value), {c: v for c, v in zip(LAUNCHES, list(times)) if v >= 0}


def residuals(h: Handle, p: DeviceProblem, st: DeviceState, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty((st.B, NRES), dtype=_dt(h.dtype), device=st.t["cx"].device)
    check(lib().am_residuals(h.ptr, ct.byref(p.c), st.B, ct.byref(st.c), _ptr(out), _stream_ptr(stream)))
    return out


def select_best(h: Handle, res, fc_tol: float, stream=None):
    """am_select_best on residual rows `res` [B, NRES] (device tensor):
    returns (index, cost, max |f_c|) of the best trajectory (synchronises)."""
    torch = _torch()
    idx = torch.full((1,), -2, dtype=torch.int32, device=res.device)
    vals = torch.zeros((2,), dtype=res.dtype, device=res.device)
    check(lib().am_select_best(h.ptr, int(res.shape[0]), _ptr(res), float(fc_tol), _ptr(idx), _ptr(vals),
                               _stream_ptr(stream)))
    v = vals.cpu().numpy()
    return int(idx.item()), float(v[0]), float(v[1])


class Server:
    """Continuous-batching replanning server (am_server_*)."""

    def __init__(self, hbm_budget: int, streams: int = 2, max_per_launch: int = 64,
                 mode: int = SERVE_CONTINUOUS, dtype: str = "f32", select_best: bool = False,
                 fc_tol: float = 0.05, idle_spin_us: int = 0):
        c = ServerConfig()
        c.hbm_budget, c.streams, c.max_per_launch = int(hbm_budget), int(streams), int(max_per_launch)
        c.mode, c.dtype = int(mode), AM_F64 if dtype == "f64" else AM_F32
        c.select_best, c.fc_tol = int(bool(select_best)), float(fc_tol)
        c.idle_spin_us = int(idle_spin_us)
        self.dtype = dtype
        s = ct.c_void_p()
        check(lib().am_server_create(ct.byref(c), ct.byref(s)))
        self._s = s
        self._meta = {}

    def submit(self, h, pb: dict, client: int, batch: int, iters: int, init=None) -> int:
        """Queues a request; with h = None the server takes the handle for
        the problem's shape from its KKT cache."""
        r = Request()
        keep_shape = None
        if h is None:
            roff = np.ascontiguousarray(np.asarray(pb["r"], np.float64))
            sh = Shape()
            sh.q, sh.nv, sh.tf, sh.m = int(pb["q"]), int(pb["nv"]), float(pb["tf"]), len(roff)
            sh.r_off = roff.ctypes.data_as(ct.POINTER(ct.c_double))
            sh.n_obs, sh.rho = len(pb["oa"]), float(pb["rho"])
            sh.rho_psi = float(pb.get("rho_psi", pb["rho"]))
            sh.dtype = AM_F64 if self.dtype == "f64" else AM_F32
            sh.flags = int(pb.get("flags", 0))
            keep_shape = (roff, sh)
            r.handle, r.shape = None, ct.pointer(sh)
            nv, q = sh.nv, sh.q
        else:
            r.handle = h.ptr
            nv, q = h.nv, h.q
        r.client, r.batch, r.iters = int(client), int(batch), int(iters)
        dp = ct.POINTER(ct.c_double)
        keep = [np.ascontiguousarray(np.asarray(pb[k], np.float64)) for k in ("ox", "oy", "oa", "ob")]
        r.obs_x, r.obs_y, r.obs_a, r.obs_b = (a.ctypes.data_as(dp) for a in keep)
        r.r_circle = float(pb["rc"])
        r.bc_x[:] = [float(v) for v in pb["bx"]]
        r.bc_y[:] = [float(v) for v in pb["by"]]
        r.bc_psi[:] = [float(v) for v in pb["bpsi"]]
        r.v_max, r.a_max = float(pb["vmax"]), float(pb["amax"])
        ini = None
        if init is not None:
            z = np.zeros((batch, nv))
            ini = np.ascontiguousarray(np.stack([np.asarray(init.get(k, z), np.float64)
                                                 for k in ("cx", "cc", "cy", "cs", "cpsi")], 1))
            r.init = ini.ctypes.data_as(dp)
        t = ct.c_int64()
        check(lib().am_server_submit(self._s, ct.byref(r), ct.byref(t)))
        del keep_shape
        self._meta[t.value] = (batch, q)
        return t.value

    def wait(self, ticket: int, timeout: float = -1.0, traj: bool = False):
        """(done, latency_s, traj [B, 3, q] or None)."""
        done, lat = ct.c_int32(), ct.c_double()
        out = None
        if traj:
            B, q = self._meta[ticket]
            out = np.zeros((B, 3, q), dtype=np.float64 if self.dtype == "f64" else np.float32)
        check(lib().am_server_wait(self._s, int(ticket), float(timeout), ct.byref(done), ct.byref(lat),
                                   out.ctypes.data_as(ct.c_void_p) if out is not None else None))
        return bool(done.value), lat.value, out

    def best(self, ticket: int):
        """(index, cost, max |f_c|) of the best trajectory of a finished request."""
        i, c, f = ct.c_int32(), ct.c_double(), ct.c_double()
        check(lib().am_server_best(self._s, int(ticket), ct.byref(i), ct.byref(c), ct.byref(f)))
        return i.value, c.value, f.value

    def stats(self):
        c, l, m = ct.c_int64(), ct.c_int64(), ct.c_int64()
        p = ct.c_size_t()
        check(lib().am_server_stats(self._s, ct.byref(c), ct.byref(l), ct.byref(p), ct.byref(m)))
        return dict(completed=c.value, launches=l.value, peak_bytes=p.value, memory_waits=m.value)

    def close(self):
        if getattr(self, "_s", None) and self._s.value:
            lib().am_server_destroy(self._s)
            self._s = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
