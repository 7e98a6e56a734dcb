"""FP64 CPU oracle for the batched AM trajectory optimizer (arXiv 2109.13030).

TEST INFRASTRUCTURE ONLY.  This package wraps ``am_oracle.c`` (plain C, FP64)
through ctypes.  It is imported by the test suite, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product path, and it shares
no code with the GPU library.

A *problem* is a dict with the keys of ``amo_problem`` (see ``am_oracle.h``):
``q, nv, tf, r, ox, oy, oa, ob, rc, bx, by, bpsi, vmax, amax, rho, rho_psi,
flags``.  A *state* is a dict of float64 arrays ``cx, cc, cy, cs, cpsi`` [B, nv],
``lam`` [B, 4nv], ``lampsi`` [B, nv], ``alpha, d`` [B, m*n, q],
``av, dv, aa, da, psihat`` [B, q]; steps update it in place.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "am_oracle.c")
_LIB = os.path.join(_HERE, "libamoracle.so")

ALPHA_LITERAL = 1
XTILDE_SLACK = 2
PSI_NO_UNWRAP = 4
LAMPSI_LITERAL = 8
Q_CS_ZERO = 16

STEP_XI1, STEP_XI2, STEP_XI3, STEP_XI4, STEP_LAMBDA = 1, 2, 3, 4, 5
NRES = 12
RES_NAMES = ("fc_max", "fc_rms", "fv_max", "fa_max", "slack_max", "heading_max",
             "bc_max", "cost", "clear_level", "v_excess", "a_excess", "nonfinite")

_dp = ct.POINTER(ct.c_double)


class _Problem(ct.Structure):
    _fields_ = [("q", ct.c_int), ("nv", ct.c_int), ("tf", ct.c_double),
                ("m", ct.c_int), ("r", _dp), ("n", ct.c_int),
                ("ox", _dp), ("oy", _dp), ("oa", _dp), ("ob", _dp),
                ("rc", ct.c_double),
                ("bx", ct.c_double * 6), ("by", ct.c_double * 6), ("bpsi", ct.c_double * 6),
                ("vmax", ct.c_double), ("amax", ct.c_double),
                ("rho", ct.c_double), ("rho_psi", ct.c_double), ("flags", ct.c_uint)]


class _State(ct.Structure):
    _fields_ = [(k, _dp) for k in ("cx", "cc", "cy", "cs", "cpsi", "lam", "lampsi",
                                   "alpha", "d", "av", "dv", "aa", "da", "psihat")]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over trajectories)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
            os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "am_oracle.h"))):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_native() -> str:
    """The same source built -O3 -march=native for timing on the host it runs
    on (the CPU baseline); the library name carries a digest of the host's
    CPU flags, so another host builds its own."""
    import hashlib
    flags = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("flags"):
                flags = line
                break
    except OSError:
        pass
    tag = hashlib.sha256((flags + open(_SRC).read() + open(os.path.join(_HERE, "am_oracle.h")).read())
                         .encode()).hexdigest()[:12]
    path = os.path.join(_HERE, f"libamoracle_native_{tag}.so")
    if not os.path.exists(path):
        tmp = path + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, path)
    return path


NATIVE_FLAGS = "gcc -O3 -march=native -fopenmp"
_lib = None
_native = None


def _bind(L):
    L.amo_basis.argtypes = [ct.c_int, ct.c_int, ct.c_double, _dp, _dp, _dp]
    L.amo_create.argtypes = [ct.POINTER(_Problem), ct.POINTER(ct.c_int)]
    L.amo_create.restype = ct.c_void_p
    L.amo_free.argtypes = [ct.c_void_p]
    L.amo_matrices.argtypes = [ct.c_void_p, _dp, _dp, _dp]
    L.amo_step.argtypes = [ct.c_void_p, ct.c_int, ct.c_int, ct.POINTER(_State)]
    L.amo_solve.argtypes = [ct.c_void_p, ct.c_int, ct.c_int, ct.POINTER(_State), _dp, ct.c_int]
    L.amo_lagrangian.argtypes = [ct.c_void_p, ct.c_int, ct.POINTER(_State), _dp]
    L.amo_residuals.argtypes = [ct.c_void_p, ct.c_int, ct.POINTER(_State), _dp]
    return L


def native_lib():
    """The -O3 -march=native build (timing only)."""
    global _native
    if _native is None:
        _native = _bind(ct.CDLL(build_native()))
    return _native


def lib():
    global _lib
    if _lib is None:
        build()
        L = ct.CDLL(_LIB)
        _lib = _bind(L)
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def basis(q: int, nv: int, tf: float):
    """Bernstein matrices P, Pdot, Pddot of eq. (param), each [q, nv]."""
    P, Pd, Pdd = (np.zeros((q, nv)) for _ in range(3))
    if lib().amo_basis(q, nv, tf, _ptr(P), _ptr(Pd), _ptr(Pdd)) != 0:
        raise ValueError("invalid basis arguments")
    return P, Pd, Pdd


def empty_state(pb: dict, B: int) -> dict:
    q, nv = int(pb["q"]), int(pb["nv"])
    mn = len(pb["r"]) * len(pb["oa"])
    z = lambda *s: np.zeros(s)
    return dict(cx=z(B, nv), cc=z(B, nv), cy=z(B, nv), cs=z(B, nv), cpsi=z(B, nv),
                lam=z(B, 4 * nv), lampsi=z(B, nv), alpha=z(B, mn, q), d=z(B, mn, q),
                av=z(B, q), dv=z(B, q), aa=z(B, q), da=z(B, q), psihat=z(B, q))


def state_from(pb: dict, init: dict) -> dict:
    """Full float64 oracle state from an initial-state dict (missing keys = 0)."""
    B = np.asarray(init["cx"]).shape[0]
    st = empty_state(pb, B)
    for k, v in init.items():
        if k in st:
            st[k][...] = np.asarray(v, dtype=np.float64).reshape(st[k].shape)
    return st


class Oracle:
    """One problem (shared by the batch): setup matrices and LU factors.
    native=True uses the -O3 -march=native build (for timing)."""

    def __init__(self, pb: dict, native: bool = False):
        self.pb = pb
        self._L = native_lib() if native else lib()
        q, nv = int(pb["q"]), int(pb["nv"])
        self.q, self.nv = q, nv
        self.m, self.n = len(pb["r"]), len(pb["oa"])
        self._keep = dict(r=_f64(pb["r"]), ox=_f64(pb["ox"], (-1,)), oy=_f64(pb["oy"], (-1,)),
                          oa=_f64(pb["oa"]), ob=_f64(pb["ob"]))
        if self.n == 0:
            for k in ("ox", "oy", "oa", "ob"):
                self._keep[k] = np.zeros(1)
        p = _Problem()
        p.q, p.nv, p.tf = q, nv, float(pb["tf"])
        p.m, p.n = self.m, self.n
        p.r = _ptr(self._keep["r"])
        p.ox, p.oy = _ptr(self._keep["ox"]), _ptr(self._keep["oy"])
        p.oa, p.ob = _ptr(self._keep["oa"]), _ptr(self._keep["ob"])
        p.rc = float(pb["rc"])
        for k in ("bx", "by", "bpsi"):
            getattr(p, k)[:] = [float(v) for v in pb[k]]
        p.vmax, p.amax = float(pb["vmax"]), float(pb["amax"])
        p.rho = float(pb["rho"])
        p.rho_psi = float(pb.get("rho_psi", pb["rho"]))
        p.flags = int(pb.get("flags", 0))
        self._p = p
        status = ct.c_int(0)
        self._ctx = self._L.amo_create(ct.byref(p), ct.byref(status))
        if not self._ctx:
            raise ValueError(f"oracle setup failed with status {status.value}")

    def __del__(self):
        if getattr(self, "_ctx", None):
            self._L.amo_free(self._ctx)
            self._ctx = None

    def _st(self, st: dict):
        s = _State()
        B = st["cx"].shape[0]
        mn = self.m * self.n
        shapes = dict(cx=(B, self.nv), cc=(B, self.nv), cy=(B, self.nv), cs=(B, self.nv),
                      cpsi=(B, self.nv), lam=(B, 4 * self.nv), lampsi=(B, self.nv),
                      alpha=(B, mn, self.q), d=(B, mn, self.q), av=(B, self.q), dv=(B, self.q),
                      aa=(B, self.q), da=(B, self.q), psihat=(B, self.q))
        for k, shp in shapes.items():
            a = st[k]
            if a.dtype != np.float64 or not a.flags.c_contiguous or a.shape != shp:
                raise ValueError(f"state[{k}] must be C-contiguous float64 {shp}, got {a.dtype} {a.shape}")
            setattr(s, k, _ptr(a))
        return s, B

    def matrices(self):
        nF = 3 * self.q + self.m * self.n * self.q
        F = np.zeros((nF, 2 * self.nv))
        K1 = np.zeros((2 * self.nv + 6, 2 * self.nv + 6))
        K2 = np.zeros((self.nv + 6, self.nv + 6))
        self._L.amo_matrices(self._ctx, _ptr(F), _ptr(K1), _ptr(K2))
        return F, K1, K2

    def step(self, which: int, st: dict):
        s, B = self._st(st)
        rc = self._L.amo_step(self._ctx, B, which, ct.byref(s))
        if rc != 0:
            raise RuntimeError(f"amo_step failed: {rc}")

    def solve(self, st: dict, K: int, hist: bool = False, nthreads: int = 0):
        s, B = self._st(st)
        h = np.zeros((max(K, 1), B)) if hist else None
        rc = self._L.amo_solve(self._ctx, B, K, ct.byref(s), _ptr(h) if hist else None, nthreads)
        if rc != 0:
            raise RuntimeError(f"amo_solve failed: {rc}")
        return h[:K] if hist else None

    def lagrangian(self, st: dict):
        s, B = self._st(st)
        out = np.zeros(B)
        self._L.amo_lagrangian(self._ctx, B, ct.byref(s), _ptr(out))
        return out

    def residuals(self, st: dict):
        s, B = self._st(st)
        out = np.zeros((B, NRES))
        self._L.amo_residuals(self._ctx, B, ct.byref(s), _ptr(out))
        return out

    def trajectories(self, st: dict):
        """x, y, psi on the grid (eq. param) from the state's coefficients."""
        P, _, _ = basis(self.q, self.nv, float(self.pb["tf"]))
        return st["cx"] @ P.T, st["cy"] @ P.T, st["cpsi"] @ P.T
