"""The FP32 atan2 and sincos of the iteration kernels (csrc/am_device.h with
the coefficients of csrc/am_poly.h): the header is what its generator
writes, and an FP32 emulation of the kernels' evaluation order meets the
error bounds the kernels rely on (no GPU needed)."""
import re

import numpy as np

from paper_2109_13030_amd import gen_poly

f32 = np.float32


def _consts():
    text = open(gen_poly.HEADER).read()
    arr = {k: np.array([f32(float(v.rstrip("f"))) for v in re.search(k + r"\[\d+\] = \{([^}]*)\}", text)
                        .group(1).split(",")]) for k in ("kAtanP", "kSinS", "kCosC")}
    sc = {k: f32(float(re.search(k + r" = ([^;]*)f;", text).group(1)))
          for k in ("kHalfPiHi", "kHalfPiLo", "kTwoOverPi", "kHalfPi", "kPi")}
    return arr, sc


def fma(a, b, c):
    """fmaf: the FP32 product is exact in FP64; one rounding of the sum to FP64
    then to FP32 (a double rounding that can differ from fmaf by one unit in
    the last place in rare cases, well inside the bounds tested)."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(f32)


def atan2_f32(y, x, rcp_ulps=0):
    """The kernel's atan2: min/max ratio through a reciprocal (the hardware
    reciprocal is within one unit in the last place; rcp_ulps shifts it),
    r P(r^2) by Horner with fmaf, then the octant fix-ups."""
    arr, sc = _consts()
    ax, ay = np.abs(x), np.abs(y)
    mx, mn = np.maximum(ax, ay), np.minimum(ax, ay)
    rc = (f32(1) / mx).astype(f32)
    if rcp_ulps:
        rc = np.nextafter(rc, f32(np.inf) if rcp_ulps > 0 else f32(0)).astype(f32)
    r = (mn * rc).astype(f32)
    u = (r * r).astype(f32)
    p = np.full_like(u, arr["kAtanP"][0])
    for c in arr["kAtanP"][1:]:
        p = fma(p, u, np.full_like(u, c))
    a = (r * p).astype(f32)
    a = np.where(ay > ax, (sc["kHalfPi"] - a).astype(f32), a)
    a = np.where(x < 0, (sc["kPi"] - a).astype(f32), a)
    return np.copysign(a, y).astype(f32)


def sincos_f32(a):
    """The kernel's sincos: nearest multiple k of pi/2, two-constant
    reduction with fmaf, the two polynomials, quadrant selection."""
    arr, sc = _consts()
    k = np.rint((a * sc["kTwoOverPi"]).astype(f32)).astype(f32)
    r = fma(-k, np.full_like(a, sc["kHalfPiHi"]), a)
    r = fma(-k, np.full_like(a, sc["kHalfPiLo"]), r)
    u = (r * r).astype(f32)
    ps = np.full_like(u, arr["kSinS"][0])
    for c in arr["kSinS"][1:]:
        ps = fma(ps, u, np.full_like(u, c))
    sr = fma((r * u).astype(f32), ps, r)
    pc = np.full_like(u, arr["kCosC"][0])
    for c in arr["kCosC"][1:]:
        pc = fma(pc, u, np.full_like(u, c))
    cr = fma((u * u).astype(f32), pc, fma(np.full_like(u, f32(-0.5)), u, np.ones_like(u)))
    qd = k.astype(np.int64) & 3
    s0 = np.where(qd & 1, cr, sr)
    c0 = np.where(qd & 1, sr, cr)
    s = np.where(qd & 2, -s0, s0)
    c = np.where((qd + 1) & 2, -c0, c0)
    return s.astype(f32), c.astype(f32)


def test_header_is_the_generators_output():
    assert open(gen_poly.HEADER).read() == gen_poly.render()


def test_fits_are_near_minimax():
    """The FP64 fits equioscillate: their absolute error on the grid is within
    a few percent of its maximum at many points (Lawson's fixed point)."""
    patan, psin, pcos = gen_poly.fit()
    r = np.linspace(0, 1, 20001)
    e = np.abs(np.polyval(patan[::-1], r * r) * r - np.arctan(r))
    assert e.max() < 1e-8
    assert (e > 0.97 * e.max()).sum() >= 8


def test_atan2_error_bound():
    """Within 3.2e-7 rad of atan2 over 1e6 directions in all octants with a
    correctly rounded reciprocal, and within 3.7e-7 rad with the reciprocal
    one unit in the last place off either way (the hardware reciprocal's
    bound)."""
    th = np.linspace(-np.pi, np.pi, 1_000_001)
    rad = np.exp(np.linspace(-6, 6, th.size))
    x, y = (rad * np.cos(th)).astype(f32), (rad * np.sin(th)).astype(f32)
    want = np.arctan2(y.astype(np.float64), x.astype(np.float64))
    for ulps in (0, 1, -1):
        got = atan2_f32(y, x, ulps).astype(np.float64)
        d = np.abs(np.angle(np.exp(1j * (got - want))))
        assert d.max() < (3.2e-7 if ulps == 0 else 3.7e-7), (ulps, d.max())


def test_sincos_error_bound():
    """Within 1e-7 of sin and cos for |a| <= 1e3 (1e6 points) and exact on
    the quadrant boundaries' signs."""
    a = np.linspace(-1000.0, 1000.0, 1_000_001).astype(f32)
    s, c = sincos_f32(a)
    a64 = a.astype(np.float64)
    assert np.abs(s - np.sin(a64)).max() < 1e-7
    assert np.abs(c - np.cos(a64)).max() < 1e-7
    s0, c0 = sincos_f32(np.array([0.0], f32))
    assert s0[0] == 0.0 and c0[0] == 1.0
