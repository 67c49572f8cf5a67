"""Accuracy of the float64 series the render's control stage and the adjoint
evaluate on the GPU (exp2 and log2 by Tang's table-driven method, sin of a
phase in cycles by quarter-cycle folding + Taylor, expm1 by Taylor for small
arguments, sine and cosine by half-cycle reduction + Taylor), re-evaluated
here step by step in numpy float64 with the same reductions, tables and
numbers of terms, against numpy's library functions.  The render's parity
tests see these functions only through audio at 1e-4; this pins the ~1e-13
relative accuracy they are documented with (about 1e-16 per function)."""
import math

import numpy as np

LN2 = math.log(2.0)


def horner(coefs, x):
    p = np.full_like(x, coefs[0])
    for c in coefs[1:]:
        p = p * x + c
    return p


def _tables():
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2104_12922_amd", "csrc", "gen_series_tables.py")
    spec = importlib.util.spec_from_file_location("gen_series_tables", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    e, l, c = mod.tables()
    return (np.array([float(v) for v in e]), np.array([float(v) for v in l]),
            np.array([float(v) for v in c]))


EXP2_T, LOG2_T, INV_C = _tables()


def exp2_series(y):
    y = np.clip(y, -1100.0, 1023.0)
    nd = np.rint(y * 256.0)
    n = nd.astype(np.int64)
    z = (y - nd / 256.0) * LN2                       # exact difference
    p = horner([1.0 / math.factorial(k) for k in range(5, -1, -1)], z)
    return np.ldexp(EXP2_T[n & 255] * p, n >> 8)


def log2_series(x):
    m, e = np.frexp(x)
    low = m < 0.70710678118654752
    m = np.where(low, 2.0 * m, m)
    e = np.where(low, e - 1, e)
    j = np.rint((m - 1.0) * 256.0).astype(np.int64) + 76
    # u = fma(m, 1/c, -1): the product in extended precision, one rounding
    u = (m.astype(np.longdouble) * INV_C[j].astype(np.longdouble) - 1).astype(np.float64)
    p = horner([(-1.0) ** (k + 1) / k for k in range(7, 0, -1)], u)
    return (LOG2_T[j] + e.astype(np.float64)) + p * u / LN2


def sin_cycles_series(p):
    r = p - np.rint(p)
    r = np.where(r > 0.25, 0.5 - r, r)
    r = np.where(r < -0.25, -0.5 - r, r)
    a = 2.0 * math.pi * r
    coefs = [(-1.0) ** (k // 2) / math.factorial(k) for k in range(23, 0, -2)]
    return horner(coefs, a * a) * a


def expm1_small(x):
    return horner([1.0 / math.factorial(k) for k in range(8, 0, -1)], x) * x


def rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def test_exp2_series():
    y = np.random.default_rng(0).uniform(-1070.0, 30.0, 200000)
    assert rel(exp2_series(y), np.exp2(y)).max() < 1e-15
    assert exp2_series(np.array([-1200.0]))[0] == 0.0        # clamped, underflows to 0


def test_log2_series():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.random(100000), 10.0 ** rng.uniform(-300, 0, 100000),
                        1.0 - 10.0 ** rng.uniform(-15, -1, 50000)])
    x = x[(x > 0) & (x < 1)]
    ref = np.log2(x)
    assert (np.abs(log2_series(x) - ref) / np.maximum(np.abs(ref), 1e-3)).max() < 1e-14


def test_pow_from_series_matches_power():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.random(100000), 10.0 ** rng.uniform(-30, 0, 100000)])
    x = x[(x > 0) & (x < 1)]
    for alpha in (0.1, 0.5, 1.0, 2.0, 6.0):
        p = exp2_series(alpha * log2_series(x))
        assert rel(p, x ** alpha).max() < 1e-13


def test_sin_cycles_series():
    p = np.concatenate([np.random.default_rng(3).random(200000), [0.0, 0.25, 0.5, 0.75]])
    assert np.abs(sin_cycles_series(p) - np.sin(2.0 * np.pi * p)).max() < 2e-15


def test_expm1_small_branch():
    x = np.random.default_rng(4).uniform(-1.0 / 64, 1.0 / 64, 200000)
    assert rel(expm1_small(x), np.expm1(x)).max() < 1e-15


def sincos_cycles_series(th):
    n = np.rint(2.0 * th)
    a = (th - 0.5 * n) * 2.0 * math.pi
    a2 = a * a
    s = horner([(-1.0) ** k / math.factorial(2 * k + 1) for k in range(11, -1, -1)], a2) * a
    pc = horner([(-1.0) ** k / math.factorial(2 * k + 2) for k in range(10, -1, -1)], a2)
    c = 1.0 - a2 * pc
    sg = np.where(n.astype(np.int64) & 1, -1.0, 1.0)
    return sg * s, sg * c


def test_sincos_cycles_series():
    """sin and cos of 2 pi th by half-cycle reduction and degree-23/22 Taylor
    series (the phase adjoints of both VCOs), over phases of up to 2000 cycles:
    absolute error of a few float64 ulps of th, relative error near the zero
    crossings at float64 level."""
    rng = np.random.default_rng(5)
    th = np.concatenate([rng.uniform(-4.0, 4.0, 200000), rng.uniform(0.0, 2000.0, 100000),
                         np.arange(-8, 9) * 0.25])
    s, c = sincos_cycles_series(th)
    fr = th - np.rint(th)
    assert np.abs(s - np.sin(2.0 * np.pi * fr)).max() < 4e-15
    assert np.abs(c - np.cos(2.0 * np.pi * fr)).max() < 4e-15
    th0 = 0.5 + 1e-9 * rng.uniform(-1.0, 1.0, 1000)   # near a zero crossing of the sine
    r = th0 - 0.5                                        # exact
    s0, _ = sincos_cycles_series(th0)
    assert (np.abs(s0 + np.sin(2.0 * np.pi * r)) <= 1e-15 * np.abs(np.sin(2.0 * np.pi * r)) + 1e-24).all()
