"""FP64 unary ops of the op-list kernels against the host C library, in ulps.

Each op runs as one index task over a 1-D store (one launch point), through
the C ABI.  Inputs cover every binade (uniform bit patterns, denormals
included), the neighbourhoods of the points where the kernels change
argument reduction or formula, and the special values; the oracle is
libm called element by element.  NaN must map to NaN and infinities and
zeros must match exactly.
"""
import numpy as np
import pytest

import synth
from gpu_util import ctx, note, upload
from oracle import cnum

pytestmark = pytest.mark.gpu

SPECIALS = [0.0, -0.0, np.inf, -np.inf, np.nan, 1.0, -1.0, 5e-324, -5e-324, 2.2250738585072014e-308,
            1.7976931348623157e308, -1.7976931348623157e308, 0.5, 2.0]


def _bits(seed, n, lo, hi):
    """n doubles whose bit patterns are uniform in [lo, hi)."""
    r = synth.raw64(seed, 0, n)
    b = np.uint64(lo) + r % np.uint64(hi - lo)
    return b.view(np.float64)


def _around(x0, k):
    """x0 and its k nearest neighbours on each side."""
    return x0 + np.arange(-k, k + 1) * np.spacing(abs(x0))


def _run(op, x):
    c = ctx()
    n = x.size
    hx = upload(c, x)
    hy = c.store_create([n], "f64")
    t = c.part_tiling([n])
    c.submit(op, [1], [(hx, t, "R"), (hy, t, "W")])
    c.flush()
    return c.store_read(hy, [n], "f64")


def _ulps(g, o):
    """Distance in representable doubles (+0 and -0 count as one value)."""
    a, b = g.view(np.int64), o.view(np.int64)
    lo = np.iinfo(np.int64).min
    oa, ob = np.where(a < 0, lo - a, a), np.where(b < 0, lo - b, b)
    same = (oa >= 0) == (ob >= 0)
    with np.errstate(over="ignore"):
        d_same = np.abs(oa - ob).astype(np.float64)   # exact: both on one side of zero
    d_cross = np.abs(oa).astype(np.float64) + np.abs(ob).astype(np.float64)
    return np.where(same, d_same, d_cross)


def _check(op, x, g, o, max_ulp):
    nan_g, nan_o = np.isnan(g), np.isnan(o)
    assert np.array_equal(nan_g, nan_o), "%s: NaN at %s" % (op, x[nan_g != nan_o][:5])
    fin = ~nan_o & np.isfinite(o)
    inf = ~nan_o & ~np.isfinite(o)
    assert np.array_equal(g[inf], o[inf]), "%s: infinities differ at %s" % (op, x[inf][g[inf] != o[inf]][:5])
    zero = fin & (o == 0)
    assert np.array_equal(np.signbit(g[zero]), np.signbit(o[zero])), "%s: sign of zero" % op
    d = _ulps(g[fin], o[fin])
    worst = int(d.max()) if d.size else 0
    note("%s: %d values, max %d ulp, mean %.3f ulp" % (op, x.size, worst, float(d.mean()) if d.size else 0.0))
    if worst > max_ulp:
        i = int(np.argmax(d))
        xs = x[fin][i]
        pytest.fail("%s: %d ulp at x=%r (got %r, libm %r)" % (op, worst, xs, g[fin][i], o[fin][i]))


def test_log_f64():
    T = float(np.sqrt(0.5))
    x = np.concatenate([
        _bits(11, 1 << 18, 1, 0x7FF0000000000000),          # every positive binade
        1.0 + synth.uniform(12, 0, 1 << 16, -1e-3, 1e-3),   # log near 0
        _around(1.0, 2000), _around(T, 200), _around(2 * T, 200), _around(0.5, 200), _around(2.0, 200),
        -_bits(13, 512, 1, 0x7FF0000000000000),              # negative: NaN
        np.array(SPECIALS)])
    note("log n=%d" % x.size)
    _check("log", x, _run("log", x), cnum.log(x), 2)


def test_erf_f64():
    s = 0.84375
    x = np.concatenate([
        synth.uniform(21, 0, 1 << 18, -7.0, 7.0),
        _bits(22, 1 << 16, 1, 0x3FF0000000000000),           # (0, 1) over every binade
        -_bits(23, 1 << 16, 1, 0x3FF0000000000000),
        _around(s, 300), _around(-s, 300), _around(6.0, 300), _around(-6.0, 300),
        _around(5.9, 300), _around(1.0, 300), _around(2.0, 300),
        _bits(24, 4096, 0x4018000000000000, 0x7FF0000000000000),   # beyond 6
        np.array(SPECIALS)])
    note("erf n=%d" % x.size)
    _check("erf", x, _run("erf", x), cnum.erf(x), 3)


def test_exp_sqrt_f64():
    x = np.concatenate([synth.uniform(31, 0, 1 << 17, -745.5, 709.9), _around(0.0, 100),
                        _around(709.782712893384, 300), _around(-708.3964185322641, 300),   # overflow, denormal
                        _around(-745.1332191019411, 300), _around(-746.0, 50), _around(710.0, 50),
                        np.array(SPECIALS)])
    _check("exp", x, _run("exp", x), cnum.exp(x), 2)
    y = np.concatenate([_bits(32, 1 << 17, 0, 0x7FF0000000000000), np.array(SPECIALS)])
    with np.errstate(invalid="ignore"):   # the negative specials
        ref = np.sqrt(y)
    _check("sqrt", y, _run("sqrt", y), ref, 0)
