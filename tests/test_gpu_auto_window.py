"""Automatic window sizing on the GPU: the windows it settles on give the
same groups, hence the same bits, as a fixed window large enough for every
fusion (Black-Scholes from a window of 2, CG from 1), and the results agree
with the oracle."""
import numpy as np
import pytest

import paper_2406_18109_amd as dfx
import synth
from gpu_util import bs_run, note, rel_err_floor, upload
from oracle import workloads as wl

pytestmark = pytest.mark.gpu


def test_auto_window_black_scholes_bit_identical():
    n = 3 * 4096 + 77
    note("auto window: black-scholes n=%d" % n)
    c = dfx.Context(device=0, window_size=2, auto_window=64)
    (S, K, T, r, sig, rv), call_a, put_a = bs_run(c, n, passes=2)
    assert [g["prefix_len"] for g in c.groups()] == [28, 28] and c.window_size() == 32
    c.close()
    c = dfx.Context(device=0, window_size=64)
    _, call_f, put_f = bs_run(c, n, passes=2)
    c.close()
    assert np.array_equal(call_a, call_f) and np.array_equal(put_a, put_f)
    oc, op = wl.black_scholes(S, K, T, r, sig, rv)
    assert rel_err_floor(call_a, oc) <= 1e-12 and rel_err_floor(put_a, op) <= 1e-12


def test_auto_window_cg_bit_identical():
    m = 96
    note("auto window: cg %d^2" % m)
    rowptr, col, val = synth.poisson_csr(m, 2)
    b = synth.rhs(m * m, synth.CG64_SEED)
    out = []
    for window, auto in ((1, 64), (16, 0)):
        c = dfx.Context(device=0, window_size=window, auto_window=auto)
        cg = dfx.apps.CG(c, *[upload(c, a) for a in (rowptr, col, val, b)], m * m)
        rho = []
        for _ in range(20):
            cg.iteration()
            rho.append(float(c.store_read(cg.rho, [], "f64")))
        out.append((rho, c.store_read(cg.x, [m * m], "f64"), [g["prefix_len"] for g in c.groups()]))
        c.close()
    (ra, xa, ga), (rf, xf, gf) = out
    assert ga == gf and ra == rf and np.array_equal(xa, xf)
    xo, ho = wl.cg(rowptr, col, val, b, 20)
    assert rel_err_floor(xa, xo) <= 1e-12
    for g, o in zip(ra, ho[1:]):
        assert abs(g - o) <= 1e-10 * o


def test_window_16_black_scholes_split_bit_identical():
    """A fixed window of 16 cuts the Black-Scholes group to what one kernel
    holds (6, 6, 6, then the last 10 at the flush); every op still rounds on
    its own, so the results equal the one-pass window's bit for bit."""
    n = 3 * 4096 + 77
    note("window 16: black-scholes split n=%d" % n)
    c = dfx.Context(device=0, window_size=16)
    (S, K, T, r, sig, rv), call_s, put_s = bs_run(c, n)
    assert [g["prefix_len"] for g in c.groups()] == [6, 6, 6, 10]
    c.close()
    c = dfx.Context(device=0, window_size=64)
    _, call_f, put_f = bs_run(c, n)
    c.close()
    assert np.array_equal(call_s, call_f) and np.array_equal(put_s, put_f)
    oc, op = wl.black_scholes(S, K, T, r, sig, rv)
    assert rel_err_floor(call_s, oc) <= 1e-12 and rel_err_floor(put_s, op) <= 1e-12
