"""Pins for the oracle's Black-Scholes evaluation (section 7 benchmark).

Independent checks: put-call parity, 40-digit mpmath evaluation of the closed
form, no-arbitrage bounds, monotonicity, and the stream evaluator reproducing
the direct evaluation when fed the same stream written as tasks."""
import math

import mpmath
import numpy as np
import pytest

import synth
from oracle import workloads as wl
from oracle import stream
from oracle.ir import NoneP, Task, Tiling


def _prices(n, dtype=np.float64):
    S, K, T = synth.bs_inputs(n, dtype)
    r, sig, rv = wl.bs_scalars(synth.BS_RATE, synth.BS_VOL, dtype)
    S, K, T = (a.astype(np.float64) for a in (S, K, T))
    call, put = wl.black_scholes(S, K, T, r, sig, rv)
    return S, K, T, r, sig, rv, call, put


def test_put_call_parity():
    S, K, T, r, sig, rv, call, put = _prices(200000)
    Kd = K * np.exp(-r * T)
    err = np.abs(call - put - (S - Kd))
    assert np.all(err <= 8 * np.finfo(np.float64).eps * (S + K))


def test_mpmath_40_digits():
    S, K, T, r, sig, rv, call, put = _prices(400)
    mpmath.mp.dps = 40
    worst = 0.0
    for i in range(400):
        s, k, t = mpmath.mpf(S[i]), mpmath.mpf(K[i]), mpmath.mpf(T[i])
        R, V = mpmath.mpf(r), mpmath.mpf(sig)
        d1 = (mpmath.log(s / k) + (R + V * V / 2) * t) / (V * mpmath.sqrt(t))
        d2 = d1 - V * mpmath.sqrt(t)
        N = lambda x: (mpmath.erf(x / mpmath.sqrt(2)) + 1) / 2
        kd = k * mpmath.exp(-R * t)
        c = s * N(d1) - kd * N(d2)
        p = kd * (1 - N(d2)) - s * (1 - N(d1))
        for got, ex in ((call[i], c), (put[i], p)):
            e = abs(mpmath.mpf(got) - ex) / max(abs(ex), 1)
            worst = max(worst, float(e))
    # a few ulps of prices up to 100 through ~30 roundings; far inside 1e-12
    assert worst < 1e-13, worst


def test_no_arbitrage_bounds_and_monotone():
    S, K, T, r, sig, rv, call, put = _prices(100000)
    Kd = K * np.exp(-r * T)
    tol = 1e-12 * np.maximum(np.abs(call), 1)
    assert np.all(call >= np.maximum(S - Kd, 0) - tol)
    assert np.all(call <= S + tol)
    assert np.all(put >= np.maximum(Kd - S, 0) - tol)
    # monotone: call increasing in S, decreasing in K
    base = np.full(50, 50.0)
    Ss = np.linspace(10, 100, 50)
    T1 = np.full(50, 1.0)
    c1, _ = wl.black_scholes(Ss, base, T1, r, sig, rv)
    assert np.all(np.diff(c1) > 0)
    c2, p2 = wl.black_scholes(base, Ss, T1, r, sig, rv)
    assert np.all(np.diff(c2) < 0) and np.all(np.diff(p2) > 0)


def test_float32_inputs_are_exact_float32_values():
    S32, K32, T32 = synth.bs_inputs(1000, np.float32)
    S64, K64, T64 = synth.bs_inputs(1000, np.float64)
    assert np.array_equal(S32, S64.astype(np.float32))
    r, sig, rv = wl.bs_scalars(0.02, 0.3, np.float32)
    assert r == float(np.float32(0.02)) and sig == float(np.float32(0.3))


def bs_tasks(n):
    """The Black-Scholes stream as IR tasks over one launch point."""
    T1 = Tiling((n,), (0,))
    N0 = NoneP()
    d = (1,)
    prog = [
        ("sqrt", ["T"], "sqrtT", ()), ("mul", ["sqrtT", "sig"], "vs", ()),
        ("div", ["S", "K"], "SK", ()), ("log", ["SK"], "lnSK", ()),
        ("mul", ["T", "rv"], "A", ()), ("add", ["lnSK", "A"], "B", ()),
        ("div", ["B", "vs"], "d1", ()), ("sub", ["d1", "vs"], "d2", ()),
        ("mul_imm", ["d1"], "e1", (wl.INV_SQRT2,)), ("erf", ["e1"], "f1", ()),
        ("add_imm", ["f1"], "g1", (1.0,)), ("mul_imm", ["g1"], "N1", (0.5,)),
        ("mul_imm", ["d2"], "e2", (wl.INV_SQRT2,)), ("erf", ["e2"], "f2", ()),
        ("add_imm", ["f2"], "g2", (1.0,)), ("mul_imm", ["g2"], "N2", (0.5,)),
        ("mul", ["T", "r"], "rT", ()), ("neg", ["rT"], "nrT", ()),
        ("exp", ["nrT"], "disc", ()), ("mul", ["K", "disc"], "Kd", ()),
        ("mul", ["S", "N1"], "SN1", ()), ("mul", ["Kd", "N2"], "KN2", ()),
        ("sub", ["SN1", "KN2"], "call", ()), ("rsub_imm", ["N2"], "oN2", (1.0,)),
        ("rsub_imm", ["N1"], "oN1", (1.0,)), ("mul", ["Kd", "oN2"], "KoN2", ()),
        ("mul", ["S", "oN1"], "SoN1", ()), ("sub", ["KoN2", "SoN1"], "put", ()),
    ]
    scal = {"sig", "rv", "r"}
    tasks = []
    for op, ins, out, imm in prog:
        args = [(a, N0 if a in scal else T1, "R") for a in ins] + [(out, T1, "W")]
        tasks.append(Task(op, d, args, imm))
    return tasks, [p[2] for p in prog]


def test_stream_evaluator_matches_direct_evaluation_bitwise():
    n = 5000
    S, K, T, r, sig, rv, call, put = _prices(n)
    tasks, outs = bs_tasks(n)
    st = {"S": S.copy(), "K": K.copy(), "T": T.copy(),
          "r": np.array(r), "sig": np.array(sig), "rv": np.array(rv)}
    for o in outs:
        st[o] = np.zeros(n)
    stream.evaluate(tasks, st)
    assert np.array_equal(st["call"], call)
    assert np.array_equal(st["put"], put)
