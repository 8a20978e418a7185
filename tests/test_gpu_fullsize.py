"""Parity at the full sizes of the measured workloads, run as bench.py runs
them (one fused pass per Black-Scholes step, window 16 for the iterative
solvers, one CG iteration captured as a graph and replayed):

- Black-Scholes over 2^26 options, FP64 and FP32: a seeded sample of 64K
  options against the oracle element by element, and put-call parity on
  every option;
- Jacobi on an 8192 x 8192 grid (seeded random values, so every point
  carries information): the whole grid bit for bit after two sweeps, and
  both residuals;
- CG on the 256^3 7-point Poisson matrix: every element of x after three
  iterations (one eager, two graph replays) and the residual history.
"""
import numpy as np
import pytest

import paper_2406_18109_amd as dfx
import synth
from gpu_util import bs_run, ctx, note, rel_err_floor, upload
from oracle import workloads as wl

pytestmark = pytest.mark.gpu
TOL_ELEM_F64 = 1e-12   # |g-o| <= 1e-12 max(|o|, 1)
TOL_ELEM_F32 = 1e-4    # float32 stream against the float64 oracle
TOL_RED = 1e-10        # reductions and CG residuals, relative


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_black_scholes_full_size(dtype):
    n = 1 << 26
    note("bs full size %s n=%d" % (dtype, n))
    c = ctx()
    (S, K, T, r, sig, rv), call, put = bs_run(c, n, dtype)
    assert [g["prefix_len"] for g in c.groups()][-1] == 28   # the whole stream in one pass
    c.close()
    note("bs full size: oracle on the sample")
    idx = np.unique(np.concatenate([[0, n - 1], (synth.raw64(77, 0, 1 << 16) % np.uint64(n)).astype(np.int64)]))
    oc, op = wl.black_scholes(S[idx].astype(np.float64), K[idx].astype(np.float64), T[idx].astype(np.float64),
                              r, sig, rv)
    tol = TOL_ELEM_F64 if dtype == "f64" else TOL_ELEM_F32
    assert rel_err_floor(call[idx], oc) <= tol
    assert rel_err_floor(put[idx], op) <= tol
    # C - P = S - K exp(-rT) on every option, to the rounding of the terms (each at most S or K)
    note("bs full size: put-call parity")
    S64, K64 = S.astype(np.float64), K.astype(np.float64)
    gap = np.abs((call.astype(np.float64) - put.astype(np.float64)) - (S64 - K64 * np.exp(-r * T.astype(np.float64))))
    rel = 1e-13 if dtype == "f64" else 2e-6
    assert np.all(gap <= rel * (S64 + K64)), float(np.max(gap / (S64 + K64)))


def test_jacobi_full_size():
    N, sweeps = 8192, 2
    note("jacobi full size N=%d" % N)
    g0 = synth.uniform(91, 0, N * N, 0.0, 1.0).reshape(N, N)
    c = ctx(window=16)
    G = upload(c, g0)
    J = dfx.apps.Jacobi(c, G, N)
    res = [float(c.store_read(J.sweep(), [], "f64")) for _ in range(sweeps)]
    grid = c.store_read(G, [N, N], "f64")
    c.close()
    note("jacobi full size: oracle")
    ref = g0.copy()
    del g0
    ores = wl.jacobi(ref, sweeps)
    assert np.array_equal(grid, ref)
    for g, o in zip(res, ores):
        assert abs(g - o) <= TOL_RED * abs(o)


def test_cg256_full_size_graph():
    m, dim, n = 256, 3, 256 ** 3
    note("cg 256^3 full size")
    rowptr, col, val = synth.poisson_csr(m, dim)
    b = synth.rhs(n, synth.CG256_SEED)
    c = ctx(window=16)
    hs = [upload(c, a) for a in (rowptr, col, val, b)]
    cg = dfx.apps.CG(c, *hs, n)
    rho = [float(c.store_read(cg.rho, [], "f64"))]
    cg.iteration()
    rho.append(float(c.store_read(cg.rho, [], "f64")))
    c.graph_begin()
    cg.iteration()
    g = c.graph_end()
    for _ in range(2):
        c.graph_launch(g)
        rho.append(float(c.store_read(cg.rho, [], "f64")))
    x = c.store_read(cg.x, [n], "f64")
    c.close()
    note("cg 256^3 full size: oracle")
    xo, ho = wl.cg(rowptr, col, val, b, 3)
    assert len(rho) == len(ho) == 4
    for k, (gv, o) in enumerate(zip(rho, ho)):
        assert abs(gv - o) <= TOL_RED * abs(o), k
    assert rel_err_floor(x, xo) <= TOL_ELEM_F64


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    with open(path) as fh:
        return [float(line) for line in fh if not line.startswith("#")]


def test_cg256_rho_history_500_iterations():
    """The residual history rho_k = r_k.r_k of 500 CG iterations on the
    256^3 system, as the bench runs them (one eager iteration, then one
    iteration recorded as a graph and replayed), against the oracle's
    history stored in tests/golden/cg256_rho.txt (written by
    tests/golden/make_cg256_rho.py, which calls only the oracle)."""
    m, dim, n, iters = 256, 3, 256 ** 3, 500
    ho = _golden("cg256_rho.txt")
    assert len(ho) == iters + 1
    note("cg 256^3: %d iterations against the stored oracle history" % iters)
    rowptr, col, val = synth.poisson_csr(m, dim)
    b = synth.rhs(n, synth.CG256_SEED)
    c = ctx(window=16)
    hs = [upload(c, a) for a in (rowptr, col, val, b)]
    del rowptr, col, val
    cg = dfx.apps.CG(c, *hs, n)
    rho = [float(c.store_read(cg.rho, [], "f64"))]
    cg.iteration()
    rho.append(float(c.store_read(cg.rho, [], "f64")))
    c.graph_begin()
    cg.iteration()
    g = c.graph_end()
    for k in range(iters - 1):
        c.graph_launch(g)
        rho.append(float(c.store_read(cg.rho, [], "f64")))
        if k % 100 == 99:
            note("cg 256^3: %d iterations" % (k + 2))
    c.close()
    worst = max(abs(gv - o) / o for gv, o in zip(rho, ho))
    note("cg 256^3: worst relative difference of rho over %d iterations %.2e" % (iters, worst))
    for k, (gv, o) in enumerate(zip(rho, ho)):
        assert abs(gv - o) <= TOL_RED * abs(o), (k, gv, o)
