"""Pins for the oracle's multigrid V-cycle (the evaluation's GMG
application, textbook cycle): the convergence rate of V(2,2) weighted-Jacobi
multigrid on the 2-D Poisson problem and the converged solution against
SciPy's direct solve; and one two-grid cycle against the same cycle written
with dense matrices and an exact coarse solve (the oracle's coarse level
runs enough sweeps to reach it)."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import workloads as wl


def _dense(M, shape):
    rp, col, val = M
    return sp.csr_matrix((val, col, rp), shape=shape).toarray()


def test_vcycle_rate_and_direct_solve():
    m = 63
    levels = synth.gmg_levels(m, 5)
    b = synth.rhs(m * m, 4200)
    x, hist = wl.gmg(levels, b, 10)
    rates = [np.sqrt(hist[k + 1] / hist[k]) for k in range(10)]
    assert max(rates) < 0.2, rates
    A = sp.csr_matrix((levels[0][0][2], levels[0][0][1], levels[0][0][0]), shape=(m * m, m * m))
    xd = spla.spsolve(A.tocsc(), b)
    assert np.max(np.abs(x - xd)) <= 1e-7 * np.max(np.abs(xd))


def test_two_grid_cycle_against_dense_exact_coarse_solve():
    mf, mc = 7, 3
    levels = synth.gmg_levels(mf, 2)
    b = synth.rhs(mf * mf, 4201)
    x, _ = wl.gmg(levels, b, 1, nu1=2, nu2=1, nu_c=400)
    (A, w, R, P), (Ac, _, _, _) = levels
    nf, nc = mf * mf, mc * mc
    A, R, P, Ac = _dense(A, (nf, nf)), _dense(R, (nc, nf)), _dense(P, (nf, nc)), _dense(Ac, (nc, nc))
    S = np.eye(nf) - w * A                      # x <- S x + w b
    y = np.zeros(nf)
    for _ in range(2):
        y = S @ y + w * b
    y = y + P @ np.linalg.solve(Ac, R @ (b - A @ y))
    y = S @ y + w * b
    assert np.max(np.abs(x - y)) <= 1e-12 * np.max(np.abs(y))
