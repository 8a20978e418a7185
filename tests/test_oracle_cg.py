"""Pins for the oracle's conjugate gradient (sparse Krylov benchmark of section 7).

Independent checks: a manufactured integer solution, eigenvector right-hand
sides (one and two iterations), rational-exact CG on tiny grids, and SciPy's
direct solver."""
import math
from fractions import Fraction

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import cnum
from oracle import workloads as wl


def _scipy_mat(rowptr, col, val):
    n = rowptr.size - 1
    return sp.csr_matrix((val, col, rowptr), shape=(n, n))


def test_manufactured_integer_solution():
    m = 24
    rowptr, col, val = synth.poisson_csr(m, 2)
    n = m * m
    xs = (synth.raw64(77, 0, n) % np.uint64(17)).astype(np.int64) - 8
    xs = xs.astype(np.float64)
    b = cnum.spmv(rowptr, col, val, xs)  # integer arithmetic: exact
    assert np.array_equal(b, _scipy_mat(rowptr, col, val) @ xs)
    tol = 1e-12
    x, hist = wl.cg(rowptr, col, val, b, 10 * m, tol=tol)
    kappa = (1 + math.cos(math.pi / (m + 1))) / (1 - math.cos(math.pi / (m + 1)))
    assert math.sqrt(hist[-1]) <= tol * math.sqrt(hist[0])
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * tol


def test_eigenvector_rhs_one_and_two_iterations():
    m = 15
    rowptr, col, val = synth.poisson_csr(m, 2)
    i = np.arange(m)
    I, L = np.meshgrid(i, i, indexing="xy")  # x fastest: index = I + L*m
    def eig(j, k):
        v = np.sin(j * np.pi * (I + 1) / (m + 1)) * np.sin(k * np.pi * (L + 1) / (m + 1))
        lam = 4 - 2 * math.cos(j * math.pi / (m + 1)) - 2 * math.cos(k * math.pi / (m + 1))
        return v.ravel(), lam
    b, lam = eig(2, 3)
    x, hist = wl.cg(rowptr, col, val, b, 1)
    assert np.max(np.abs(x - b / lam)) < 1e-14
    assert hist[1] / hist[0] < 1e-26
    b2, lam2 = eig(5, 1)
    x, hist = wl.cg(rowptr, col, val, b + b2, 2)
    assert np.max(np.abs(x - (b / lam + b2 / lam2))) < 1e-13
    assert hist[2] / hist[0] < 1e-26


def _cg_exact(rowptr, col, val, b, iters):
    n = len(b)
    A = [[(int(col[k]), Fraction(float(val[k]))) for k in range(rowptr[i], rowptr[i + 1])] for i in range(n)]
    x = [Fraction(0)] * n
    r = [Fraction(float(v)) for v in b]
    p = list(r)
    rho = sum(v * v for v in r)
    xs = []
    for _ in range(iters):
        if rho == 0:
            break
        q = [sum(a * p[c] for c, a in A[i]) for i in range(n)]
        alpha = rho / sum(pi * qi for pi, qi in zip(p, q))
        x = [xi + alpha * pi for xi, pi in zip(x, p)]
        r = [ri - alpha * qi for ri, qi in zip(r, q)]
        rho_new = sum(v * v for v in r)
        beta = rho_new / rho
        rho = rho_new
        p = [ri + beta * pi for ri, pi in zip(r, p)]
        xs.append([float(v) for v in x])
    return xs


def test_rational_exact_cg_tiny_grids():
    for m in (3, 4):
        rowptr, col, val = synth.poisson_csr(m, 2)
        n = m * m
        b = synth.rhs(n, 900 + m)
        exact = _cg_exact(rowptr, col, val, b, n - 1)
        for k in range(1, len(exact) + 1):
            x, _ = wl.cg(rowptr, col, val, b, k)
            ex = np.array(exact[k - 1])
            assert np.max(np.abs(x - ex)) <= 1e-13 * max(1.0, np.max(np.abs(ex)))


def test_scipy_direct_solve_cg64():
    m = 64
    rowptr, col, val = synth.poisson_csr(m, 2)
    b = synth.rhs(m * m, synth.CG64_SEED)
    x, hist = wl.cg(rowptr, col, val, b, 2000, tol=1e-11)
    ref = spla.spsolve(_scipy_mat(rowptr, col, val).tocsc(), b)
    kappa = 1.0 / (1 - math.cos(math.pi / (m + 1))) * 2
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= kappa * 1e-11
    # true residual agrees with the recursive one
    res = b - cnum.spmv(rowptr, col, val, x)
    assert np.linalg.norm(res) <= 2e-11 * np.linalg.norm(b)
