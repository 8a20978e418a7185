"""Pins for the oracle's GMG solver (the evaluation's GMG application: CG
preconditioned by one multigrid V-cycle with injection restriction and a
weighted-Jacobi smoother).

Independent checks:
- the level operators against their definitions evaluated directly on 2-D
  grid functions: injection samples the coarse points exactly, bilinear
  interpolation reproduces bilinear functions wherever its stencil stays
  inside the grid, the operator is the 5-point stencil scaled by 4^-l;
- the input generator's matrices (synth, used by the GPU path) equal the
  oracle's, entry for entry;
- with M = I the solver is plain CG, bit for bit the CG oracle;
- one V-cycle on two levels against the same cycle written with dense
  matrices;
- the converged x against SciPy's direct solve, and the convergence rate;
- planted mistakes in a copy of the solver fail these pins.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import workloads as wl


def _sp(M, shape):
    rp, col, val = M
    return sp.csr_matrix((val, col, rp), shape=shape)


def _grid(seed, m):
    return synth.uniform(seed, 0, m * m, -1.0, 1.0).reshape(m, m)   # [j, i], x fastest


def test_injection_samples_coarse_points():
    for mc in (1, 3, 7):
        mf = 2 * mc + 1
        (_, R, _), _ = wl.gmg_operators(mf, 2)
        u = _grid(5100 + mc, mf)
        got = (_sp(R, (mc * mc, mf * mf)) @ u.ravel()).reshape(mc, mc)
        assert np.array_equal(got, u[1::2, 1::2])


def test_bilinear_prolongation_reproduces_bilinear_functions():
    mc = 7
    mf = 2 * mc + 1
    (_, _, P), _ = wl.gmg_operators(mf, 2)
    P = _sp(P, (mf * mf, mc * mc))
    # v = a + b X + c Y + d X Y with dyadic coefficients: exact in FP64
    a, b, c, d = 0.75, -1.5, 0.25, 0.125
    v = lambda X, Y: a + b * X + c * Y + d * X * Y
    J, I = np.mgrid[0:mc, 0:mc]
    fine = (P @ v(2.0 * I + 1, 2.0 * J + 1).ravel()).reshape(mf, mf)   # coarse (I, J) sits at fine 2I+1
    j, i = np.mgrid[0:mf, 0:mf]
    inside = (i >= 1) & (i <= mf - 2) & (j >= 1) & (j <= mf - 2)   # no coarse neighbour outside
    assert np.array_equal(fine[inside], v(i * 1.0, j * 1.0)[inside])
    # next to the boundary the missing coarse neighbour counts as zero
    assert fine[0, 0] == 0.25 * v(1.0, 1.0)


def test_operators_are_rediscretised_five_point_stencils():
    m0, nlev = 31, 4
    ops = wl.gmg_operators(m0, nlev)
    m = m0
    for l, (A, _, _) in enumerate(ops):
        u = _grid(5200 + l, m)
        pad = np.pad(u, 1)
        ref = (4 * pad[1:-1, 1:-1] - pad[:-2, 1:-1] - pad[2:, 1:-1] - pad[1:-1, :-2] - pad[1:-1, 2:]) * 0.25 ** l
        got = (_sp(A, (m * m, m * m)) @ u.ravel()).reshape(m, m)
        assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))
        m = (m - 1) // 2
    assert wl.gmg_weights(ops) == [wl.GMG_OMEGA / (4.0 * 0.25 ** l) for l in range(nlev)]


def test_generator_matrices_equal_the_oracles():
    for m0, nlev in ((7, 2), (63, 5), (127, 6)):
        for (A, R, P), (A2, diag, R2, P2) in zip(wl.gmg_operators(m0, nlev), synth.gmg_levels(m0, nlev)):
            for X, Y in ((A, A2), (R, R2), (P, P2)):
                if X is None:
                    assert Y is None
                    continue
                for a, b in zip(X, Y):
                    assert a.dtype == b.dtype and np.array_equal(a, b)
            assert diag == float(A[2][A[1] == np.repeat(np.arange(A[0].size - 1), np.diff(A[0]))][0])


def test_identity_preconditioner_is_plain_cg():
    m = 24
    rowptr, col, val = synth.poisson_csr(m, 2)
    ops = [((rowptr, col, val), None, None)]
    b = synth.rhs(m * m, 5300)
    x1, h1 = wl.pcg_gmg(ops, b, 30, precondition=False)
    x2, h2 = wl.cg(rowptr, col, val, b, 30)
    assert np.array_equal(x1, x2) and h1 == h2


def test_vcycle_two_levels_against_dense():
    mf, mc = 7, 3
    ops = wl.gmg_operators(mf, 2)
    w = wl.gmg_weights(ops)
    b = synth.rhs(mf * mf, 5301)
    got = wl.vcycle(ops, w, 0, b, nu1=2, nu2=1, nu_c=3)
    (A, R, P), (Ac, _, _) = ops
    nf, nc = mf * mf, mc * mc
    A, R, P, Ac = (_sp(M, s).toarray() for M, s in ((A, (nf, nf)), (R, (nc, nf)), (P, (nf, nc)), (Ac, (nc, nc))))
    S, Sc = np.eye(nf) - w[0] * A, np.eye(nc) - w[1] * Ac     # x <- S x + w b
    y = np.zeros(nf)
    for _ in range(2):
        y = S @ y + w[0] * b
    bc, yc = R @ (b - A @ y), np.zeros(nc)
    for _ in range(3):
        yc = Sc @ yc + w[1] * bc
    y = S @ (y + P @ yc) + w[0] * b
    assert np.max(np.abs(got - y)) <= 1e-13 * np.max(np.abs(y))


def _direct(ops, b):
    rp, col, val = ops[0][0]
    n = rp.size - 1
    return spla.spsolve(_sp((rp, col, val), (n, n)).tocsc(), b)


def _check_solver(solver):
    """Fails (AssertionError) unless `solver` converges like the V-cycle-
    preconditioned CG should (rr below 1e-16 of its start within 14
    iterations on 63^2, and x equal to the direct solve) and, with the
    identity preconditioner, is plain CG bit for bit."""
    m, nlev = 63, 5
    ops = wl.gmg_operators(m, nlev)
    b = synth.rhs(m * m, 5302)
    x, hist = solver(ops, b, 14)
    assert hist[-1] <= 1e-16 * hist[0], hist[-1] / hist[0]
    xd = _direct(ops, b)
    assert np.max(np.abs(x - xd)) <= 1e-7 * np.max(np.abs(xd))
    x1, h1 = solver(ops, b, 12, precondition=False)
    x2, h2 = wl.cg(*ops[0][0], b, 12)
    assert np.array_equal(x1, x2) and h1 == h2


def test_converges_to_direct_solve():
    _check_solver(wl.pcg_gmg)
    m, nlev = 127, 6
    ops = wl.gmg_operators(m, nlev)
    b = synth.rhs(m * m, 5303)
    x, hist = wl.pcg_gmg(ops, b, 16)
    # CG residuals are not monotone: bound the mean reduction per iteration
    rate = (hist[-1] / hist[0]) ** (1.0 / 32)
    assert rate < 0.3 and np.sqrt(hist[-1] / hist[0]) < 1e-9, rate
    xd = _direct(ops, b)
    assert np.max(np.abs(x - xd)) <= 1e-8 * np.max(np.abs(xd))
    # the unpreconditioned method is far slower on the same system
    _, hist0 = wl.pcg_gmg(ops, b, 16, precondition=False)
    assert np.sqrt(hist0[-1] / hist0[0]) > 1e-2


# ---- planted mistakes --------------------------------------------------------
def _planted(mistake):
    """A copy of the oracle's solver with one plausible mistake."""
    from oracle import cnum

    def mv(M, v):
        return cnum.spmv(M[0], M[1], M[2], v)

    def vcycle(ops, w, l, bl):
        A, R, P = ops[l]

        def sweeps(x, k):
            for _ in range(k):
                r = (mv(A, x) - bl) if mistake == "residual sign" else (bl - mv(A, x))
                x = x + w[l] * r
            return x

        x = np.zeros_like(bl)
        if R is None:
            return sweeps(x, 8)
        x = sweeps(x, 2)
        r = bl - mv(A, x)
        if mistake == "transposed restriction":    # R replaced by P^T (each row sums to 4)
            Pt = _sp(P, (bl.size, int(P[1].max()) + 1)).T.tocsr()
            bc = Pt @ r
        else:
            bc = mv(R, r)
        xc = vcycle(ops, w, l + 1, bc)
        if mistake != "dropped correction":
            x = x + mv(P, xc)
        return sweeps(x, 2)

    def solver(ops, b, iters, precondition=True):
        w = wl.gmg_weights(ops)
        A = ops[0][0]
        M = (lambda r: vcycle(ops, w, 0, r)) if precondition else (lambda r: r.copy())
        x = np.zeros_like(b)
        r = b.copy()
        z = M(r)
        p = z.copy()
        rho = cnum.fsum_prod(r, z)
        hist = [cnum.fsum_prod(r, r)]
        for _ in range(iters):
            q = mv(A, p)
            alpha = rho / cnum.fsum_prod(p, q)
            x = x + alpha * p
            r = r - alpha * q
            hist.append(cnum.fsum_prod(r, r))
            z = M(r)
            rho_new = cnum.fsum_prod(r, z)
            beta = rho_new / rho
            rho = rho_new
            p = z if mistake == "dropped beta term" else z + beta * p
        return x, hist

    return solver


def test_planted_mistakes_fail_the_pins():
    for mistake in ("residual sign", "transposed restriction", "dropped correction", "dropped beta term"):
        try:
            _check_solver(_planted(mistake))
        except AssertionError:
            continue
        raise AssertionError("planted mistake not caught: " + mistake)
    _check_solver(_planted("none"))   # the copy itself, unchanged, passes
