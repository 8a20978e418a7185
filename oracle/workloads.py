"""Plain FP64 definitions of the three workloads of section 7, unfused.

Test infrastructure only.  Each function performs the same elementwise
steps, in the same order, as the task stream the fused path executes, and
materialises every intermediate as a full array.  Transcendentals call the
host C library (oracle/cnum.c); reductions are exactly rounded.

  black_scholes  European call and put prices with an erf-based normal CDF
                 (section 7's Black-Scholes benchmark; the paper gives no
                 formula, so the standard closed form is used):
                   d1 = (ln(S/K) + (r + sigma^2/2) T) / (sigma sqrt(T))
                   d2 = d1 - sigma sqrt(T)
                   N(x) = (erf(x / sqrt(2)) + 1) / 2
                   call = S N(d1) - K e^{-rT} N(d2)
                   put  = K e^{-rT} (1 - N(d2)) - S (1 - N(d1))
  jacobi_sweep   one sweep of the 5-point stencil of section 2 (the
                 motivating example): work = 0.2 (c + n + e + w + s) over the
                 interior, the squared-difference residual sum(work - c)^2,
                 then center <- work
  cg             conjugate gradient (Hestenes-Stiefel) as issued by the
                 sparse Krylov benchmark of section 7: q = A p, alpha = rho/(p.q),
                 x += alpha p, r -= alpha q, rho' = r.r, beta = rho'/rho,
                 p = beta p + r
  bicgstab       BiCGSTAB (van der Vorst, SIAM J. Sci. Stat. Comput. 13(2),
                 1992), unpreconditioned, the further Krylov method the
                 evaluation's task-count table lists; the paper gives no
                 formula, so the published recurrence is used with x0 = 0
                 and the shadow residual r^ = r0 = b
  pcg_gmg        the evaluation's GMG application: CG preconditioned by one
                 multigrid V-cycle with injection restriction and a
                 weighted-Jacobi smoother (gmg_operators builds the level
                 operators from their one-dimensional factors; vcycle is the
                 preconditioner)
"""
from __future__ import annotations

import math

import numpy as np

from . import cnum

INV_SQRT2 = 0.70710678118654752440  # 1/sqrt(2) rounded to double


def bs_scalars(r: float, sigma: float, dtype=np.float64):
    """The broadcast scalars the stream reads: r, sigma and r + sigma^2/2.

    For a float32 stream they are rounded to float32 (each rounding of the
    float32 evaluation of r + 0.5*sigma*sigma); the oracle then computes with
    their exact values in float64."""
    if dtype == np.float32:
        f = np.float32
        r32, s32 = f(r), f(sigma)
        rv = f(r32 + f(f(0.5) * f(s32 * s32)))
        return float(r32), float(s32), float(rv)
    rv = r + 0.5 * (sigma * sigma)
    return r, sigma, rv


def black_scholes(S, K, T, r, sigma, rv, c=INV_SQRT2):
    """Call and put prices, each step one materialised FP64 array."""
    S = np.asarray(S, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    sqrtT = np.sqrt(T)
    vs = sqrtT * sigma
    SK = S / K
    lnSK = cnum.log(SK)
    A = T * rv
    B = lnSK + A
    d1 = B / vs
    d2 = d1 - vs
    e1 = d1 * c
    f1 = cnum.erf(e1)
    g1 = f1 + 1.0
    N1 = g1 * 0.5
    e2 = d2 * c
    f2 = cnum.erf(e2)
    g2 = f2 + 1.0
    N2 = g2 * 0.5
    rT = T * r
    nrT = -rT
    disc = cnum.exp(nrT)
    Kd = K * disc
    SN1 = S * N1
    KN2 = Kd * N2
    call = SN1 - KN2
    oN2 = 1.0 - N2
    oN1 = 1.0 - N1
    KoN2 = Kd * oN2
    SoN1 = S * oN1
    put = KoN2 - SoN1
    return call, put


def jacobi_sweep(grid):
    """One sweep on a full (N, N) grid in place; returns sum((work-c)^2) exactly rounded."""
    c = grid[1:-1, 1:-1]
    n = grid[0:-2, 1:-1]
    s = grid[2:, 1:-1]
    w = grid[1:-1, 0:-2]
    e = grid[1:-1, 2:]
    t1 = c + n
    t2 = t1 + e
    t3 = t2 + w
    avg = t3 + s
    work = avg * 0.2
    d = work - c
    ss = cnum.fsum_prod(d, d)
    grid[1:-1, 1:-1] = work
    return ss


def jacobi(grid, sweeps):
    """`sweeps` sweeps in place; returns the list of residual norms sqrt(ss)."""
    res = []
    for _ in range(sweeps):
        res.append(math.sqrt(jacobi_sweep(grid)))
    return res


def jacobi_naive(grid, sweeps):
    """The same sweeps written as plain double loops with no views.

    Pure Python: tiny grids only."""
    g = [list(map(float, row)) for row in np.asarray(grid)]
    N = len(g)
    res = []
    for _ in range(sweeps):
        work = [[0.0] * N for _ in range(N)]
        sq = []
        for i in range(1, N - 1):
            for j in range(1, N - 1):
                t = g[i][j] + g[i - 1][j]
                t = t + g[i][j + 1]
                t = t + g[i][j - 1]
                t = t + g[i + 1][j]
                wv = t * 0.2
                work[i][j] = wv
                d = wv - g[i][j]
                sq.append(d * d)
        for i in range(1, N - 1):
            for j in range(1, N - 1):
                g[i][j] = work[i][j]
        res.append(math.sqrt(math.fsum(sq)))
    return np.array(g), res


def cg(rowptr, col, val, b, iters, tol=None):
    """Conjugate gradient from x0 = 0.

    Returns (x, rho_history) where rho_history[k] = r_k . r_k (k = 0..done).
    With `tol`, stops once sqrt(rho_k) <= tol * ||b||."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rho = cnum.fsum_prod(r, r)
    hist = [rho]
    bnorm = math.sqrt(rho)
    for _ in range(iters):
        if tol is not None and math.sqrt(rho) <= tol * bnorm:
            break
        q = cnum.spmv(rowptr, col, val, p)
        pq = cnum.fsum_prod(p, q)
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        rho_new = cnum.fsum_prod(r, r)
        beta = rho_new / rho
        rho = rho_new
        p = beta * p
        p = p + r
        hist.append(rho)
    return x, hist


def bicgstab(rowptr, col, val, b, iters):
    """BiCGSTAB from x0 = 0, shadow residual r^ = r0 = b, started from
    rho = alpha = omega = 1 and p = v = 0 (so the first p is r0).  One
    iteration, in this order:
      rho' = r^.r;  beta = (rho'/rho) (alpha/omega);  rho = rho'
      p = r + beta (p - omega v);  v = A p;  alpha = rho / (r^.v)
      s = r - alpha v;  t = A s;  omega = (t.s) / (t.t)
      x = (x + alpha p) + omega s;  r = s - omega t
    Returns (x, history) where history[k] = r_k . r_k (k = 0..iters)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    rhat = b.copy()
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    rho = alpha = omega = 1.0
    hist = [cnum.fsum_prod(r, r)]
    for _ in range(iters):
        rho_new = cnum.fsum_prod(rhat, r)
        beta = (rho_new / rho) * (alpha / omega)
        rho = rho_new
        p = r + beta * (p - omega * v)
        v = cnum.spmv(rowptr, col, val, p)
        alpha = rho / cnum.fsum_prod(rhat, v)
        s = r - alpha * v
        t = cnum.spmv(rowptr, col, val, s)
        omega = cnum.fsum_prod(t, s) / cnum.fsum_prod(t, t)
        x = (x + alpha * p) + omega * s
        r = s - omega * t
        hist.append(cnum.fsum_prod(r, r))
    return x, hist


# ---------------------------------------------------------------------------
# Geometric multigrid as the evaluation describes its GMG application: a
# CG-based solver whose preconditioner is one V-cycle, with the injection
# restriction operator and a weighted-Jacobi smoother.  What the paper leaves
# open is read as follows: bilinear prolongation, the 5-point operator
# rediscretised on each coarser grid, V(2,2) with weight 2/3, 8 smoothing
# sweeps on the coarsest grid, and the V-cycle started from zero.
# ---------------------------------------------------------------------------
GMG_OMEGA = 2.0 / 3.0


def _csr(M):
    """(rowptr int32, col int32, val float64) of a SciPy sparse matrix with
    the columns of every row ascending and no stored zeros."""
    import scipy.sparse as sp
    M = sp.csr_matrix(M)
    M.eliminate_zeros()
    M.sort_indices()
    return M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64)


def gmg_operators(m0, nlev):
    """The hierarchy of the m0 x m0 Dirichlet Poisson problem, m0 = 2^k - 1.

    Level l has side m_l = (m_{l-1} - 1) / 2.  Each operator is built from
    its one-dimensional factors (Kronecker products), unknowns numbered with
    x fastest:
      A_l = 4^-l (I (x) T + T (x) I), T = tridiag(-1, 2, -1) of size m_l: the
            5-point operator of the finest grid's h^2 units rediscretised on
            a grid of spacing 2^l h;
      R_l = Ri (x) Ri, Ri[J, 2J+1] = 1: injection, coarse point (I, J) takes
            the fine value at (2I+1, 2J+1);
      P_l = Pi (x) Pi, Pi[2J, J] = Pi[2J+2, J] = 1/2, Pi[2J+1, J] = 1: bilinear
            interpolation with zero Dirichlet values outside the grid.
    Returns [(A, R, P)] as CSR triples (R = P = None on the coarsest level)."""
    import scipy.sparse as sp
    out, m = [], m0
    for l in range(nlev):
        T = sp.diags([-np.ones(m - 1), 2.0 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
        I = sp.identity(m)
        A = (sp.kron(I, T) + sp.kron(T, I)) * (0.25 ** l)
        if l == nlev - 1:
            out.append((_csr(A), None, None))
            break
        if m % 2 == 0 or m < 3:
            raise ValueError("side must be 2^k - 1 on every level but the last")
        mc = (m - 1) // 2
        Ri = sp.lil_matrix((mc, m))
        Pi = sp.lil_matrix((m, mc))
        for J in range(mc):
            Ri[J, 2 * J + 1] = 1.0
            Pi[2 * J, J] = 0.5
            Pi[2 * J + 1, J] = 1.0
            Pi[2 * J + 2, J] = 0.5
        out.append((_csr(A), _csr(sp.kron(Ri, Ri)), _csr(sp.kron(Pi, Pi))))
        m = mc
    return out


def gmg_weights(ops, omega=GMG_OMEGA):
    """The smoothing weight of each level: omega over the operator's diagonal
    (constant on a level), one rounded division."""
    out = []
    for (rp, col, val), _, _ in ops:
        d = val[col == np.repeat(np.arange(rp.size - 1), np.diff(rp))]
        assert np.all(d == d[0])
        out.append(omega / float(d[0]))
    return out


def vcycle(ops, w, l, bl, nu1=2, nu2=2, nu_c=8):
    """One V-cycle for A_l e = bl from e = 0.  A smoothing sweep is
    q = A x, r = bl - q, x = x + w_l r.  Level l: nu1 sweeps; r = bl - A x;
    b' = R r; x' = the cycle on level l+1; x = x + P x'; nu2 sweeps.  The
    coarsest level does nu_c sweeps."""
    A, R, P = ops[l]

    def sweeps(x, k):
        for _ in range(k):
            q = cnum.spmv(A[0], A[1], A[2], x)
            r = bl - q
            x = x + w[l] * r
        return x

    x = np.zeros_like(bl)
    if R is None:
        return sweeps(x, nu_c)
    x = sweeps(x, nu1)
    q = cnum.spmv(A[0], A[1], A[2], x)
    r = bl - q
    bc = cnum.spmv(R[0], R[1], R[2], r)
    xc = vcycle(ops, w, l + 1, bc, nu1, nu2, nu_c)
    e = cnum.spmv(P[0], P[1], P[2], xc)
    x = x + e
    return sweeps(x, nu2)


def pcg_gmg(ops, b, iters, nu1=2, nu2=2, nu_c=8, omega=GMG_OMEGA, precondition=True):
    """Preconditioned CG from x0 = 0 with M = one V-cycle on the finest level
    (precondition=False: M = I, which is plain CG).  One iteration, in this
    order:
      q = A p; pq = p.q; alpha = rho/pq; x = x + alpha p; r = r - alpha q;
      rr = r.r; z = M r; rho' = r.z; beta = rho'/rho; rho = rho';
      p = beta p; p = p + z
    with z0 = M b, p0 = z0, rho0 = r0.z0.  Returns (x, history) where
    history[k] = r_k . r_k (k = 0..iters)."""
    A = ops[0][0]
    w = gmg_weights(ops, omega)
    b = np.asarray(b, dtype=np.float64)
    M = (lambda r: vcycle(ops, w, 0, r, nu1, nu2, nu_c)) if precondition else (lambda r: r.copy())
    x = np.zeros_like(b)
    r = b.copy()
    z = M(r)
    p = z.copy()
    rho = cnum.fsum_prod(r, z)
    hist = [cnum.fsum_prod(r, r)]
    for _ in range(iters):
        q = cnum.spmv(A[0], A[1], A[2], p)
        pq = cnum.fsum_prod(p, q)
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        hist.append(cnum.fsum_prod(r, r))
        z = M(r)
        rho_new = cnum.fsum_prod(r, z)
        beta = rho_new / rho
        rho = rho_new
        p = beta * p
        p = p + z
    return x, hist
