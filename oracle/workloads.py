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
  gmg            geometric multigrid V-cycles (the evaluation's GMG
                 application; its source is not given, so the textbook
                 cycle is used: weighted-Jacobi smoothing, full-weighting
                 restriction, bilinear prolongation, rediscretised coarse
                 operators, smoothing sweeps on the coarsest grid)
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


def gmg(levels, b, cycles, nu1=2, nu2=2, nu_c=30):
    """V-cycles from x0 = 0.  levels[l] = (A, w, R, P): the level's CSR
    operator, its smoothing weight (omega / diagonal), restriction to level
    l+1 and prolongation from it (None on the coarsest level).  A smoothing
    sweep is q = A x, r = b - q, x = x + w r.  One cycle on level l: nu1
    sweeps; r = b - A x; b' = R r; x' = the cycle on level l+1 from 0;
    x = x + P x'; nu2 sweeps.  The coarsest level does nu_c sweeps.
    Returns (x, history) with history[k] = |b - A x_k|^2 (k = 0..cycles)."""
    b = np.asarray(b, dtype=np.float64)

    def mv(M, v):
        return cnum.spmv(M[0], M[1], M[2], v)

    def smooth(l, bl, x, sweeps):
        A, w = levels[l][0], levels[l][1]
        for _ in range(sweeps):
            r = bl - mv(A, x)
            x = x + w * r
        return x

    def cycle(l, bl, x):
        if l == len(levels) - 1:
            return smooth(l, bl, x, nu_c)
        A, _, R, P = levels[l]
        x = smooth(l, bl, x, nu1)
        r = bl - mv(A, x)
        bc = mv(R, r)
        xc = cycle(l + 1, bc, np.zeros(R[0].size - 1))
        x = x + mv(P, xc)
        return smooth(l, bl, x, nu2)

    x = np.zeros_like(b)
    hist = [cnum.fsum_prod(b, b)]
    for _ in range(cycles):
        x = cycle(0, b, x)
        r = b - mv(levels[0][0], x)
        hist.append(cnum.fsum_prod(r, r))
    return x, hist
