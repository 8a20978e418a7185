"""Task streams of the workloads of section 7 (and BiCGSTAB), issued through the binding.

These play the part of the application (the NumPy/SciPy-style program whose
library calls become index tasks): each function submits tasks and drops its
references to intermediates the way Python name rebinding would, so the
library's temporary analysis sees the same reference state the paper's
runtime would.  No arithmetic happens here.
"""
from __future__ import annotations

from ._binding import Context

INV_SQRT2 = 0.70710678118654752440

# Black-Scholes (section 7): one index task per NumPy operation; sig, rv and r
# are 0-d stores broadcast through the None partition.
BS_STREAM = [
    ("sqrt", ["T"], "sqrtT", ()), ("mul", ["sqrtT", "sig"], "vs", ()),
    ("div", ["S", "K"], "SK", ()), ("log", ["SK"], "lnSK", ()),
    ("mul", ["T", "rv"], "A", ()), ("add", ["lnSK", "A"], "B", ()),
    ("div", ["B", "vs"], "d1", ()), ("sub", ["d1", "vs"], "d2", ()),
    ("mul_imm", ["d1"], "e1", (INV_SQRT2,)), ("erf", ["e1"], "f1", ()),
    ("add_imm", ["f1"], "g1", (1.0,)), ("mul_imm", ["g1"], "N1", (0.5,)),
    ("mul_imm", ["d2"], "e2", (INV_SQRT2,)), ("erf", ["e2"], "f2", ()),
    ("add_imm", ["f2"], "g2", (1.0,)), ("mul_imm", ["g2"], "N2", (0.5,)),
    ("mul", ["T", "r"], "rT", ()), ("neg", ["rT"], "nrT", ()),
    ("exp", ["nrT"], "disc", ()), ("mul", ["K", "disc"], "Kd", ()),
    ("mul", ["S", "N1"], "SN1", ()), ("mul", ["Kd", "N2"], "KN2", ()),
    ("sub", ["SN1", "KN2"], "call", ()), ("rsub_imm", ["N2"], "oN2", (1.0,)),
    ("rsub_imm", ["N1"], "oN1", (1.0,)), ("mul", ["Kd", "oN2"], "KoN2", ()),
    ("mul", ["S", "oN1"], "SoN1", ()), ("sub", ["KoN2", "SoN1"], "put", ()),
]
BS_SCALARS = ("sig", "rv", "r")


def bs_drift(ctx: Context, r, sig, dtype="f64"):
    """The drift term rv = r + sigma^2/2 that the pricing stream reads, formed
    the way a NumPy program would before its pricing loop: three single tasks
    on 0-d stores (sigma*sigma, times 0.5, plus r), each rounded in the
    stores' dtype.  Returns the rv store."""
    none = ctx.part_none()
    sq, half, rv = (ctx.store_create([], dtype) for _ in range(3))
    ctx.submit("mul", [], [(sig, none, "R"), (sig, none, "R"), (sq, none, "W")])
    ctx.submit("mul_imm", [], [(sq, none, "R"), (half, none, "W")], (0.5,))
    ctx.submit("add", [], [(r, none, "R"), (half, none, "R"), (rv, none, "W")])
    ctx.store_release(sq)
    ctx.store_release(half)
    return rv


def black_scholes(ctx: Context, S, K, T, r, sig, rv, n, dtype="f64", points=1):
    """Submit one pricing pass; returns (call, put) store handles.

    S, K, T are 1-D stores of n options, r/sig/rv 0-d stores; the launch
    domain has `points` points, each pricing n/points options."""
    assert n % points == 0
    tile = ctx.part_tiling([n // points])
    none = ctx.part_none()
    names = {"S": S, "K": K, "T": T, "r": r, "sig": sig, "rv": rv}
    made = []
    for op, ins, out, imm in BS_STREAM:
        o = ctx.store_create([n], dtype)
        args = [(names[a], none if a in BS_SCALARS else tile, "R") for a in ins]
        args.append((o, tile, "W"))
        ctx.submit(op, [points], args, imm)
        names[out] = o
        made.append(out)
    # leaving the pricing function drops every local but the results
    for m in made:
        if m not in ("call", "put"):
            ctx.store_release(names[m])
    return names["call"], names["put"]


class Jacobi:
    """5-point stencil sweeps over aliasing views of one grid (section 2)."""

    def __init__(self, ctx: Context, grid: int, N: int, points=(1, 1)):
        self.ctx, self.grid, self.N = ctx, grid, N
        m = N - 2
        assert m % points[0] == 0 and m % points[1] == 0
        self.points = list(points)
        tile = [m // points[0], m // points[1]]
        self.m = m
        self.view = {k: ctx.part_tiling(tile, off) for k, off in
                     (("c", (1, 1)), ("n", (0, 1)), ("s", (2, 1)), ("w", (1, 0)), ("e", (1, 2)))}
        self.T0 = ctx.part_tiling(tile, (0, 0))
        self.none = ctx.part_none()
        self.live = {}   # names the program currently binds

    def _bind(self, name, store):
        old = self.live.get(name)
        self.live[name] = store
        if old is not None:
            self.ctx.store_release(old)

    def sweep(self):
        """avg = c + n + e + w + s; work = 0.2*avg; ss = sum((work-c)^2);
        center[:] = work; res = sqrt(ss).  Returns the res store."""
        c, G, V, T0, d = self.ctx, self.grid, self.view, self.T0, self.points
        mk = lambda: c.store_create([self.m, self.m], "f64")
        t1 = mk(); c.submit("add", d, [(G, V["c"], "R"), (G, V["n"], "R"), (t1, T0, "W")])
        t2 = mk(); c.submit("add", d, [(t1, T0, "R"), (G, V["e"], "R"), (t2, T0, "W")])
        c.store_release(t1)
        t3 = mk(); c.submit("add", d, [(t2, T0, "R"), (G, V["w"], "R"), (t3, T0, "W")])
        c.store_release(t2)
        avg = mk(); c.submit("add", d, [(t3, T0, "R"), (G, V["s"], "R"), (avg, T0, "W")])
        c.store_release(t3)
        self._bind("avg", avg)
        work = mk(); c.submit("mul_imm", d, [(avg, T0, "R"), (work, T0, "W")], (0.2,))
        self._bind("work", work)
        dd = mk(); c.submit("sub", d, [(work, T0, "R"), (G, V["c"], "R"), (dd, T0, "W")])
        self._bind("d", dd)
        ss = c.store_create([], "f64")
        c.submit("sumsq", d, [(dd, T0, "R"), (ss, self.none, "Rd")], (1,))
        self._bind("ss", ss)
        c.submit("copy", d, [(work, T0, "R"), (G, V["c"], "W")])
        res = c.store_create([], "f64")
        c.submit("sqrt", [], [(ss, self.none, "R"), (res, self.none, "W")])
        self._bind("res", res)
        return res

    def release_all(self):
        for s in self.live.values():
            self.ctx.store_release(s)
        self.live.clear()


class CG:
    """Conjugate gradient (Hestenes-Stiefel) as issued by a SciPy-style
    program: SpMV, dot products, scalar divides, axpys (section 7)."""

    def __init__(self, ctx: Context, rowptr, col, val, b, n, points=1):
        self.ctx, self.n = ctx, n
        c = ctx
        self.rowptr, self.col, self.val = rowptr, col, val
        self.none = c.part_none()
        self.tile = c.part_tiling([n // points])
        self.img = c.part_image(col, self.none)
        self.d = [points]
        vec = lambda: c.store_create([n], "f64")
        sc = lambda: c.store_create([], "f64")
        self.x, self.r, self.p, self.q = vec(), vec(), vec(), vec()
        self.pq, self.rho, self.rho_new, self.alpha, self.beta = sc(), sc(), sc(), sc(), sc()
        T, N, d = self.tile, self.none, self.d
        # x = 0; r = b; p = r; rho = r.r
        c.submit("fill", d, [(self.x, T, "W")], (0.0,))
        c.submit("copy", d, [(b, T, "R"), (self.r, T, "W")])
        c.submit("copy", d, [(self.r, T, "R"), (self.p, T, "W")])
        c.submit("dot", d, [(self.r, T, "R"), (self.r, T, "R"), (self.rho, N, "Rd")], (1,))

    def iteration(self):
        c, T, N, d = self.ctx, self.tile, self.none, self.d
        x, r, p, q = self.x, self.r, self.p, self.q
        c.submit("spmv_csr", d, [(self.rowptr, N, "R"), (self.col, N, "R"), (self.val, N, "R"),
                                 (p, self.img, "R"), (q, T, "W")])
        c.submit("dot", d, [(p, T, "R"), (q, T, "R"), (self.pq, N, "Rd")], (1,))
        c.submit("div", [], [(self.rho, N, "R"), (self.pq, N, "R"), (self.alpha, N, "W")])
        c.submit("axpy", d, [(self.alpha, N, "R"), (p, T, "R"), (x, T, "RW")], (1.0,))
        c.submit("axpy", d, [(self.alpha, N, "R"), (q, T, "R"), (r, T, "RW")], (-1.0,))
        c.submit("dot", d, [(r, T, "R"), (r, T, "R"), (self.rho_new, N, "Rd")], (1,))
        c.submit("div", [], [(self.rho_new, N, "R"), (self.rho, N, "R"), (self.beta, N, "W")])
        c.submit("copy", [], [(self.rho_new, N, "R"), (self.rho, N, "W")])
        c.submit("mul", d, [(p, T, "R"), (self.beta, N, "R"), (p, T, "W")])
        c.submit("add", d, [(p, T, "R"), (r, T, "R"), (p, T, "W")])


class BiCGSTAB:
    """BiCGSTAB (van der Vorst 1992), unpreconditioned, as a SciPy-style
    program would issue it: two SpMVs, four dot products (r^.r, r^.v, t.s,
    t.t) and the residual norm r.r per iteration, scalar divides, axpys.
    x0 = 0, shadow residual r^ = r0 = b; rho, alpha and omega start at 1 and
    p, v at 0, so the first direction is r0.  One iteration:
      rho' = r^.r; beta = (rho'/rho)(alpha/omega); rho = rho'
      p = r + beta (p - omega v); v = A p; alpha = rho / (r^.v)
      s = r - alpha v; t = A s; omega = (t.s)/(t.t)
      x = (x + alpha p) + omega s; r = s - omega t; rr = r.r
    The first rho' is formed at set-up, each later one at the end of the
    previous iteration."""

    def __init__(self, ctx: Context, rowptr, col, val, b, n, points=1):
        self.ctx, self.n = ctx, n
        c = ctx
        self.rowptr, self.col, self.val = rowptr, col, val
        self.none = c.part_none()
        self.tile = c.part_tiling([n // points])
        self.img = c.part_image(col, self.none)
        self.d = [points]
        vec = lambda: c.store_create([n], "f64")
        sc = lambda: c.store_create([], "f64")
        self.x, self.r, self.rhat, self.p, self.v, self.s, self.t = (vec() for _ in range(7))
        self.rho, self.rho_new, self.alpha, self.omega = sc(), sc(), sc(), sc()
        self.beta, self.rv, self.ts, self.tt, self.rr = sc(), sc(), sc(), sc(), sc()
        T, N, d = self.tile, self.none, self.d
        c.submit("fill", d, [(self.x, T, "W")], (0.0,))
        c.submit("copy", d, [(b, T, "R"), (self.r, T, "W")])
        c.submit("copy", d, [(b, T, "R"), (self.rhat, T, "W")])
        c.submit("fill", d, [(self.p, T, "W")], (0.0,))
        c.submit("fill", d, [(self.v, T, "W")], (0.0,))
        for sc_ in (self.rho, self.alpha, self.omega):
            c.submit("fill", [], [(sc_, N, "W")], (1.0,))
        c.submit("dot", d, [(self.r, T, "R"), (self.r, T, "R"), (self.rr, N, "Rd")], (1,))
        c.submit("dot", d, [(self.rhat, T, "R"), (self.r, T, "R"), (self.rho_new, N, "Rd")], (1,))

    def iteration(self):
        c, T, N, d = self.ctx, self.tile, self.none, self.d
        x, r, rhat, p, v, s, t = self.x, self.r, self.rhat, self.p, self.v, self.s, self.t
        sp = lambda src, dst: c.submit("spmv_csr", d, [(self.rowptr, N, "R"), (self.col, N, "R"),
                                                        (self.val, N, "R"), (src, self.img, "R"), (dst, T, "W")])
        # beta = (rho'/rho) * (alpha/omega): two temporaries the expression drops
        q1, q2 = c.store_create([], "f64"), c.store_create([], "f64")
        c.submit("div", [], [(self.rho_new, N, "R"), (self.rho, N, "R"), (q1, N, "W")])
        c.submit("div", [], [(self.alpha, N, "R"), (self.omega, N, "R"), (q2, N, "W")])
        c.submit("mul", [], [(q1, N, "R"), (q2, N, "R"), (self.beta, N, "W")])
        c.store_release(q1)
        c.store_release(q2)
        c.submit("copy", [], [(self.rho_new, N, "R"), (self.rho, N, "W")])
        c.submit("axpy", d, [(self.omega, N, "R"), (v, T, "R"), (p, T, "RW")], (-1.0,))
        c.submit("mul", d, [(p, T, "R"), (self.beta, N, "R"), (p, T, "W")])
        c.submit("add", d, [(p, T, "R"), (r, T, "R"), (p, T, "W")])
        sp(p, v)
        c.submit("dot", d, [(rhat, T, "R"), (v, T, "R"), (self.rv, N, "Rd")], (1,))
        c.submit("div", [], [(self.rho, N, "R"), (self.rv, N, "R"), (self.alpha, N, "W")])
        c.submit("copy", d, [(r, T, "R"), (s, T, "W")])
        c.submit("axpy", d, [(self.alpha, N, "R"), (v, T, "R"), (s, T, "RW")], (-1.0,))
        sp(s, t)
        c.submit("dot", d, [(t, T, "R"), (s, T, "R"), (self.ts, N, "Rd")], (1,))
        c.submit("dot", d, [(t, T, "R"), (t, T, "R"), (self.tt, N, "Rd")], (1,))
        c.submit("div", [], [(self.ts, N, "R"), (self.tt, N, "R"), (self.omega, N, "W")])
        c.submit("axpy", d, [(self.alpha, N, "R"), (p, T, "R"), (x, T, "RW")], (1.0,))
        c.submit("axpy", d, [(self.omega, N, "R"), (s, T, "R"), (x, T, "RW")], (1.0,))
        c.submit("copy", d, [(s, T, "R"), (r, T, "W")])
        c.submit("axpy", d, [(self.omega, N, "R"), (t, T, "R"), (r, T, "RW")], (-1.0,))
        c.submit("dot", d, [(r, T, "R"), (r, T, "R"), (self.rr, N, "Rd")], (1,))
        # the next iteration's rho' = r^.r, issued here so that it joins this
        # window (also when one iteration is captured as a graph)
        c.submit("dot", d, [(rhat, T, "R"), (r, T, "R"), (self.rho_new, N, "Rd")], (1,))


class GMG:
    """The evaluation's GMG application as a SciPy program issues it: CG
    preconditioned by one multigrid V-cycle, with the injection restriction
    operator and a weighted-Jacobi smoother.  Every operator application,
    restriction and prolongation is an SpMV task with its own CSR matrix;
    every vector update an elementwise task.

    `levels[l]` = (A, diag, R, P): the level's CSR operator (store handles),
    the value of its diagonal, and the transfers to and from level l+1
    (R = P = None on the coarsest level); `sizes[l]` its unknowns.  The
    smoothing weight of a level, omega / diag, is formed by single tasks at
    set-up.  A sweep is q = A x, r = b - q, x = x + w r (an axpy with the
    weight as a 0-d store); the V-cycle on level l starts from x = 0 and
    does nu1 sweeps, b' = R (b - A x), the cycle on level l+1, x = x + P x',
    nu2 sweeps; the coarsest level does nu_c sweeps.  The finest level's
    right-hand side is CG's residual r and its x is CG's z = M r.  One CG
    iteration:
      q = A p; pq = p.q; alpha = rho/pq; x += alpha p; r -= alpha q;
      rr = r.r; z = M r; rho' = r.z; beta = rho'/rho; rho = rho';
      p = beta p; p = p + z
    Per-level residual stores and the weights persist, so an iteration
    allocates nothing once one has run (it can be recorded as a graph)."""

    def __init__(self, ctx: Context, levels, sizes, b, nu1=2, nu2=2, nu_c=8, omega=2.0 / 3.0):
        c = ctx
        self.ctx, self.levels, self.sizes = c, levels, sizes
        self.nu1, self.nu2, self.nu_c = nu1, nu2, nu_c
        self.none = c.part_none()
        self.tile = [c.part_tiling([n]) for n in sizes]
        self.img = {}
        for A, _, R, P in levels:
            for M in (A, R, P):
                if M is not None:
                    self.img[M[1]] = c.part_image(M[1], self.none)
        vec = lambda n: c.store_create([n], "f64")
        sc = lambda: c.store_create([], "f64")
        n0, T, N = sizes[0], self.tile[0], self.none
        # CG state; the V-cycle's finest level solves into z from rhs r
        self.x, self.r, self.z, self.p, self.q = (vec(n0) for _ in range(5))
        self.pq, self.rho, self.rho_new, self.alpha, self.beta, self.rr = (sc() for _ in range(6))
        self.lx = [self.z] + [vec(n) for n in sizes[1:]]
        self.lb = [self.r] + [vec(n) for n in sizes[1:]]
        self.lr = [vec(n) for n in sizes]
        # w_l = omega / diag_l
        self.w = []
        om = sc()
        c.submit("fill", [], [(om, N, "W")], (omega,))
        for _, diag, _, _ in levels:
            d, h = sc(), sc()
            c.submit("fill", [], [(d, N, "W")], (diag,))
            c.submit("div", [], [(om, N, "R"), (d, N, "R"), (h, N, "W")])
            c.store_release(d)
            self.w.append(h)
        c.store_release(om)
        # x = 0; r = b; z = M r; p = z; rho = r.z; rr = r.r
        c.submit("fill", [1], [(self.x, T, "W")], (0.0,))
        c.submit("copy", [1], [(b, T, "R"), (self.r, T, "W")])
        c.submit("dot", [1], [(self.r, T, "R"), (self.r, T, "R"), (self.rr, N, "Rd")], (1,))
        self._cycle(0)
        c.submit("copy", [1], [(self.z, T, "R"), (self.p, T, "W")])
        c.submit("dot", [1], [(self.r, T, "R"), (self.z, T, "R"), (self.rho, N, "Rd")], (1,))

    def _spmv(self, M, src, dst, l_dst):
        c, N = self.ctx, self.none
        c.submit("spmv_csr", [1], [(M[0], N, "R"), (M[1], N, "R"), (M[2], N, "R"),
                                   (src, self.img[M[1]], "R"), (dst, self.tile[l_dst], "W")])

    def _residual(self, l):
        c, T = self.ctx, self.tile[l]
        q = c.store_create([self.sizes[l]], "f64")
        self._spmv(self.levels[l][0], self.lx[l], q, l)
        c.submit("sub", [1], [(self.lb[l], T, "R"), (q, T, "R"), (self.lr[l], T, "W")])
        c.store_release(q)
        return self.lr[l]

    def _smooth(self, l, sweeps):
        c, T, N = self.ctx, self.tile[l], self.none
        for _ in range(sweeps):
            r = self._residual(l)
            c.submit("axpy", [1], [(self.w[l], N, "R"), (r, T, "R"), (self.lx[l], T, "RW")], (1.0,))

    def _cycle(self, l):
        c, T = self.ctx, self.tile[l]
        c.submit("fill", [1], [(self.lx[l], T, "W")], (0.0,))
        if l == len(self.levels) - 1:
            self._smooth(l, self.nu_c)
            return
        _, _, R, P = self.levels[l]
        self._smooth(l, self.nu1)
        r = self._residual(l)
        self._spmv(R, r, self.lb[l + 1], l + 1)
        self._cycle(l + 1)
        e = c.store_create([self.sizes[l]], "f64")
        self._spmv(P, self.lx[l + 1], e, l)
        c.submit("add", [1], [(self.lx[l], T, "R"), (e, T, "R"), (self.lx[l], T, "W")])
        c.store_release(e)
        self._smooth(l, self.nu2)

    def iteration(self):
        c, T, N, d = self.ctx, self.tile[0], self.none, [1]
        x, r, z, p, q = self.x, self.r, self.z, self.p, self.q
        A = self.levels[0][0]
        c.submit("spmv_csr", d, [(A[0], N, "R"), (A[1], N, "R"), (A[2], N, "R"),
                                 (p, self.img[A[1]], "R"), (q, T, "W")])
        c.submit("dot", d, [(p, T, "R"), (q, T, "R"), (self.pq, N, "Rd")], (1,))
        c.submit("div", [], [(self.rho, N, "R"), (self.pq, N, "R"), (self.alpha, N, "W")])
        c.submit("axpy", d, [(self.alpha, N, "R"), (p, T, "R"), (x, T, "RW")], (1.0,))
        c.submit("axpy", d, [(self.alpha, N, "R"), (q, T, "R"), (r, T, "RW")], (-1.0,))
        c.submit("dot", d, [(r, T, "R"), (r, T, "R"), (self.rr, N, "Rd")], (1,))
        self._cycle(0)
        c.submit("dot", d, [(r, T, "R"), (z, T, "R"), (self.rho_new, N, "Rd")], (1,))
        c.submit("div", [], [(self.rho_new, N, "R"), (self.rho, N, "R"), (self.beta, N, "W")])
        c.submit("copy", [], [(self.rho_new, N, "R"), (self.rho, N, "W")])
        c.submit("mul", d, [(p, T, "R"), (self.beta, N, "R"), (p, T, "W")])
        c.submit("add", d, [(p, T, "R"), (z, T, "R"), (p, T, "W")])
