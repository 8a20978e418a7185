"""Pins for the oracle's Jacobi stencil (the motivating example of section 2).

Independent checks: bitwise equality with plain double loops (no views),
exact discrete harmonic fixed points, SciPy's direct solve for the
one-hot-edge boundary problem, and the discrete maximum principle."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import stream
from oracle import workloads as wl
from oracle.ir import NoneP, Task, Tiling


def test_matches_naive_loops_bitwise():
    rng = np.random.default_rng(3)
    for N in (3, 5, 9, 16):
        g = rng.random((N, N))
        g_naive, res_naive = wl.jacobi_naive(g.copy(), 3)
        g2 = g.copy()
        res = wl.jacobi(g2, 3)
        assert np.array_equal(g2, g_naive)
        assert res == res_naive


def test_harmonic_fixed_point():
    # u = a + b i + c j + d (i^2 - j^2) + e i j is exactly 5-point harmonic,
    # hence a fixed point of the 0.2-weighted update as well.
    for N, coef in ((8, (3, 1, -2, 1, 2)), (12, (-5, 2, 1, -1, 1))):
        a, b, c, d, e = coef
        i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
        u = (a + b * i + c * j + d * (i * i - j * j) + e * i * j).astype(np.float64)
        g = u.copy()
        g[1:-1, 1:-1] = 0.0
        for _ in range(20000):
            r = wl.jacobi_sweep(g)
            if r < 1e-26:
                break
        assert np.max(np.abs(g - u)) < 1e-10 * max(1.0, np.abs(u).max())
        # an exact fixed point stays exactly fixed
        g3 = u.copy()
        assert wl.jacobi_sweep(g3) == 0.0 or np.max(np.abs(g3 - u)) < 1e-12 * np.abs(u).max()


def _direct_edge_solution(N):
    m = N - 2
    n = m * m
    main = 4.0 * np.ones(n)
    A = sp.diags([main], [0], format="lil")
    for i in range(m):
        for j in range(m):
            k = i * m + j
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < m and 0 <= jj < m:
                    A[k, ii * m + jj] = -1.0
    b = np.zeros(n)
    b[:m] = 1.0  # first interior row touches boundary row 0 (value 1)
    return spla.spsolve(A.tocsc(), b).reshape(m, m)


def test_converges_to_direct_solve_and_max_principle():
    N = 10
    g = synth.jacobi_grid(N)
    for k in range(6000):
        r = wl.jacobi_sweep(g)
        if k % 500 == 0:
            assert g.min() >= 0.0 and g.max() <= 1.0
        if r < 1e-28:
            break
    ref = _direct_edge_solution(N)
    assert np.max(np.abs(g[1:-1, 1:-1] - ref)) < 1e-10


def stencil_tasks(N, domain=(1, 1), with_residual=True):
    """One sweep as IR tasks: 5 offset views of `grid`, temporaries, COPY."""
    m = N - 2
    tile = tuple(m // d for d in domain)
    view = {"c": (1, 1), "n": (0, 1), "s": (2, 1), "w": (1, 0), "e": (1, 2)}
    P = {k: Tiling(tile, off) for k, off in view.items()}
    T0 = Tiling(tile, (0, 0))
    G = "grid"
    t = [
        Task("add", domain, [(G, P["c"], "R"), (G, P["n"], "R"), ("t1", T0, "W")]),
        Task("add", domain, [("t1", T0, "R"), (G, P["e"], "R"), ("t2", T0, "W")]),
        Task("add", domain, [("t2", T0, "R"), (G, P["w"], "R"), ("t3", T0, "W")]),
        Task("add", domain, [("t3", T0, "R"), (G, P["s"], "R"), ("avg", T0, "W")]),
        Task("mul_imm", domain, [("avg", T0, "R"), ("work", T0, "W")], (0.2,)),
    ]
    if with_residual:
        t += [
            Task("sub", domain, [("work", T0, "R"), (G, P["c"], "R"), ("d", T0, "W")]),
            Task("sumsq", domain, [("d", T0, "R"), ("ss", NoneP(), "Rd")], (1,)),
        ]
    t.append(Task("copy", domain, [("work", T0, "R"), (G, P["c"], "W")]))
    return t


def test_stream_evaluator_reproduces_naive_loops():
    rng = np.random.default_rng(5)
    for N, dom in ((6, (1, 1)), (6, (2, 2)), (10, (2, 4))):
        g = rng.random((N, N))
        g_naive, res_naive = wl.jacobi_naive(g.copy(), 1)
        m = N - 2
        st = {"grid": g.copy(), "ss": np.array(0.0)}
        for s in ("t1", "t2", "t3", "avg", "work", "d"):
            st[s] = np.zeros((m, m))
        stream.evaluate(stencil_tasks(N, dom), st)
        assert np.array_equal(st["grid"], g_naive)
        assert np.sqrt(st["ss"]) == res_naive[0]
