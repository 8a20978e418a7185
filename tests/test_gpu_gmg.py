"""The GMG solver (apps.GMG: CG preconditioned by one multigrid V-cycle with
injection restriction and a weighted-Jacobi smoother) on the GPU against the
oracle.  Every step is an SpMV summed in CSR order, an elementwise op or a
dot product, so x matches the oracle to the rounding of the same operations
(the dot products differ only in summation order); fused equals unfused bit
for bit.  The oracle builds its own level operators (oracle.workloads
gmg_operators); the GPU gets the input generator's."""
import numpy as np
import pytest

import paper_2406_18109_amd as dfx
import synth
from gpu_util import note, rel_err_floor, upload
from oracle import workloads as wl

pytestmark = pytest.mark.gpu
TOL_ELEM_F64 = 1e-12
TOL_RED = 1e-10


def _solver(c, m, nlev, b):
    levels = synth.gmg_levels(m, nlev)
    lev = [(tuple(upload(c, a) for a in A), diag, None if R is None else tuple(upload(c, a) for a in R),
            None if P is None else tuple(upload(c, a) for a in P)) for A, diag, R, P in levels]
    sizes = [A[0].size - 1 for A, _, _, _ in levels]
    return dfx.apps.GMG(c, lev, sizes, upload(c, b))


def _run(m, nlev, b, iters, fuse):
    c = dfx.Context(device=0, window_size=16, fuse=fuse)
    g = _solver(c, m, nlev, b)
    rr = [float(c.store_read(g.rr, [], "f64"))]
    for _ in range(iters):
        g.iteration()
        rr.append(float(c.store_read(g.rr, [], "f64")))
    x = c.store_read(g.x, [m * m], "f64")
    c.close()
    return rr, x


def _check_oracle(m, nlev, b, iters, x, rr, n_rr=None):
    """x to the elementwise tolerance; the first n_rr residual norms (all by
    default) to the reduction tolerance."""
    xo, ho = wl.pcg_gmg(wl.gmg_operators(m, nlev), b, iters)
    assert rel_err_floor(x, xo) <= TOL_ELEM_F64
    assert len(rr) == len(ho)
    n_rr = len(rr) if n_rr is None else n_rr
    for k, (g, o) in enumerate(zip(rr[:n_rr], ho[:n_rr])):
        assert abs(g - o) <= TOL_RED * o, (k, g, o)


@pytest.mark.parametrize("m,nlev", [(127, 6), (63, 5)])
def test_gmg_fused_unfused_oracle(m, nlev):
    note("gmg m=%d levels=%d" % (m, nlev))
    b = synth.rhs(m * m, 4210 + nlev)
    rr_f, x_f = _run(m, nlev, b, 3, True)
    rr_u, x_u = _run(m, nlev, b, 3, False)
    assert rr_f == rr_u and np.array_equal(x_f, x_u)
    _check_oracle(m, nlev, b, 3, x_f, rr_f)


def test_gmg_converges():
    """Run to the tolerance on 63^2: the residual falls below 1e-8 of |b|
    within 14 iterations, as the oracle's does.  Once the residual is many
    orders below |b| its rounding noise is a large part of it, so the
    residual norms are compared over the first six iterations."""
    m, nlev = 63, 5
    note("gmg convergence m=%d" % m)
    b = synth.rhs(m * m, 4300)
    rr, x = _run(m, nlev, b, 14, True)
    assert np.sqrt(rr[-1] / rr[0]) <= 1e-8
    _check_oracle(m, nlev, b, 14, x, rr, n_rr=7)


def test_gmg_1023_full_size_graph():
    """The benchmarked size (1023^2, 9 levels), run as the bench runs it:
    one eager iteration, then one iteration recorded as a graph and
    replayed twice."""
    m, nlev = 1023, 9
    note("gmg full size %d^2" % m)
    b = synth.rhs(m * m, synth.GMG_SEED)
    c = dfx.Context(device=0, window_size=16)
    g = _solver(c, m, nlev, b)
    rr = [float(c.store_read(g.rr, [], "f64"))]
    g.iteration()
    rr.append(float(c.store_read(g.rr, [], "f64")))
    c.graph_begin()
    g.iteration()
    gid = c.graph_end()
    for _ in range(2):
        c.graph_launch(gid)
        rr.append(float(c.store_read(g.rr, [], "f64")))
    x = c.store_read(g.x, [m * m], "f64")
    c.graph_destroy(gid)
    c.close()
    note("gmg full size: oracle")
    _check_oracle(m, nlev, b, 3, x, rr)
