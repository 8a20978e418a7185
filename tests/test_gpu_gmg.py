"""Multigrid V-cycles (apps.GMG) on the GPU against the oracle: every step
is an SpMV summed in CSR order or an elementwise op, so x matches the
oracle to rounding of the same operations; fused equals unfused bit for
bit; the residual norms within the reduction tolerance.  The operators
include the rectangular restriction and prolongation matrices."""
import numpy as np
import pytest

import paper_2406_18109_amd as dfx
import synth
from gpu_util import note, rel_err_floor, upload
from oracle import workloads as wl

pytestmark = pytest.mark.gpu


def _run(levels, b, cycles, fuse):
    c = dfx.Context(device=0, window_size=16, fuse=fuse)
    lev = [(tuple(upload(c, a) for a in A), w, None if R is None else tuple(upload(c, a) for a in R),
            None if P is None else tuple(upload(c, a) for a in P)) for A, w, R, P in levels]
    sizes = [A[0].size - 1 for A, _, _, _ in levels]
    g = dfx.apps.GMG(c, lev, sizes, upload(c, b))
    rr = []
    for _ in range(cycles):
        g.cycle()
        rr.append(float(c.store_read(g.rr, [], "f64")))
    x = c.store_read(g.x[0], [sizes[0]], "f64")
    c.close()
    return rr, x


@pytest.mark.parametrize("m,nlev", [(127, 6), (63, 3)])
def test_gmg_fused_unfused_oracle(m, nlev):
    note("gmg m=%d levels=%d" % (m, nlev))
    levels = synth.gmg_levels(m, nlev)
    b = synth.rhs(m * m, 4210 + nlev)
    rr_f, x_f = _run(levels, b, 2, True)
    rr_u, x_u = _run(levels, b, 2, False)
    assert rr_f == rr_u and np.array_equal(x_f, x_u)
    xo, ho = wl.gmg(levels, b, 2)
    assert rel_err_floor(x_f, xo) <= 1e-12
    for k, g in enumerate(rr_f):
        assert abs(g - ho[k + 1]) <= 1e-10 * ho[k + 1], k


def test_gmg_1023_full_size_graph():
    """The benchmarked size (1023^2, 9 levels), run as the bench runs it:
    one eager cycle, then one cycle recorded as a graph and replayed."""
    m, nlev = 1023, 9
    note("gmg full size %d^2" % m)
    levels = synth.gmg_levels(m, nlev)
    b = synth.rhs(m * m, synth.GMG_SEED)
    c = dfx.Context(device=0, window_size=16)
    lev = [(tuple(upload(c, a) for a in A), w, None if R is None else tuple(upload(c, a) for a in R),
            None if P is None else tuple(upload(c, a) for a in P)) for A, w, R, P in levels]
    sizes = [A[0].size - 1 for A, _, _, _ in levels]
    g = dfx.apps.GMG(c, lev, sizes, upload(c, b))
    c.sync()
    g.cycle()
    rr = [float(c.store_read(g.rr, [], "f64"))]
    c.graph_begin()
    g.cycle()
    gid = c.graph_end()
    for _ in range(2):
        c.graph_launch(gid)
        rr.append(float(c.store_read(g.rr, [], "f64")))
    x = c.store_read(g.x[0], [m * m], "f64")
    c.graph_destroy(gid)
    c.close()
    note("gmg full size: oracle")
    xo, ho = wl.gmg(levels, b, 3)
    assert rel_err_floor(x, xo) <= 1e-12
    for k, v in enumerate(rr):
        assert abs(v - ho[k + 1]) <= 1e-10 * ho[k + 1], k
