"""Plans loaded from the on-disk cache execute with no analysis and give the
same bits as the plans the saving context built (Black-Scholes, CG,
BiCGSTAB), and those results agree with the oracle."""
import numpy as np
import pytest

import paper_2406_18109_amd as dfx
import synth
from gpu_util import bs_run, note, rel_err_floor, upload
from oracle import workloads as wl

pytestmark = pytest.mark.gpu


M_CD = 48


def _systems():
    rowptr, col, val = synth.convdiff_csr(M_CD, 2)
    return (rowptr, col, val), synth.rhs(M_CD * M_CD, 4130)


def _run(c):
    _, call, put = bs_run(c, 3 * 4096 + 77, passes=2)
    m = M_CD
    (rowptr, col, val), b = _systems()
    hs = [upload(c, a) for a in (rowptr, col, val, b)]
    res = [call, put]
    for cls in (dfx.apps.CG, dfx.apps.BiCGSTAB):
        s = cls(c, *hs, m * m)
        for _ in range(5):
            s.iteration()
        res.append(c.store_read(s.x, [m * m], "f64"))
    return res


def _check_oracle(res):
    call, put, x_cg, x_bi = res
    n = 3 * 4096 + 77
    S, K, T = synth.bs_inputs(n)
    oc, op = wl.black_scholes(S, K, T, *wl.bs_scalars(synth.BS_RATE, synth.BS_VOL))
    assert rel_err_floor(call, oc) <= 1e-12 and rel_err_floor(put, op) <= 1e-12
    (rowptr, col, val), b = _systems()
    # CG on the nonsymmetric matrix is still a well-defined stream of tasks
    assert rel_err_floor(x_cg, wl.cg(rowptr, col, val, b, 5)[0]) <= 1e-12
    assert rel_err_floor(x_bi, wl.bicgstab(rowptr, col, val, b, 5)[0]) <= 1e-12


def test_loaded_plans_bit_identical(tmp_path):
    path = str(tmp_path / "plans.bin")
    note("plan cache: save")
    a = dfx.Context(device=0, window_size=64)
    ra = _run(a)
    n = a.plan_cache_save(path)
    a.close()
    note("plan cache: load %d plans" % n)
    b = dfx.Context(device=0, window_size=64)
    assert b.plan_cache_load(path) == n
    rb = _run(b)
    st = b.stats()
    b.close()
    assert st["memo_misses"] == 0
    for x, y in zip(ra, rb):
        assert np.array_equal(x, y)
    _check_oracle(rb)


def test_capture_from_loaded_plans_without_eager_run(tmp_path):
    """A context that loads the cache records a CG iteration as a graph
    with no eager iteration first: plans and their workspaces come from the
    load, and the iteration's work stores get their memory from host writes
    (stores are allocated at their first write; a recording cannot
    allocate).  Three replays equal three eager iterations of the saving
    context bit for bit."""
    path = str(tmp_path / "plans.bin")
    m = 40
    rowptr, col, val = synth.poisson_csr(m, 2)
    b = synth.rhs(m * m, 4140)
    note("plan cache: eager cg %d^2, save" % m)
    a = dfx.Context(device=0, window_size=16)
    cg = dfx.apps.CG(a, *[upload(a, v) for v in (rowptr, col, val, b)], m * m)
    rho_a = [float(a.store_read(cg.rho, [], "f64"))]
    for _ in range(3):
        cg.iteration()
        rho_a.append(float(a.store_read(cg.rho, [], "f64")))
    x_a = a.store_read(cg.x, [m * m], "f64")
    a.plan_cache_save(path)
    a.close()
    note("plan cache: load, capture with no eager iteration")
    c = dfx.Context(device=0, window_size=16)
    c.plan_cache_load(path)
    cg = dfx.apps.CG(c, *[upload(c, v) for v in (rowptr, col, val, b)], m * m)
    rho_c = [float(c.store_read(cg.rho, [], "f64"))]
    # overwritten or started afresh by the iteration, so the values do not matter
    c.store_write(cg.q, np.zeros(m * m))
    for s in (cg.pq, cg.alpha, cg.rho_new, cg.beta):
        c.store_write(s, np.zeros(()))
    c.graph_begin()
    cg.iteration()
    g = c.graph_end()
    for _ in range(3):
        c.graph_launch(g)
        rho_c.append(float(c.store_read(cg.rho, [], "f64")))
    x_c = c.store_read(cg.x, [m * m], "f64")
    st = c.stats()
    c.graph_destroy(g)
    c.close()
    assert st["memo_misses"] == 0
    assert rho_c == rho_a and np.array_equal(x_c, x_a)
    xo, ho = wl.cg(rowptr, col, val, b, 3)
    assert rel_err_floor(x_c, xo) <= 1e-12
    for g, o in zip(rho_c, ho):
        assert abs(g - o) <= 1e-10 * o
