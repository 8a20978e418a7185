"""dfx_flush_noalloc (the allocation-free flush) against dfx_flush through the
C ABI: CG iterations (SpMV + dot, axpy + axpy + dot, scalar tasks) whose
reductions take their block sums from the library's fixed scratch array,
on two systems in a row, the second smaller, each bit for bit the result of
the ordinary flush and within tolerance of the oracle."""
import numpy as np
import pytest

import paper_2406_18109_amd as dfx
from paper_2406_18109_amd import _binding as B
import synth
from gpu_util import note, rel_err_floor, upload
from oracle import workloads as wl

pytestmark = pytest.mark.gpu


def _cg(m, iters, noalloc):
    """CG on the m x m Poisson system: set-up and the first iteration with
    the ordinary flush (they give every store its memory), the remaining
    iterations flushed with dfx_flush_noalloc when `noalloc`."""
    rowptr, col, val = synth.poisson_csr(m, 2)
    b = synth.rhs(m * m, 4400 + m)
    c = dfx.Context(device=0, window_size=16)
    cg = dfx.apps.CG(c, *[upload(c, a) for a in (rowptr, col, val, b)], m * m)
    rho = [float(c.store_read(cg.rho, [], "f64"))]
    cg.iteration()
    c.flush()
    rho.append(float(c.store_read(cg.rho, [], "f64")))
    for _ in range(iters - 1):
        cg.iteration()
        if noalloc:
            c.flush_noalloc()
        else:
            c.flush()
        rho.append(float(c.store_read(cg.rho, [], "f64")))
    x = c.store_read(cg.x, [m * m], "f64")
    c.close()
    return (rowptr, col, val, b), rho, x


def test_noalloc_flush_equals_flush_on_two_calls():
    iters = 6
    for m in (300, 40):   # 22 tiles, then one tile
        note("noalloc flush: cg %d^2" % m)
        sysm, rho_n, x_n = _cg(m, iters, True)
        _, rho_f, x_f = _cg(m, iters, False)
        assert rho_n == rho_f and np.array_equal(x_n, x_f)
        xo, ho = wl.cg(*sysm, iters)
        assert rel_err_floor(x_n, xo) <= 1e-12
        for g, o in zip(rho_n, ho):
            assert abs(g - o) <= 1e-10 * o


def test_noalloc_flush_refuses_a_group_that_needs_memory():
    note("noalloc flush: a new store")
    c = dfx.Context(device=0, window_size=16)
    n = 5000
    a = upload(c, synth.uniform(4500, 0, n, -1.0, 1.0))
    T = c.part_tiling([n])
    out = c.store_create([n], "f64")          # never written: no memory yet
    c.submit("mul_imm", [1], [(a, T, "R"), (out, T, "W")], (2.0,))
    with pytest.raises(B.DfxError) as e:
        c.flush_noalloc()
    assert e.value.code == B.ESTATE
    c.flush()                                 # the ordinary flush allocates and runs it
    assert np.array_equal(c.store_read(out, [n], "f64"), 2.0 * c.store_read(a, [n], "f64"))
    c.close()
