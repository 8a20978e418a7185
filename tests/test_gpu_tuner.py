"""The launch-shape tuner changes nothing but time: after an untimed warm-up
a memoised pass runs twice at each of 1x, 2x and 4x the default tiles per
wave, then at the fastest, and every execution's results are bit-identical
to a context with the tuner off (each candidate keeps a block's tiles an
aligned subtree of the canonical reduction tree)."""
import numpy as np
import pytest

import paper_2406_18109_amd as dfx
import synth
from gpu_util import note, upload

pytestmark = pytest.mark.gpu
REPS = 9   # warm-up, each candidate twice, the fixing execution, one more


def _ctx(tune):
    return dfx.Context(device=0, window_size=16, tune=tune)


def _reductions(tune, n):
    c = _ctx(tune)
    x = upload(c, synth.uniform(5, 0, n, -1.0, 1.0))
    y = upload(c, synth.uniform(5, 1, n, -1.0, 1.0))
    t = c.part_tiling([n])
    none = c.part_none()
    out = []
    for _ in range(REPS):
        s = c.store_create([], "f64")
        d = c.store_create([], "f64")
        z = c.store_create([n], "f64")
        c.submit("mul", [1], [(x, t, "R"), (y, t, "R"), (z, t, "W")])
        c.submit("sum", [1], [(z, t, "R"), (s, none, "Rd")], (1,))
        c.submit("dot", [1], [(x, t, "R"), (z, t, "R"), (d, none, "Rd")], (1,))
        out.append((float(c.store_read(s, [], "f64")), float(c.store_read(d, [], "f64")),
                    c.store_read(z, [n], "f64")))
        for h in (s, d, z):
            c.store_release(h)
    c.close()
    return out


def test_tuned_reductions_bit_identical():
    n = (1 << 22) + 77   # 1025 tiles, ragged tail
    note("tuner: reductions n=%d" % n)
    on, off = _reductions(True, n), _reductions(False, n)
    for (s1, d1, z1), (s0, d0, z0) in zip(on, off):
        assert s1 == s0 and d1 == d0 and np.array_equal(z1, z0)


def _jacobi(tune, N):
    c = _ctx(tune)
    G = upload(c, synth.uniform(6, 0, N * N, 0.0, 1.0).reshape(N, N))
    J = dfx.apps.Jacobi(c, G, N)
    res = [float(c.store_read(J.sweep(), [], "f64")) for _ in range(REPS)]
    grid = c.store_read(G, [N, N], "f64")
    c.close()
    return res, grid


def test_tuned_jacobi_bit_identical():
    N = 2050   # 1024 tiles in the update pass
    note("tuner: jacobi N=%d" % N)
    (r1, g1), (r0, g0) = _jacobi(True, N), _jacobi(False, N)
    assert r1 == r0 and np.array_equal(g1, g0)


def _cg(tune, m):
    c = _ctx(tune)
    rowptr, col, val = synth.poisson_csr(m, 3)
    n = m ** 3
    hs = [upload(c, a) for a in (rowptr, col, val, synth.rhs(n, synth.CG256_SEED))]
    cg = dfx.apps.CG(c, *hs, n)
    rho = []
    for _ in range(REPS):
        cg.iteration()
        rho.append(float(c.store_read(cg.rho, [], "f64")))
    x = c.store_read(cg.x, [n], "f64")
    c.close()
    return rho, x


def test_tuned_cg_bit_identical():
    m = 64   # 262144 rows, 64 tiles
    note("tuner: cg 3-D m=%d" % m)
    (r1, x1), (r0, x0) = _cg(True, m), _cg(False, m)
    assert r1 == r0 and np.array_equal(x1, x0)


@pytest.mark.parametrize("rows", ["1", "2"])
def test_rows_per_step_bit_identical(rows, monkeypatch):
    """Arithmetic passes of 4096 tiles take the one-row kernels (all waves
    resident at four per SIMD); forcing one or two rows per step gives the
    same bits, since rows are visited in order either way."""
    n = 4096 * 4096 - 5   # 4096 tiles, ragged tail
    note("rows per step: auto against %s, n=%d" % (rows, n))
    auto = _reductions(False, n)
    monkeypatch.setenv("DFX_ARITH_ROWS", rows)
    forced = _reductions(False, n)
    for (s1, d1, z1), (s0, d0, z0) in zip(forced, auto):
        assert s1 == s0 and d1 == d0 and np.array_equal(z1, z0)
