"""Launch shapes that must not change a bit, each against its own switch:
row_split (waves per tile of passes without reductions), col_shift (strips
started early so that views misaligned alike access aligned vectors),
red_split (compiled passes with one reduction: a block of four waves per
tile, summands added in the canonical order; red_glob: a one-tile pass
over four blocks, its summands added by the block-sum reduction), fin_attach (a compiled
one-block pass reduces the block sums an earlier pass left, in place of the
block-sum kernel) and realign (compiled passes whose outputs share one
misalignment and inputs another: strips shifted for the outputs, inputs
loaded as aligned vectors and shifted across lanes).  Every workload runs with the shape on and with it off
and must give identical results; the misaligned views are also checked
against numpy."""
import numpy as np
import pytest

import paper_2406_18109_amd as dfx
import synth
from gpu_util import note, upload
from test_gpu_parity import cg_gpu, jacobi_gpu

pytestmark = pytest.mark.gpu

SWITCHES = ("DFX_ROW_SPLIT", "DFX_COL_SHIFT", "DFX_RED_SPLIT", "DFX_FIN_ATTACH", "DFX_REALIGN", "DFX_RED_GLOB")


def _runs(monkeypatch, fn, jit):
    """fn() with every shape on, then with each switched off in turn."""
    out = []
    for off in (None,) + SWITCHES:
        for s in SWITCHES:
            monkeypatch.delenv(s, raising=False)
        if off:
            monkeypatch.setenv(off, "0")
        if jit:
            monkeypatch.setenv("DFX_JIT", "2")
        else:
            monkeypatch.delenv("DFX_JIT", raising=False)
        out.append((off, fn()))
    for s in SWITCHES + ("DFX_JIT",):
        monkeypatch.delenv(s, raising=False)
    return out


def _same(results):
    (_, ref) = results[0]
    for off, r in results[1:]:
        for a, b in zip(ref, r):
            assert np.array_equal(np.asarray(a), np.asarray(b)), off


@pytest.mark.parametrize("jit", [0, 2])
def test_jacobi_shapes(monkeypatch, jit):
    note("shapes jacobi 131 jit=%d" % jit)

    def run():
        grid, res, c = jacobi_gpu(131, 3, read_every=True)
        c.close()
        return grid, res
    _same(_runs(monkeypatch, run, jit))


@pytest.mark.parametrize("jit", [0, 2])
@pytest.mark.parametrize("m", [40, 150])
def test_cg_shapes(monkeypatch, jit, m):
    note("shapes cg %d jit=%d" % (m, jit))

    def run():
        _, rho, x, c = cg_gpu(m, 6)
        c.close()
        return rho, x
    _same(_runs(monkeypatch, run, jit))


@pytest.mark.parametrize("dtype,cols", [("f32", 1032), ("f64", 1030)])
@pytest.mark.parametrize("off", [(1, 1), (0, 1), (2, 3)])
def test_misaligned_views(monkeypatch, dtype, cols, off):
    """y[v] = a[v] + 2 b[v] and z[v] = a[v] * b[v] through one view v at
    `off`: every stream's vectors start inside a 16-byte word unless the
    strips are shifted."""
    note("shapes misaligned %s off=%s" % (dtype, off))
    npdt = np.float64 if dtype == "f64" else np.float32
    R = 70
    h, w = R - 3, cols - 3
    A = synth.uniform(11, 0, R * cols, -1.0, 1.0).astype(npdt).reshape(R, cols)
    B = synth.uniform(11, 1, R * cols, -1.0, 1.0).astype(npdt).reshape(R, cols)

    def run():
        c = dfx.Context(device=0, window_size=8)
        ha, hb = upload(c, A), upload(c, B)
        hy = upload(c, np.zeros((R, cols), npdt))
        hz = upload(c, np.zeros((R, cols), npdt))
        T0 = c.part_tiling([h, w])
        V = c.part_tiling([h, w], list(off))
        t = c.store_create([h, w], dtype)
        c.submit("mul_imm", [1, 1], [(hb, V, "R"), (t, T0, "W")], (2.0,))
        c.submit("add", [1, 1], [(ha, V, "R"), (t, T0, "R"), (hy, V, "W")])
        c.submit("mul", [1, 1], [(ha, V, "R"), (hb, V, "R"), (hz, V, "W")])
        c.store_release(t)
        y = c.store_read(hy, [R, cols], dtype)
        z = c.store_read(hz, [R, cols], dtype)
        c.close()
        return y, z
    res = _runs(monkeypatch, run, 0)
    _same(res)
    y, z = res[0][1]
    r0, c0 = off
    sa, sb = A[r0:r0 + h, c0:c0 + w], B[r0:r0 + h, c0:c0 + w]
    ey = np.zeros((R, cols), npdt)
    ez = np.zeros((R, cols), npdt)
    ey[r0:r0 + h, c0:c0 + w] = sa + sb * npdt(2.0)
    ez[r0:r0 + h, c0:c0 + w] = sa * sb
    assert np.array_equal(y, ey) and np.array_equal(z, ez)


@pytest.mark.parametrize("dtype,n", [("f64", (1 << 25) + 3 * 4096 + 77), ("f32", (1 << 24) + 5), ("f64", 70000)])
def test_fin_attach_many_blocks(monkeypatch, dtype, n):
    """A reduction over thousands of blocks (several chunks of block sums,
    the last one ragged), then a one-element task that reads its result and
    one that does not: with every pass compiled, the one-element pass reduces
    the block sums itself (one launch fewer) and every bit stays the same."""
    note("shapes fin attach %s n=%d" % (dtype, n))
    npdt = np.float64 if dtype == "f64" else np.float32
    x = synth.uniform(7, 3, n, -1.0, 1.0).astype(npdt)

    def run(attach):
        monkeypatch.setenv("DFX_JIT", "2")
        if attach:
            monkeypatch.delenv("DFX_FIN_ATTACH", raising=False)
        else:
            monkeypatch.setenv("DFX_FIN_ATTACH", "0")
        try:
            c = dfx.Context(device=0, window_size=8, tune=False)
            hx = upload(c, x)
            N, T = c.part_none(), c.part_tiling([n])
            out = []
            for rep in range(2):   # the second round runs the memoised, compiled plans
                ss = c.store_create([], dtype)
                c.submit("sumsq", [1], [(hx, T, "R"), (ss, N, "Rd")], (1,))
                two = c.store_create([], dtype)
                c.submit("sqrt", [], [(ss, N, "R"), (two, N, "W")])
                c.flush()
                c.stats_reset()
                c.submit("sumsq", [1], [(hx, T, "R"), (ss, N, "Rd")], (1,))
                c.submit("sqrt", [], [(ss, N, "R"), (two, N, "W")])
                c.flush()
                out.append((c.store_read(ss, [], dtype), c.store_read(two, [], dtype), c.stats()["launches"]))
                c.store_release(ss)
                c.store_release(two)
            c.close()
            return out[-1]
        finally:
            monkeypatch.delenv("DFX_JIT", raising=False)
            monkeypatch.delenv("DFX_FIN_ATTACH", raising=False)
    a_ss, a_r, a_l = run(True)
    b_ss, b_r, b_l = run(False)
    assert np.array_equal(a_ss, b_ss) and np.array_equal(a_r, b_r)
    assert a_l == b_l - 1, (a_l, b_l)
    ref = float(np.sum(x.astype(np.float64) ** 2))
    assert abs(float(a_ss) - ref) <= (1e-10 if dtype == "f64" else 1e-4) * ref


@pytest.mark.parametrize("dtype,cols,offs", [
    ("f64", 1030, ((1, 1), (0, 0), (2, 2), (1, 3))),    # output 1 past a word, inputs 1, 1, 0
    ("f32", 1032, ((1, 1), (0, 0), (2, 2), (1, 3))),    # output 1, inputs 3, 1, 2
    ("f32", 1032, ((0, 2), (2, 1), (1, 3), (0, 0))),    # output 2, inputs 3, 1, 2
])
def test_realigned_inputs(monkeypatch, dtype, cols, offs):
    """y[vo] = a[va] + b[vb] * c[vc] with the output view misaligned one way
    and the inputs others, every pass compiled: realigned and plain runs give
    the same bits, and numpy's."""
    note("shapes realign %s offs=%s" % (dtype, offs))
    npdt = np.float64 if dtype == "f64" else np.float32
    R = 70
    h, w = R - 3, cols - 3
    arrs = [synth.uniform(12, k, R * cols, -1.0, 1.0).astype(npdt).reshape(R, cols) for k in range(3)]

    def run():
        c = dfx.Context(device=0, window_size=8)
        ha, hb, hc = (upload(c, x) for x in arrs)
        hy = upload(c, np.zeros((R, cols), npdt))
        vo, va, vb, vc = (c.part_tiling([h, w], list(o)) for o in offs)
        T0 = c.part_tiling([h, w])
        t = c.store_create([h, w], dtype)
        c.submit("mul", [1, 1], [(hb, vb, "R"), (hc, vc, "R"), (t, T0, "W")])
        c.submit("add", [1, 1], [(ha, va, "R"), (t, T0, "R"), (hy, vo, "W")])
        c.store_release(t)
        y = c.store_read(hy, [R, cols], dtype)
        n = c.stats()["compiled_launches"]
        c.close()
        return y, n
    res = _runs(monkeypatch, run, 2)
    _same(res)
    y, n = res[0][1]
    assert n >= 1
    sl = lambda x, o: x[o[0]:o[0] + h, o[1]:o[1] + w]
    ey = np.zeros((R, cols), npdt)
    ey[offs[0][0]:offs[0][0] + h, offs[0][1]:offs[0][1] + w] = sl(arrs[0], offs[1]) + sl(arrs[1], offs[2]) * sl(arrs[2], offs[3])
    assert np.array_equal(y, ey)
