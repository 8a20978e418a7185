"""GPU parity through the C ABI: fused vs unfused (bit for bit) and GPU vs
the CPU oracle (within the stated tolerances), at sizes that span several
tiles and a ragged tail, plus edge cases."""
import math
import random

import numpy as np
import pytest

import paper_2406_18109_amd as dfx
import synth
from oracle import stream as OS
from oracle import workloads as wl
from oracle.ir import NoneP, Proj, Task, Tiling

from gpu_util import bs_run, ctx, note, rel_err, rel_err_floor, upload

pytestmark = pytest.mark.gpu

TOL_ELEM_F64 = 1e-12   # |g-o| <= 1e-12 max(|o|, 1)
TOL_ELEM_F32 = 1e-4    # float32 stream against the float64 oracle
TOL_RED = 1e-10        # reductions and CG residuals, relative


@pytest.mark.parametrize("n", [1, 77, 3 * 4096 + 77, (1 << 16) + 128])
def test_black_scholes_f64(n):
    note("bs f64 n=%d" % n)
    cf, cu = ctx(fuse=True), ctx(fuse=False)
    (S, K, T, r, sig, rv), call, put = bs_run(cf, n)
    _, call_u, put_u = bs_run(cu, n)
    assert np.array_equal(call, call_u) and np.array_equal(put, put_u)
    oc, op = wl.black_scholes(S, K, T, r, sig, rv)
    assert rel_err_floor(call, oc) <= TOL_ELEM_F64
    assert rel_err_floor(put, op) <= TOL_ELEM_F64
    assert [g["prefix_len"] for g in cf.groups()][-1] == 28
    assert cu.stats()["launches"] == 28


@pytest.mark.parametrize("n", [5, 4096 + 3, 70000])
def test_black_scholes_f32(n):
    note("bs f32 n=%d" % n)
    cf, cu = ctx(fuse=True), ctx(fuse=False)
    (S, K, T, r, sig, rv), call, put = bs_run(cf, n, "f32")
    _, call_u, put_u = bs_run(cu, n, "f32")
    assert np.array_equal(call, call_u) and np.array_equal(put, put_u)
    oc, op = wl.black_scholes(S.astype(np.float64), K.astype(np.float64), T.astype(np.float64), r, sig, rv)
    assert rel_err_floor(call, oc) <= TOL_ELEM_F32
    assert rel_err_floor(put, op) <= TOL_ELEM_F32


def test_black_scholes_multi_point_launch_and_repeat():
    n = 4 * 5000
    note("bs points=4")
    c4 = ctx()
    _, call4, put4 = bs_run(c4, n, points=4, passes=3)
    c1 = ctx()
    _, call1, put1 = bs_run(c1, n, points=1)
    assert np.array_equal(call4, call1) and np.array_equal(put4, put1)
    g = c4.groups()
    assert g[-1]["memo_hit"]


def jacobi_gpu(N, sweeps, fuse=True, window=16, read_every=False):
    c = ctx(fuse=fuse, window=window)
    g0 = synth.jacobi_grid(N)
    G = upload(c, g0)
    J = dfx.apps.Jacobi(c, G, N)
    res = []
    last = None
    for _ in range(sweeps):
        last = J.sweep()
        if read_every:
            res.append(float(c.store_read(last, [], "f64")))
    if not read_every:
        res.append(float(c.store_read(last, [], "f64")))
    grid = c.store_read(G, [N, N], "f64")
    return grid, res, c


@pytest.mark.parametrize("N", [4, 6, 34, 131, 260])
def test_jacobi_bitwise_against_oracle(N):
    note("jacobi N=%d" % N)
    sweeps = 5
    grid_f, res_f, cf = jacobi_gpu(N, sweeps, read_every=True)
    grid_u, res_u, _ = jacobi_gpu(N, sweeps, fuse=False, read_every=True)
    grid_l, res_l, _ = jacobi_gpu(N, sweeps, read_every=False)   # lazy: one flush at the end
    assert np.array_equal(grid_f, grid_u) and res_f == res_u
    assert np.array_equal(grid_f, grid_l) and res_l[-1] == res_f[-1]
    ref = synth.jacobi_grid(N)
    ores = wl.jacobi(ref, sweeps)
    # the sweep is + and * only, in the paper's order: identical bits
    assert np.array_equal(grid_f, ref)
    for g, o in zip(res_f, ores):
        assert abs(g - o) <= TOL_RED * abs(o)


def cg_gpu(m, iters, fuse=True, window=16, dim=2, seed=synth.CG64_SEED):
    c = ctx(fuse=fuse, window=window)
    rowptr, col, val = synth.poisson_csr(m, dim)
    n = m ** dim
    b = synth.rhs(n, seed)
    hs = [upload(c, a) for a in (rowptr, col, val, b)]
    cg = dfx.apps.CG(c, *hs, n)
    rho = [float(c.store_read(cg.rho, [], "f64"))]
    for _ in range(iters):
        cg.iteration()
        rho.append(float(c.store_read(cg.rho, [], "f64")))
    x = c.store_read(cg.x, [n], "f64")
    return (rowptr, col, val, b), rho, x, c


def test_cg64_fused_unfused_oracle():
    note("cg64")
    (rowptr, col, val, b), rho_f, x_f, cf = cg_gpu(64, 100)
    _, rho_u, x_u, _ = cg_gpu(64, 100, fuse=False)
    assert rho_f == rho_u and np.array_equal(x_f, x_u)
    xo, ho = wl.cg(rowptr, col, val, b, 100)
    for k, (g, o) in enumerate(zip(rho_f, ho)):
        assert abs(g - o) <= TOL_RED * abs(o), k
    assert rel_err_floor(x_f, xo) <= 1e-9


def test_cg_3d_small():
    note("cg 3d m=12")
    (rowptr, col, val, b), rho, x, _ = cg_gpu(12, 30, dim=3, seed=synth.CG256_SEED)
    xo, ho = wl.cg(rowptr, col, val, b, 30)
    for g, o in zip(rho, ho):
        assert abs(g - o) <= TOL_RED * abs(o)


@pytest.mark.parametrize("n", [1, 63, 1000, 4097, (1 << 20) + 5])
def test_reductions_canonical_order(n):
    note("reductions n=%d" % n)
    x = synth.uniform(71, 0, n, 0.0, 1.0)
    y = synth.uniform(71, 1, n, -1.0, 1.0)
    outs = []
    for fuse in (True, False):
        c = ctx(fuse=fuse)
        hx, hy = upload(c, x), upload(c, y)
        T = c.part_tiling([n])
        N0 = c.part_none()
        s1, s2, s3 = (c.store_create([], "f64") for _ in range(3))
        t = c.store_create([n], "f64")
        c.submit("copy", [1], [(hx, T, "R"), (t, T, "W")])
        c.submit("sum", [1], [(t, T, "R"), (s1, N0, "Rd")], (1,))
        c.submit("dot", [1], [(hx, T, "R"), (hy, T, "R"), (s2, N0, "Rd")], (1,))
        c.submit("sumsq", [1], [(hy, T, "R"), (s3, N0, "Rd")], (1,))
        c.store_release(t)
        outs.append([float(c.store_read(s, [], "f64")) for s in (s1, s2, s3)])
    assert outs[0] == outs[1]
    # a reduction alone equals the same reduction fused with other work
    c = ctx()
    hx = upload(c, x)
    T = c.part_tiling([n])
    s = c.store_create([], "f64")
    c.submit("sum", [1], [(hx, T, "R"), (s, c.part_none(), "Rd")], (1,))
    assert float(c.store_read(s, [], "f64")) == outs[0][0]
    from oracle import cnum
    assert rel_err(outs[0][0], cnum.fsum(x)) <= TOL_RED
    assert rel_err(outs[0][2], cnum.fsum_prod(y, y)) <= TOL_RED
    assert abs(outs[0][1] - cnum.fsum_prod(x, y)) <= TOL_RED * cnum.fsum_prod(np.abs(x), np.abs(y))


def test_reduction_accumulates_and_points_do_not_change_bits():
    n = 4 * 3001
    x = synth.uniform(72, 0, n, 0.0, 1.0)
    vals = []
    for pts in (1, 2, 4):
        c = ctx()
        hx = upload(c, x)
        T = c.part_tiling([n // pts])
        s = upload(c, np.array(0.5))
        c.submit("sum", [pts], [(hx, T, "R"), (s, c.part_none(), "Rd")], (0,))
        vals.append(float(c.store_read(s, [], "f64")))
    assert vals[0] == vals[1] == vals[2]
    from oracle import cnum
    assert rel_err(vals[0], 0.5 + cnum.fsum(x)) <= TOL_RED


def test_empty_and_scalar_cases():
    c = ctx()
    N0 = c.part_none()
    e = c.store_create([0], "f64")
    f = c.store_create([0], "f64")
    T = c.part_tiling([0])
    s = c.store_create([], "f64")
    c.submit("neg", [1], [(e, T, "R"), (f, T, "W")])
    c.submit("sum", [1], [(e, T, "R"), (s, N0, "Rd")], (1,))
    assert float(c.store_read(s, [], "f64")) == 0.0
    a = upload(c, np.array(2.0))
    b = upload(c, np.array(8.0))
    q = c.store_create([], "f64")
    c.submit("div", [], [(b, N0, "R"), (a, N0, "R"), (q, N0, "W")])
    c.submit("sqrt", [], [(q, N0, "R"), (q, N0, "W")])
    assert float(c.store_read(q, [], "f64")) == 2.0


# ---- random windows against the oracle's stream evaluator -------------------

def _random_stream(rng, shape):
    R, Cc = shape
    tile = (R - 1, Cc - 1)
    views = [Tiling(tile, (0, 0)), Tiling(tile, (1, 0)), Tiling(tile, (0, 1)), Tiling(tile, (1, 1))]
    full = Tiling(tile, (0, 0))
    stores = {"G": (R, Cc), "H": (R, Cc)}
    for k in range(6):
        stores["t%d" % k] = tile
    stores["a"] = ()
    stores["s0"] = ()
    stores["s1"] = ()
    tasks = []
    made = []
    for k in range(6):
        op = rng.choice(["add", "mul", "div", "max", "min", "sqrt", "abs", "square", "add_imm",
                         "mul_imm", "log", "exp", "erf"])
        srcs = ["G", "H"] + made
        def pick():
            s = rng.choice(srcs)
            if s in ("G", "H"):
                return (s, rng.choice(views), "R")
            return (s, full, "R")
        out = ("t%d" % k, full, "W")
        if op in ("add", "mul", "div", "max", "min"):
            b = ("a", NoneP(), "R") if rng.random() < 0.25 else pick()
            tasks.append(Task(op, (1, 1), [pick(), b, out]))
        elif op in ("add_imm", "mul_imm"):
            tasks.append(Task(op, (1, 1), [pick(), out], (rng.choice([0.25, 1.5, 3.0]),)))
        elif op in ("log", "exp", "erf", "sqrt"):
            s = rng.choice(["G", "H"])
            tasks.append(Task(op, (1, 1), [(s, rng.choice(views), "R"), out]))
        else:
            tasks.append(Task(op, (1, 1), [pick(), out]))
        made.append("t%d" % k)
    tasks.append(Task("sum", (1, 1), [(made[-1], full, "R"), ("s0", NoneP(), "Rd")], (1,)))
    tasks.append(Task("dot", (1, 1), [(made[-2], full, "R"), ("G", views[3], "R"), ("s1", NoneP(), "Rd")], (1,)))
    tasks.append(Task("copy", (1, 1), [(made[-1], full, "R"), ("H", views[0], "W")]))
    return tasks, stores


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("shape", [(7, 9), (40, 300), (131, 257)])
def test_random_windows_against_oracle(seed, shape):
    rng = random.Random(seed * 1000 + shape[1])
    tasks, stores = _random_stream(rng, shape)
    note("random window seed=%d shape=%s" % (seed, shape))
    G = synth.uniform(seed, 0, shape[0] * shape[1], 0.5, 2.0).reshape(shape)
    H = synth.uniform(seed, 1, shape[0] * shape[1], 0.5, 2.0).reshape(shape)
    ost = {"G": G.copy(), "H": H.copy(), "a": np.array(1.25), "s0": np.array(0.0), "s1": np.array(0.0)}
    for k, sh in stores.items():
        if k not in ost:
            ost[k] = np.zeros(sh)
    OS.evaluate(tasks, ost)
    results = []
    for fuse in (True, False):
        c = ctx(fuse=fuse, window=8)
        ids = {"G": upload(c, G), "H": upload(c, H), "a": upload(c, np.array(1.25))}
        for k, sh in stores.items():
            if k not in ids:
                ids[k] = c.store_create(list(sh), "f64")
        parts = {}
        def part(P):
            if P not in parts:
                parts[P] = c.part_none() if isinstance(P, NoneP) else c.part_tiling(list(P.tile), list(P.offset))
            return parts[P]
        for t in tasks:
            c.submit(t.op, list(t.domain), [(ids[s], part(P), pr) for (s, P, pr) in t.args], t.imm)
        got = {k: c.store_read(ids[k], list(stores[k]) if k in stores else [], "f64")
               for k in ("H", "s0", "s1", "t5", "t4")}
        results.append(got)
    for k in results[0]:
        assert np.array_equal(results[0][k], results[1][k]), k
    for k in ("H", "t5", "t4"):
        assert rel_err_floor(results[0][k], ost[k]) <= TOL_ELEM_F64, k
    for k in ("s0", "s1"):
        assert rel_err(results[0][k], ost[k]) <= TOL_RED, k


# ---- SpMV on irregular matrices -----------------------------------------------

def _irregular_csr(n, seed):
    """Row lengths 0..12 (every 97th row empty, rows 64..191 of length 40 so some
    64-row groups exceed the kernel's staged range), sorted distinct columns."""
    u = synth.uniform(seed, 0, n, 0.0, 1.0)
    lengths = np.floor(u * 13).astype(np.int64)
    lengths[::97] = 0
    lengths[64:192] = 40
    lengths = np.minimum(lengths, n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(lengths)
    nnz = int(rowptr[-1])
    cu = synth.uniform(seed, 1, nnz, 0.0, 1.0)
    col = np.empty(nnz, dtype=np.int32)
    for i in range(n):
        b, e = rowptr[i], rowptr[i + 1]
        if e > b:
            # distinct sorted columns: a stride walk from a random start
            start = int(cu[b] * n)
            step = max(1, n // max(1, e - b))
            col[b:e] = np.sort((start + step * np.arange(e - b)) % n)
    val = synth.uniform(seed, 2, nnz, -1.0, 1.0)
    return rowptr.astype(np.int32), col, val


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [1000, 4095, 20000])
def test_spmv_dot_irregular_rows(dtype, n, monkeypatch):
    """Fused and unfused, with the CSR range of each 64-row group staged in LDS
    and read directly: identical bits, and the oracle's sequential CSR sum."""
    note("spmv irregular n=%d %s" % (n, dtype))
    from oracle import cnum
    npdt = np.float64 if dtype == "f64" else np.float32
    rowptr, col, val = _irregular_csr(n, 40 + n)
    x = synth.uniform(41 + n, 0, n, -1.0, 1.0)
    outs = []
    for fuse, stage in ((True, "1"), (False, "1"), (True, "0")):
        monkeypatch.setenv("DFX_SPMV_STAGE", stage)
        c = ctx(fuse=fuse, window=8)
        hr, hc = upload(c, rowptr), upload(c, col)
        hv, hx = upload(c, val.astype(npdt)), upload(c, x.astype(npdt))
        hy = c.store_create([n], dtype)
        hs = c.store_create([], dtype)
        N = c.part_none()
        T = c.part_tiling([n])
        img = c.part_image(hc, N)
        c.submit("spmv_csr", [1], [(hr, N, "R"), (hc, N, "R"), (hv, N, "R"), (hx, img, "R"), (hy, T, "W")])
        c.submit("dot", [1], [(hx, T, "R"), (hy, T, "R"), (hs, N, "Rd")], (1,))
        c.flush()
        outs.append((c.store_read(hy, [n], dtype), c.store_read(hs, [], dtype)))
        c.close()
    for k in (1, 2):
        assert np.array_equal(outs[0][0], outs[k][0])
        assert np.array_equal(outs[0][1], outs[k][1])
    yo = cnum.spmv(rowptr, col, val.astype(npdt).astype(np.float64), x.astype(npdt).astype(np.float64))
    so = cnum.fsum_prod(x.astype(npdt).astype(np.float64), yo)
    # the dot of random-sign vectors may cancel: its error is measured against
    # the sum of the magnitudes of its terms
    scale = cnum.fsum(np.abs(x.astype(npdt).astype(np.float64) * yo))
    if dtype == "f64":
        # the same sequential CSR sum in the same precision: identical bits
        assert np.array_equal(outs[0][0], yo)
        assert abs(float(outs[0][1]) - so) <= TOL_RED * scale
    else:
        assert rel_err_floor(outs[0][0], yo) <= TOL_ELEM_F32
        assert abs(float(outs[0][1]) - so) <= 1e-4 * scale
