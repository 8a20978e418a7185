"""Compiled passes (dfx_config.jit) against the interpreter through the C ABI:
every workload gives the same bits with its passes compiled as interpreted
(the compiled kernel is the op-list kernel template with the pass's
instructions as constants), and the compiled path really ran (the context's
compiled_launches).  Covers transcendental passes (Black-Scholes FP64 and
FP32, ragged sizes), random 2-D windows with shifted views and unaligned
widths (the clamped and per-element step modes), SpMV + dot (CG, the GMG
V-cycle's rectangular transfers and one-tile passes), the stencil-staged
Jacobi update, graph capture of compiled passes, the allocation-free flush,
and the background compiler (jit = 1) switching a pass over mid-run."""
import numpy as np
import pytest

import paper_2406_18109_amd as dfx
import synth
from gpu_util import bs_run, note, upload
from oracle import workloads as wl
from test_gpu_parity import _random_stream, cg_gpu, jacobi_gpu
from oracle.ir import NoneP

pytestmark = pytest.mark.gpu


def _twice(monkeypatch, fn):
    """fn() interpreted, then with DFX_JIT=2 (every context compiles its
    passes synchronously at their first execution)."""
    monkeypatch.delenv("DFX_JIT", raising=False)
    a = fn()
    monkeypatch.setenv("DFX_JIT", "2")
    try:
        b = fn()
    finally:
        monkeypatch.delenv("DFX_JIT", raising=False)
    return a, b


@pytest.mark.parametrize("dtype,n", [("f64", 3 * 4096 + 77), ("f64", (1 << 16) + 128), ("f32", 70000), ("f32", 5)])
def test_black_scholes_compiled_bitwise(dtype, n, monkeypatch):
    note("jit bs %s n=%d" % (dtype, n))
    monkeypatch.delenv("DFX_JIT", raising=False)
    outs = []
    for jit in (0, 2):
        c = dfx.Context(device=0, window_size=64, jit=jit)
        _, call, put = bs_run(c, n, dtype)
        outs.append((call, put, c.stats()["compiled_launches"]))
        c.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == 0 and outs[1][2] >= 1


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("shape", [(7, 9), (131, 257)])
def test_random_windows_compiled_bitwise(seed, shape, monkeypatch):
    import random
    rng = random.Random(seed * 1000 + shape[1])
    tasks, stores = _random_stream(rng, shape)
    note("jit random window seed=%d shape=%s" % (seed, shape))
    G = synth.uniform(seed, 0, shape[0] * shape[1], 0.5, 2.0).reshape(shape)
    H = synth.uniform(seed, 1, shape[0] * shape[1], 0.5, 2.0).reshape(shape)

    def run():
        c = dfx.Context(device=0, window_size=8)
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
        got = {k: c.store_read(ids[k], list(stores[k]), "f64") for k in ("H", "s0", "s1", "t5", "t4")}
        n = c.stats()["compiled_launches"]
        c.close()
        return got, n
    (a, na), (b, nb) = _twice(monkeypatch, run)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    assert na == 0 and nb >= 1


def test_spmv_same_program_fp64_then_fp32(monkeypatch):
    """An SpMV-only pass (empty op list) compiled for FP64 and then for FP32
    in one process: each element type gets its own kernel."""
    from test_gpu_parity import _irregular_csr
    n = 4095
    rowptr, col, val = _irregular_csr(n, 40 + n)
    x = synth.uniform(41 + n, 0, n, -1.0, 1.0)
    for dtype in ("f64", "f32"):
        note("jit spmv only %s" % dtype)
        npdt = np.float64 if dtype == "f64" else np.float32

        def run():
            c = dfx.Context(device=0, window_size=8, fuse=False)
            hr, hc = upload(c, rowptr), upload(c, col)
            hv, hx = upload(c, val.astype(npdt)), upload(c, x.astype(npdt))
            hy = c.store_create([n], dtype)
            N, T = c.part_none(), c.part_tiling([n])
            c.submit("spmv_csr", [1], [(hr, N, "R"), (hc, N, "R"), (hv, N, "R"), (hx, c.part_image(hc, N), "R"),
                                       (hy, T, "W")])
            c.flush()
            y = c.store_read(hy, [n], dtype)
            k = c.stats()["compiled_launches"]
            c.close()
            return y, k
        (ya, ka), (yb, kb) = _twice(monkeypatch, run)
        assert np.array_equal(ya, yb), dtype
        assert ka == 0 and kb == 1


def test_cg_compiled_bitwise(monkeypatch):
    note("jit cg 150^2")

    def run():
        _, rho, x, c = cg_gpu(150, 12)
        n = c.stats()["compiled_launches"]
        c.close()
        return rho, x, n
    (ra, xa, na), (rb, xb, nb) = _twice(monkeypatch, run)
    assert ra == rb and np.array_equal(xa, xb)
    assert na == 0 and nb >= 12


def test_jacobi_stencil_compiled_bitwise(monkeypatch):
    note("jit jacobi 260")

    def run():
        grid, res, c = jacobi_gpu(260, 4, read_every=True)
        n = c.stats()["compiled_launches"]
        c.close()
        return grid, res, n
    (ga, ra, na), (gb, rb, nb) = _twice(monkeypatch, run)
    assert np.array_equal(ga, gb) and ra == rb
    assert na == 0 and nb >= 4
    # the sweep is + and * only: the oracle's bits
    ref = synth.jacobi_grid(260)
    wl.jacobi(ref, 4)
    assert np.array_equal(gb, ref)


def test_gmg_compiled_bitwise(monkeypatch):
    note("jit gmg 63, 5 levels")
    from test_gpu_gmg import _solver
    m, nlev = 63, 5
    b = synth.rhs(m * m, 4215)

    def run():
        c = dfx.Context(device=0, window_size=16)
        g = _solver(c, m, nlev, b)
        rr = []
        for _ in range(2):
            g.iteration()
            rr.append(float(c.store_read(g.rr, [], "f64")))
        x = c.store_read(g.x, [m * m], "f64")
        n = c.stats()["compiled_launches"]
        c.close()
        return rr, x, n
    (ra, xa, na), (rb, xb, nb) = _twice(monkeypatch, run)
    assert ra == rb and np.array_equal(xa, xb)
    assert na == 0 and nb > 0


@pytest.mark.parametrize("m", [100, 64])
def test_graph_of_compiled_passes(monkeypatch, m):
    """A CG iteration recorded as a graph after one eager (compiling)
    iteration: three replays equal three eager interpreted iterations (64^2:
    one-tile reducing passes over several blocks, their block-sum reduction
    in the next scalar pass)."""
    note("jit cg graph %d" % m)
    monkeypatch.delenv("DFX_JIT", raising=False)
    rowptr, col, val = synth.poisson_csr(m, 2)
    b = synth.rhs(m * m, 4321)
    out = []
    for jit in (0, 2):
        c = dfx.Context(device=0, window_size=16, jit=jit)
        cg = dfx.apps.CG(c, *[upload(c, a) for a in (rowptr, col, val, b)], m * m)
        cg.iteration()
        c.flush()
        rho = [float(c.store_read(cg.rho, [], "f64"))]
        if jit:
            c.stats_reset()
            c.graph_begin()
            cg.iteration()
            gid = c.graph_end()
            for _ in range(3):
                c.graph_launch(gid)
                rho.append(float(c.store_read(cg.rho, [], "f64")))
            assert c.stats()["compiled_launches"] > 0
        else:
            for _ in range(3):
                cg.iteration()
                rho.append(float(c.store_read(cg.rho, [], "f64")))
        out.append((rho, c.store_read(cg.x, [m * m], "f64")))
        c.close()
    assert out[0][0] == out[1][0] and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("m", [300, 64])
def test_noalloc_flush_compiled(monkeypatch, m):
    """dfx_flush_noalloc runs compiled passes with the scratch array (64^2:
    one-tile reducing passes over several blocks, their summands in the
    scratch array)."""
    note("jit noalloc flush cg %d" % m)
    from test_zz_no_alloc import _cg
    (_, rho_a, x_a), (_, rho_b, x_b) = _twice(monkeypatch, lambda: _cg(m, 5, True))
    assert rho_a == rho_b and np.array_equal(x_a, x_b)


def test_background_compile_switches_mid_run(monkeypatch):
    """jit = 1: the pass runs interpreted until its kernel is ready, then
    compiled; every execution gives the same bits."""
    note("jit background bs")
    monkeypatch.delenv("DFX_JIT", raising=False)
    n = 100003
    c0 = dfx.Context(device=0, window_size=64)
    _, call0, put0 = bs_run(c0, n)
    c0.close()
    c = dfx.Context(device=0, window_size=64, jit=1)
    _, call1, put1 = bs_run(c, n)
    dfx.jit_wait()
    _, call2, put2 = bs_run(c, n)
    assert c.stats()["compiled_launches"] >= 1
    info = dfx.jit_info()
    assert info["pending"] == 0 and info["compiled"] + info["disk_hits"] >= 1
    c.close()
    for a, b in ((call0, call1), (put0, put1), (call0, call2), (put0, put2)):
        assert np.array_equal(a, b)
