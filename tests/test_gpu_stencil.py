"""Stencil-shaped windows: several views of one store shifted by one row or
column (section 2's aliasing views), on grids whose interior leaves ragged
tiles in both directions.  Fused execution must equal unfused execution bit
for bit and match the oracle's op-by-op evaluation."""
import numpy as np
import pytest

import synth
from oracle import stream as OS
from oracle.ir import NoneP, Task, Tiling

from gpu_util import ctx, note, rel_err, rel_err_floor, upload

pytestmark = pytest.mark.gpu

TOL_ELEM_F64 = 1e-12
TOL_ELEM_F32 = 1e-4
TOL_RED = 1e-10


def _views(shape, shifts):
    """Interior views of an (R, C) grid shifted by (dr, dc) from offset (1, 1)."""
    R, C = shape
    tile = (R - 2, C - 2)
    return tile, [Tiling(tile, (1 + dr, 1 + dc)) for dr, dc in shifts]


def _five_point(shape):
    tile, (c, n, s, w, e) = _views(shape, [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)])
    T = Tiling(tile, (0, 0))
    d = (1, 1)
    tasks = [Task("add", d, [("G", c, "R"), ("G", n, "R"), ("t1", T, "W")]),
             Task("add", d, [("t1", T, "R"), ("G", e, "R"), ("t2", T, "W")]),
             Task("add", d, [("t2", T, "R"), ("G", w, "R"), ("t3", T, "W")]),
             Task("add", d, [("t3", T, "R"), ("G", s, "R"), ("avg", T, "W")]),
             Task("mul_imm", d, [("avg", T, "R"), ("work", T, "W")], (0.2,)),
             Task("sub", d, [("work", T, "R"), ("G", c, "R"), ("dd", T, "W")]),
             Task("sumsq", d, [("dd", T, "R"), ("ss", NoneP(), "Rd")], (1,))]
    outs = {"work": tile, "dd": tile, "ss": ()}
    temps = {"t1": tile, "t2": tile, "t3": tile, "avg": tile}
    return tasks, outs, temps


def _diagonal(shape):
    """Four diagonal neighbours and a stream of a second store."""
    tile, (a, b, c, d_) = _views(shape, [(-1, -1), (1, 1), (-1, 1), (1, -1)])
    T = Tiling(tile, (0, 0))
    d = (1, 1)
    tasks = [Task("sub", d, [("G", a, "R"), ("G", b, "R"), ("t1", T, "W")]),
             Task("mul", d, [("t1", T, "R"), ("G", c, "R"), ("t2", T, "W")]),
             Task("add", d, [("t2", T, "R"), ("G", d_, "R"), ("t3", T, "W")]),
             Task("mul", d, [("t3", T, "R"), ("H", Tiling(tile, (1, 1)), "R"), ("out", T, "W")]),
             Task("dot", d, [("out", T, "R"), ("G", a, "R"), ("s", NoneP(), "Rd")], (1,))]
    return tasks, {"out": tile, "s": ()}, {"t1": tile, "t2": tile, "t3": tile}


def _horizontal(shape):
    tile, (l, m, r) = _views(shape, [(0, -1), (0, 0), (0, 1)])
    T = Tiling(tile, (0, 0))
    d = (1, 1)
    tasks = [Task("add", d, [("G", l, "R"), ("G", r, "R"), ("t1", T, "W")]),
             Task("mul_imm", d, [("t1", T, "R"), ("t2", T, "W")], (0.5,)),
             Task("sub", d, [("G", m, "R"), ("t2", T, "R"), ("out", T, "W")])]
    return tasks, {"out": tile}, {"t1": tile, "t2": tile}


def _run_gpu(tasks, outs, temps, G, H, dtype, fuse):
    c = ctx(fuse=fuse, window=16)
    npdt = np.float64 if dtype == "f64" else np.float32
    ids = {"G": upload(c, G.astype(npdt)), "H": upload(c, H.astype(npdt))}
    for k, sh in list(outs.items()) + list(temps.items()):
        ids[k] = c.store_create(list(sh), dtype)
    parts = {}

    def part(P):
        if P not in parts:
            parts[P] = c.part_none() if isinstance(P, NoneP) else c.part_tiling(list(P.tile), list(P.offset))
        return parts[P]
    for t in tasks:
        c.submit(t.op, list(t.domain), [(ids[s], part(P), pr) for (s, P, pr) in t.args], t.imm)
    # temporaries die with the program's last reference, as in a NumPy program
    for k in temps:
        c.store_release(ids[k])
    c.flush()
    got = {k: c.store_read(ids[k], list(sh), dtype) for k, sh in outs.items()}
    c.close()
    return got


@pytest.mark.parametrize("make", [_five_point, _diagonal, _horizontal])
@pytest.mark.parametrize("shape", [(67, 301), (34, 131), (130, 258)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_shifted_views_fused_unfused_oracle(make, shape, dtype):
    note("stencil %s shape=%s %s" % (make.__name__, shape, dtype))
    tasks, outs, temps = make(shape)
    n = shape[0] * shape[1]
    G = synth.uniform(7, 0, n, 0.5, 2.0).reshape(shape)
    H = synth.uniform(7, 1, n, 0.5, 2.0).reshape(shape)
    npdt = np.float64 if dtype == "f64" else np.float32
    fused = _run_gpu(tasks, outs, temps, G, H, dtype, True)
    unfused = _run_gpu(tasks, outs, temps, G, H, dtype, False)
    for k in outs:
        assert np.array_equal(fused[k], unfused[k]), k
    ost = {"G": G.astype(npdt).astype(np.float64), "H": H.astype(npdt).astype(np.float64)}
    for k, sh in list(outs.items()) + list(temps.items()):
        ost[k] = np.zeros(sh)
    OS.evaluate(tasks, ost)
    tol = TOL_ELEM_F64 if dtype == "f64" else TOL_ELEM_F32
    for k, sh in outs.items():
        if sh == ():
            assert rel_err(fused[k], ost[k]) <= (TOL_RED if dtype == "f64" else TOL_ELEM_F32), k
        else:
            assert rel_err_floor(fused[k], ost[k]) <= tol, k
