"""Pins for the oracle's fusion analysis (sections 3-5) against the paper's
worked examples and against brute-force dependence maps."""
import random

import numpy as np

from oracle import analysis as A
from oracle.ir import Image, NoneP, Proj, Task, Tiling, points, substore_points, tiling_box

from test_oracle_jacobi import stencil_tasks


# --- Section 3.1, the Tiling examples and the sub-store-bounds formula ------

def test_tiling_examples():
    # 2x2 tiles of a 4x4 store over a 2x2 domain
    P = Tiling((2, 2), (0, 0))
    assert tiling_box(P, (1, 0), (4, 4)) == ((2, 0), (4, 2))
    # 1x4 row tiles over a 4x1 domain
    P = Tiling((1, 4), (0, 0))
    assert tiling_box(P, (3, 0), (4, 4)) == ((3, 0), (4, 4))
    # tiles offset by (1, 1)
    P = Tiling((2, 2), (1, 1))
    assert tiling_box(P, (0, 0), (4, 4)) == ((1, 1), (3, 3))
    assert tiling_box(P, (1, 1), (4, 4)) == ((3, 3), (4, 4))  # clipped
    # a size-4 vector blocked over a 2-D domain, second dim dropped: aliased
    P = Tiling((2,), (0,), Proj((0,)))
    assert substore_points((4,), P, (0, 0)) == substore_points((4,), P, (0, 1)) == {(0,), (1,)}
    assert substore_points((4,), P, (1, 1)) == {(2,), (3,)}


# --- Section 4.1, dependence maps ------------------------------------------

def test_dependence_maps_pointwise_and_stencil():
    shapes = {"A": (4,), "B": (4,)}
    T = Tiling((1,), (0,))
    t1 = Task("w", (4,), [("A", T, "W")])
    t2 = Task("r", (4,), [("A", T, "R"), ("B", T, "W")])
    D = A.dependence_map(t1, t2, shapes)
    assert all(D[p] == {p} for p in D)
    assert A.fusible(t1, t2, shapes)
    t3 = Task("r", (4,), [("A", Tiling((1,), (-1,)), "R"), ("A", T, "R"),
                          ("A", Tiling((1,), (1,)), "R"), ("B", T, "W")])
    D = A.dependence_map(t1, t3, shapes)
    for (p,) in D:
        assert D[(p,)] == {(q,) for q in (p - 1, p, p + 1) if 0 <= q < 4}
    assert not A.fusible(t1, t3, shapes)
    # write through one partition, read through another: not point-wise
    t4 = Task("r", (4,), [("A", Tiling((1,), (1,)), "R"), ("B", T, "W")])
    assert not A.fusible(t1, t4, shapes)
    # reductions to the same store do not depend on each other
    t5 = Task("rd", (4,), [("A", NoneP(), "Rd")])
    t6 = Task("rd", (4,), [("A", NoneP(), "Rd")])
    assert A.fusible(t5, t6, {"A": ()})


# --- Section 2 / figure 1: the stencil stream --------------------------------

def _shapes_stencil(N):
    m = N - 2
    s = {"grid": (N, N), "ss": ()}
    for k in ("t1", "t2", "t3", "avg", "work", "d"):
        s[k] = (m, m)
    return s


def test_figure1_stencil_prefix_and_temporaries():
    N = 6
    tasks = stencil_tasks(N, (2, 2), with_residual=False)
    # the next iteration's first task follows the COPY
    nxt = stencil_tasks(N, (2, 2), with_residual=False)
    window = tasks + nxt[:1]
    shapes = _shapes_stencil(N)
    f = A.longest_prefix(window)
    assert f == 5  # 4 ADD + MULT fuse; the COPY does not
    temps = A.temporaries(window, f, app_live={"grid"}, shapes=shapes)
    assert temps == {"t1", "t2", "t3", "avg"}  # work is read by the pending COPY
    assert A.prefix_fusible(window[:f], shapes)
    # the COPY cannot fuse with the next iteration's reads of the views
    rest = window[f:]
    assert A.longest_prefix(rest) == 1
    assert not A.prefix_fusible(rest[:2], shapes)


def test_stencil_with_residual_prefix():
    N = 6
    tasks = stencil_tasks(N, (1, 1))
    shapes = _shapes_stencil(N)
    f = A.longest_prefix(tasks)
    assert f == 7
    temps = A.temporaries(tasks, f, app_live={"grid", "ss"}, shapes=shapes)
    assert temps == {"t1", "t2", "t3", "avg", "d"}


# --- Section 5.1 / figure 5: temporaries -------------------------------------

def test_figure5_temporaries():
    n = 8
    T = Tiling((4,), (0,))
    half = Tiling((2,), (4,))
    d = (2,)
    window = [
        Task("mul_imm", d, [("x", T, "R"), ("z", T, "W")], (2.0,)),
        Task("add", d, [("y", T, "R"), ("z", T, "R"), ("w", T, "W")]),
        Task("pow", d, [("w", T, "R"), ("v", T, "W")]),
        Task("sumsq", d, [("w", half, "R"), ("norm", NoneP(), "Rd")], (1,)),
    ]
    shapes = {k: (n,) for k in "xyzwv"}
    shapes["norm"] = ()
    f = A.longest_prefix(window)
    assert f == 3
    assert A.temporaries(window, f, app_live={"v", "norm"}, shapes=shapes) == {"z"}
    assert A.prefix_fusible(window[:f], shapes)
    assert not A.prefix_fusible(window, shapes)


# --- Section 5.2 / figure 6: isomorphic streams ------------------------------

def test_figure6_canonical_forms():
    d = (1,)
    T = Tiling((4,), (0,))

    def mk(pairs):
        return [Task("t%d" % i, d, [(a, T, "R"), (b, T, "W")]) for i, (a, b) in enumerate(pairs)]

    left = mk([("S1", "S2"), ("S2", "S1"), ("S1", "S3"), ("S3", "S1")])
    mid = mk([("S5", "S6"), ("S6", "S5"), ("S5", "S7"), ("S7", "S5")])
    right = mk([("S5", "S6"), ("S6", "S5"), ("S7", "S7"), ("S7", "S5")])
    assert A.canonical(left) == A.canonical(mid)
    assert A.canonical(left) != A.canonical(right)
    assert A.store_pattern(left) == (((0, "R"), (1, "W")), ((1, "R"), (0, "W")),
                                     ((0, "R"), (2, "W")), ((2, "R"), (0, "W")))


# --- Soundness theorem (section 4.3), by brute force --------------------------

def _random_window(rng, n_tasks):
    stores = {"A": (4,), "B": (4,), "C": (4,), "D": (4,), "s": ()}
    parts = [Tiling((2,), (0,)), Tiling((1,), (0,)), Tiling((1,), (1,)),
             Tiling((2,), (0,), Proj((0,))), NoneP()]
    doms = [(2,), (4,), (2, 2)]
    win = []
    for _ in range(n_tasks):
        dom = rng.choice(doms[:2]) if rng.random() < 0.85 else (2, 2)
        args = []
        for _ in range(rng.randint(1, 3)):
            s = rng.choice(["A", "B", "C", "D", "s"])
            if s == "s":
                P, pr = NoneP(), rng.choice(["R", "Rd"])
            else:
                P = rng.choice(parts)
                if isinstance(P, Tiling) and P.proj.keep is not None and len(dom) != 2:
                    P = Tiling((1,), (0,))
                if isinstance(P, Tiling) and P.proj.keep is None and len(dom) == 2:
                    P = Tiling((2,), (0,), Proj((0,)))
                pr = rng.choice(["R", "W", "RW", "Rd"])
            args.append((s, P, pr))
        t = Task("op", dom, args)
        if A.legal(t, stores):
            win.append(t)
    return win, stores


def test_soundness_property_random_windows():
    rng = random.Random(1234)
    checked = 0
    for _ in range(400):
        win, shapes = _random_window(rng, rng.randint(2, 7))
        if not win:
            continue
        f = A.longest_prefix(win)
        assert f >= 1
        assert A.prefix_fusible(win[:f], shapes)
        checked += f
    assert checked > 400


def test_image_partition_dependence():
    # y = A x through Image(col): reading x via the gathered coordinates after
    # writing x through a Tiling is a cross-point dependence.
    data = {"col": np.array([0, 1, 1, 2, 3, 2, 3, 0])}
    shapes = {"x": (4,), "col": (8,), "y": (4,)}
    Tx = Tiling((2,), (0,))
    img = Image("col", Tiling((4,), (0,)))
    t1 = Task("w", (2,), [("x", Tx, "W")])
    t2 = Task("spmv", (2,), [("col", Tiling((4,), (0,)), "R"), ("x", img, "R"), ("y", Tx, "W")])
    assert not A.fusible(t1, t2, shapes, data)
    assert A.longest_prefix([t1, t2]) == 1  # Image != Tiling: the constraint breaks too


def test_legality_examples():
    shapes = {"C": (4,)}
    assert not A.legal(Task("op", (2,), [("C", NoneP(), "W")]), shapes)
    assert A.legal(Task("op", (1,), [("C", NoneP(), "W")]), shapes)
    assert A.legal(Task("op", (2,), [("C", NoneP(), "Rd")]), shapes)
    assert A.legal(Task("op", (2,), [("C", Tiling((2,), (0,)), "RW")]), shapes)
    assert not A.legal(Task("op", (2,), [("C", Tiling((2,), (0,)), "W"),
                                         ("C", Tiling((2,), (1,)), "R")]), shapes)
