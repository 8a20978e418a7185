"""The library's fusion analysis (through the C ABI, analysis-only context)
against the oracle's definitional analysis and the paper's worked examples."""
import random
import re
import os

import numpy as np
import pytest

import paper_2406_18109_amd as dfx
from paper_2406_18109_amd import _binding as B
from oracle import analysis as OA
from oracle.ir import NoneP, Proj, Task, Tiling

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "dfx.h")).read()
    declared = set(re.findall(r"^\s*(?:int|const char\*)\s+(dfx_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 26
    L = dfx.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert set(B.SIGNATURES) == declared


class Mirror:
    """Issue the same window to the library and keep it as oracle IR."""

    def __init__(self, window_size=64, fuse=True, memo=True):
        self.ctx = dfx.Context(device=-1, window_size=window_size, fuse=fuse, memo=memo)
        self.ids = {}
        self.names = {}
        self.shapes = {}
        self.tasks = []
        self._parts = {}

    def store(self, name, shape):
        s = self.ctx.store_create(list(shape), "f64")
        self.ids[name] = s
        self.names[s] = name
        self.shapes[name] = tuple(shape)
        return s

    def part(self, P):
        if P in self._parts:
            return self._parts[P]
        if isinstance(P, NoneP):
            h = self.ctx.part_none()
        else:
            if P.proj.keep is None:
                pj = self.ctx.proj_identity(len(P.tile))
                h = self.ctx.part_tiling(list(P.tile), list(P.offset), pj)
            else:
                raise NotImplementedError
        self._parts[P] = h
        return h

    def submit(self, t: Task):
        self.tasks.append(t)
        self.ctx.submit(t.op, list(t.domain), [(self.ids[s], self.part(P), pr) for (s, P, pr) in t.args],
                        t.imm)

    def release(self, name):
        self.ctx.store_release(self.ids[name])


def oracle_groups(tasks, shapes, app_live):
    out = []
    w = list(tasks)
    while w:
        f = OA.longest_prefix(w)
        temps = OA.temporaries(w, f, app_live, shapes)
        out.append((f, temps))
        w = w[f:]
    return out


def lib_groups(m: Mirror):
    return [(g["prefix_len"], {m.names[s] for s in g["temporaries"]}) for g in m.ctx.groups()]


def test_figure1_stencil_stream():
    from test_oracle_jacobi import stencil_tasks
    N = 6
    m = Mirror(window_size=64)
    m.store("grid", (N, N))
    for k in ("t1", "t2", "t3", "avg", "work", "d"):
        m.store(k, (N - 2, N - 2))
    m.store("ss", ())
    tasks = stencil_tasks(N, (2, 2), with_residual=False)
    for t in tasks:
        m.submit(t)
    for k in ("t1", "t2", "t3", "avg"):
        m.release(k)
    m.ctx.flush()
    got = lib_groups(m)
    assert got == [(5, {"t1", "t2", "t3", "avg"}), (1, set())]
    assert got == oracle_groups(tasks, m.shapes, app_live={"grid", "work", "d", "ss"})


def test_figure5_temporaries_stream():
    m = Mirror(window_size=64)
    for k in "xyzwv":
        m.store(k, (8,))
    m.store("norm", ())
    T = Tiling((4,), (0,))
    half = Tiling((2,), (4,))
    d = (2,)
    tasks = [
        Task("mul_imm", d, [("x", T, "R"), ("z", T, "W")], (2.0,)),
        Task("add", d, [("y", T, "R"), ("z", T, "R"), ("w", T, "W")]),
        Task("square", d, [("w", T, "R"), ("v", T, "W")]),
        Task("sumsq", d, [("w", half, "R"), ("norm", NoneP(), "Rd")], (1,)),
    ]
    for t in tasks:
        m.submit(t)
    for k in "xyzw":
        m.release(k)
    m.ctx.flush()
    got = lib_groups(m)
    assert got[0] == (3, {"z"})
    assert got == oracle_groups(tasks, m.shapes, app_live={"v", "norm"})


def test_black_scholes_stream_fuses_to_one_group():
    ctx = dfx.Context(device=-1, window_size=64)
    n = 1 << 12
    S, K, T = (ctx.store_create([n], "f64") for _ in range(3))
    r, sig, rv = (ctx.store_create([], "f64") for _ in range(3))
    call, put = dfx.apps.black_scholes(ctx, S, K, T, r, sig, rv, n)
    ctx.flush()
    g = ctx.groups()
    assert len(g) == 1 and g[0]["prefix_len"] == len(dfx.apps.BS_STREAM) == 28
    assert len(g[0]["temporaries"]) == 26
    assert g[0]["n_passes"] == 1
    # 3 inputs + 2 outputs, 8 bytes each (plus the three 8-byte broadcasts)
    assert g[0]["alg_bytes"] == 5 * 8 * n + 3 * 8
    # a second, isomorphic pass hits the memo table
    call2, put2 = dfx.apps.black_scholes(ctx, S, K, T, r, sig, rv, n)
    ctx.flush()
    g = ctx.groups()
    assert g[1]["memo_hit"] and g[1]["prefix_len"] == 28


def test_black_scholes_unfused_materialises_everything():
    ctx = dfx.Context(device=-1, window_size=64, fuse=False)
    n = 1 << 10
    S, K, T = (ctx.store_create([n], "f64") for _ in range(3))
    r, sig, rv = (ctx.store_create([], "f64") for _ in range(3))
    dfx.apps.black_scholes(ctx, S, K, T, r, sig, rv, n)
    ctx.flush()
    g = ctx.groups()
    assert [x["prefix_len"] for x in g] == [1] * 28
    assert all(not x["temporaries"] for x in g)


def test_jacobi_windows_and_temporaries():
    ctx = dfx.Context(device=-1, window_size=16)
    N = 34
    grid = ctx.store_create([N, N], "f64")
    J = dfx.apps.Jacobi(ctx, grid, N)
    for _ in range(6):
        J.sweep()
    ctx.flush()
    g = ctx.groups()
    lens = [x["prefix_len"] for x in g]
    # per sweep: the fused stencil+residual (7 tasks), COPY alone, sqrt alone
    assert lens == [7, 1, 1] * 6
    fused = g[0]
    assert len(fused["temporaries"]) == 5   # t1, t2, t3, avg, d
    # the steady state replays a memoised analysis
    assert sum(x["memo_hit"] for x in g) >= 9
    # fused pass: grid read once (N*N minus 4 corners) + work written
    assert fused["alg_bytes"] == 8 * (N * N - 4) + 8 * (N - 2) ** 2 + 2 * 8


def test_cg_windows():
    ctx = dfx.Context(device=-1, window_size=16)
    n = 64
    rp = ctx.store_create([n + 1], "i32")
    col = ctx.store_create([5 * n], "i32")
    val = ctx.store_create([5 * n], "f64")
    b = ctx.store_create([n], "f64")
    cg = dfx.apps.CG(ctx, rp, col, val, b, n)
    for _ in range(4):
        cg.iteration()
    ctx.flush()
    lens = [x["prefix_len"] for x in ctx.groups()]
    # setup (fill, copy, copy, dot), then per iteration
    # [spmv, dot] [alpha] [axpy, axpy, dot] [beta, rho] [scale, axpy]
    assert lens[0] == 4
    assert lens[1:] == [2, 1, 3, 2, 2] * 4
    kinds = [x["pass_kind"] for x in ctx.groups()][1:6]
    assert kinds == [[1], [2], [0], [2], [0]]


def test_bicgstab_windows():
    ctx = dfx.Context(device=-1, window_size=16)
    n = 64
    rp = ctx.store_create([n + 1], "i32")
    col = ctx.store_create([5 * n], "i32")
    val = ctx.store_create([5 * n], "f64")
    b = ctx.store_create([n], "f64")
    bi = dfx.apps.BiCGSTAB(ctx, rp, col, val, b, n)
    ctx.flush()
    g0 = len(ctx.groups())
    for _ in range(4):
        bi.iteration()
    ctx.flush()
    g = ctx.groups()[g0:]
    lens = [x["prefix_len"] for x in g]
    # 22 tasks per iteration in 8 groups:
    # [beta's two divides and product, rho <- rho'] [p - omega v, * beta, + r]
    # [spmv, r^.v] [alpha] [s = r - alpha v (copy, axpy)] [spmv, t.s, t.t] [omega]
    # [x += alpha p, x += omega s, r = s - omega t (copy, axpy), r.r, next rho' = r^.r]
    assert lens == [4, 3, 2, 1, 2, 3, 1, 6] * 4
    assert [x["pass_kind"] for x in g[:8]] == [[2], [0], [1], [2], [0], [1], [2], [0]]
    # beta's two quotients are temporaries of the scalar window
    assert len(g[0]["temporaries"]) == 2


def _bs_groups(window, auto):
    ctx = dfx.Context(device=-1, window_size=window, auto_window=auto)
    n = 1 << 10
    S, K, T = (ctx.store_create([n], "f64") for _ in range(3))
    r, sig, rv = (ctx.store_create([], "f64") for _ in range(3))
    dfx.apps.black_scholes(ctx, S, K, T, r, sig, rv, n, "f64", 1)
    ctx.flush()
    return [g["prefix_len"] for g in ctx.groups()], ctx.window_size()


def _solver_groups(cls, window, auto, iters=6):
    ctx = dfx.Context(device=-1, window_size=window, auto_window=auto)
    n = 64
    rp = ctx.store_create([n + 1], "i32")
    col = ctx.store_create([5 * n], "i32")
    val = ctx.store_create([5 * n], "f64")
    b = ctx.store_create([n], "f64")
    s = cls(ctx, rp, col, val, b, n)
    for _ in range(iters):
        s.iteration()
    ctx.flush()
    return [g["prefix_len"] for g in ctx.groups()], ctx.window_size()


def test_auto_window_grows_while_everything_fuses():
    """Automatic window sizing (the evaluation's choice of window sizes): a
    full window that fuses as a whole doubles instead of being dispatched."""
    lens, w = _bs_groups(2, 0)
    assert lens == [2] * 14 and w == 2
    lens, w = _bs_groups(2, 64)
    assert lens == [28] and w == 32          # 2 -> 4 -> 8 -> 16 -> 32, then the flush
    lens, w = _bs_groups(2, 16)
    # capped at 16: a full window of 16 fuses as a whole, but with the
    # application still naming most intermediates the group needs more
    # output streams than a kernel has, so its longest prefix that lowers
    # (6 tasks) is dispatched; the flush takes the last 10 at once
    assert lens == [6, 6, 6, 10] and w == 16
    assert _bs_groups(16, 0) == ([6, 6, 6, 10], 16)
    for cls in (dfx.apps.CG, dfx.apps.BiCGSTAB):
        fixed, _ = _solver_groups(cls, 16, 0)
        auto, w = _solver_groups(cls, 1, 64)
        assert auto == fixed and w == 8, cls.__name__


def test_auto_window_jacobi_matches_fixed():
    def run(window, auto):
        ctx = dfx.Context(device=-1, window_size=window, auto_window=auto)
        G = ctx.store_create([34, 34], "f64")
        J = dfx.apps.Jacobi(ctx, G, 34)
        for _ in range(5):
            J.sweep()
        ctx.flush()
        return [g["prefix_len"] for g in ctx.groups()], ctx.window_size()
    fixed, _ = run(16, 0)
    auto, w = run(1, 256)
    assert auto == fixed and w <= 16


def test_auto_window_config_checked():
    for kw in (dict(window_size=8, auto_window=4), dict(window_size=1, auto_window=-1),
               dict(window_size=1, auto_window=8, fuse=False)):
        with pytest.raises(dfx.DfxError):
            dfx.Context(device=-1, **kw)


def test_validation_rejects_illegal_tasks_and_keeps_window():
    ctx = dfx.Context(device=-1, window_size=64)
    a = ctx.store_create([8], "f64")
    b = ctx.store_create([8], "f64")
    s = ctx.store_create([], "f64")
    T = ctx.part_tiling([4])
    N = ctx.part_none()
    ctx.submit("add", [2], [(a, T, "R"), (a, T, "R"), (b, T, "W")])
    with pytest.raises(B.DfxError) as e:
        ctx.submit("add", [2], [(a, T, "R"), (b, T, "R")])    # arity
    assert e.value.code == B.EINVAL
    with pytest.raises(B.DfxError):
        ctx.submit("copy", [2], [(a, T, "R"), (s, N, "W")])  # writing None from 2 points
    with pytest.raises(B.DfxError):
        ctx.submit("copy", [3], [(a, T, "R"), (b, T, "W")])  # tiles leave the store
    with pytest.raises(B.DfxError):
        ctx.submit("copy", [2], [(a, T, "W"), (b, T, "W")])  # privilege of input
    T2 = ctx.part_tiling([4], [4])
    with pytest.raises(B.DfxError):
        ctx.submit("add", [1], [(a, T2, "R"), (a, T, "R"), (a, T, "W")])  # writes an aliased view
    i = ctx.store_create([8], "i32")
    with pytest.raises(B.DfxError):
        ctx.submit("neg", [2], [(i, T, "R"), (b, T, "W")])   # integer elementwise
    assert ctx.stats()["tasks_submitted"] == 1
    ctx.flush()
    assert [g["prefix_len"] for g in ctx.groups()] == [1]


def _random_abi_window(rng):
    shapes = {"A": (4,), "B": (4,), "C": (4,), "D": (4,), "s": (), "u": ()}
    parts = [Tiling((2,), (0,)), Tiling((1,), (0,)), Tiling((1,), (1,)), Tiling((1,), (2,))]
    win = []
    for _ in range(rng.randint(2, 9)):
        dom = rng.choice([(2,), (4,), (1,)])
        kind = rng.random()
        if kind < 0.15:
            # single task on scalars
            a, o = rng.sample(["s", "u"], 2)
            win.append(Task("neg", (), [(a, NoneP(), "R"), (o, NoneP(), "W")]))
            continue
        tiles = [p for p in parts if p.tile[0] * dom[0] + p.offset[0] <= 4]
        P = rng.choice(tiles)
        Ps = [p for p in tiles if p.tile == P.tile]
        ins = [(rng.choice("ABCD"), rng.choice(Ps), "R") for _ in range(rng.randint(1, 2))]
        if kind < 0.3:
            win.append(Task("sum", dom, [ins[0], (rng.choice("su"), NoneP(), "Rd")], (0,)))
            continue
        out = (rng.choice("ABCD"), P, "W")
        ok = all(not (s == out[0] and p != out[1]) for (s, p, _) in ins)
        if not ok:
            continue
        if len(ins) == 1:
            win.append(Task("neg", dom, ins + [out]))
        else:
            win.append(Task("add", dom, ins + [out]))
    return win, shapes


def test_analysis_matches_oracle_on_random_windows():
    rng = random.Random(99)
    compared = 0
    for trial in range(250):
        win, shapes = _random_abi_window(rng)
        m = Mirror(window_size=1000)
        for k, sh in shapes.items():
            m.store(k, sh)
        legal = []
        for t in win:
            if not OA.legal(t, shapes):
                continue
            try:
                m.submit(t)
            except B.DfxError:
                continue
            legal.append(t)
        if not legal:
            continue
        dropped = set(rng.sample(sorted(shapes), rng.randint(0, 3)))
        for k in dropped:
            m.release(k)
        m.ctx.flush()
        got = lib_groups(m)
        exp = oracle_groups(legal, shapes, app_live=set(shapes) - dropped)
        assert got == exp, (trial, legal)
        # soundness: every dispatched group is brute-force fusible
        pos = 0
        for f, _ in got:
            assert OA.prefix_fusible(legal[pos:pos + f], shapes)
            pos += f
        compared += len(got)
    assert compared > 300


def test_memo_isomorphic_streams_share_plans():
    """Figure 6: isomorphic streams reuse the analysis, a differing one does not."""
    ctx = dfx.Context(device=-1, window_size=4)
    T = ctx.part_tiling([4])
    S = {k: ctx.store_create([4], "f64") for k in ("S1", "S2", "S3", "S5", "S6", "S7")}

    def issue(pairs):
        for a, b in pairs:
            ctx.submit("neg", [1], [(S[a], T, "R"), (S[b], T, "W")])
        ctx.flush()

    issue([("S1", "S2"), ("S2", "S1"), ("S1", "S3"), ("S3", "S1")])
    n0 = ctx.stats()["memo_misses"]
    issue([("S5", "S6"), ("S6", "S5"), ("S5", "S7"), ("S7", "S5")])
    assert ctx.stats()["memo_misses"] == n0   # all hits
    issue([("S5", "S6"), ("S6", "S5"), ("S7", "S7"), ("S7", "S5")])
    assert ctx.stats()["memo_misses"] > n0
