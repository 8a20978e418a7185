"""The on-disk plan cache (host logic, analysis-only contexts): plans saved
from one context are found by another whose partition handles differ (keys
encode partitions by structure), give the same groups with no analysis, and
a damaged or missing file is rejected without touching the memo table."""
import os

import pytest

import paper_2406_18109_amd as dfx


def _streams(ctx, shift_handles=False):
    if shift_handles:
        # other partitions first, so every handle differs from the saving context
        ctx.part_tiling([7])
        ctx.part_tiling([3, 5])
        ctx.part_none()
    n = 1 << 10
    S, K, T = (ctx.store_create([n], "f64") for _ in range(3))
    r, sig, rv = (ctx.store_create([], "f64") for _ in range(3))
    dfx.apps.black_scholes(ctx, S, K, T, r, sig, rv, n, "f64", 1)
    ctx.flush()
    m = 64
    rp = ctx.store_create([m + 1], "i32")
    col = ctx.store_create([5 * m], "i32")
    val = ctx.store_create([5 * m], "f64")
    b = ctx.store_create([m], "f64")
    for cls in (dfx.apps.CG, dfx.apps.BiCGSTAB):
        s = cls(ctx, rp, col, val, b, m)
        for _ in range(3):
            s.iteration()
        ctx.flush()
    G = ctx.store_create([34, 34], "f64")
    J = dfx.apps.Jacobi(ctx, G, 34)
    for _ in range(3):
        J.sweep()
    ctx.flush()
    return [(g["prefix_len"], g["n_passes"], tuple(g["pass_kind"])) for g in ctx.groups()]


def test_saved_plans_serve_another_context(tmp_path):
    path = str(tmp_path / "plans.bin")
    a = dfx.Context(device=-1, window_size=16)
    ga = _streams(a)
    misses = a.stats()["memo_misses"]
    saved = a.plan_cache_save(path)
    assert saved == misses > 0
    b = dfx.Context(device=-1, window_size=16)
    assert b.plan_cache_load(path) == saved
    gb = _streams(b, shift_handles=True)
    st = b.stats()
    assert gb == ga
    assert st["memo_misses"] == 0 and st["memo_hits"] == len(gb)
    # loading again adds nothing (keys already present)
    assert b.plan_cache_load(path) == 0


def test_structurally_different_window_misses(tmp_path):
    path = str(tmp_path / "plans.bin")
    a = dfx.Context(device=-1, window_size=4)
    x, y = a.store_create([100], "f64"), a.store_create([100], "f64")
    a.submit("add", [1], [(x, a.part_tiling([100]), "R"), (y, a.part_tiling([100]), "R"), (y, a.part_tiling([100]), "W")])
    a.flush()
    a.plan_cache_save(path)
    b = dfx.Context(device=-1, window_size=4)
    b.plan_cache_load(path)
    x, y = b.store_create([100], "f64"), b.store_create([100], "f64")
    t = b.part_tiling([50])   # two points of 50: another partition and launch domain
    b.submit("add", [2], [(x, t, "R"), (y, t, "R"), (y, t, "W")])
    b.flush()
    assert b.stats()["memo_misses"] == 1


def test_damaged_and_missing_files_rejected(tmp_path):
    path = str(tmp_path / "plans.bin")
    a = dfx.Context(device=-1, window_size=16)
    _streams(a)
    a.plan_cache_save(path)
    data = open(path, "rb").read()
    bad = bytearray(data)
    bad[-9] ^= 0x40                      # a byte of the body: checksum mismatch
    cases = {"flip": bytes(bad), "trunc": data[:-3], "magic": b"XXXXXXXX" + data[8:]}
    for name, blob in cases.items():
        p = str(tmp_path / (name + ".bin"))
        open(p, "wb").write(blob)
        b = dfx.Context(device=-1, window_size=16)
        with pytest.raises(dfx.DfxError) as e:
            b.plan_cache_load(p)
        assert e.value.code == -1, name
        _streams(b)
        assert b.stats()["memo_misses"] > 0, name
    b = dfx.Context(device=-1, window_size=16)
    with pytest.raises(dfx.DfxError) as e:
        b.plan_cache_load(os.path.join(str(tmp_path), "absent.bin"))
    assert e.value.code == -8
    c = dfx.Context(device=-1, window_size=16, memo=False)
    with pytest.raises(dfx.DfxError) as e:
        c.plan_cache_load(path)
    assert e.value.code == -4
