"""Compiled passes, host side (no GPU): the kernel of every pass of the
Black-Scholes (FP64 and FP32), CG, BiCGSTAB, Jacobi (stencil-staged) and GMG
streams is generated and compiled by hiprtc for gfx950 in an analysis-only
context; one program instantiated for two element types gives two kernels;
the on-disk cache serves a second process without compiling and rejects a
damaged file."""
import json
import os
import subprocess
import sys

import paper_2406_18109_amd as dfx

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

_CHILD = r"""
import json, sys
sys.path.insert(0, %(root)r)
sys.path.insert(0, %(tests)r)
import paper_2406_18109_amd as dfx
import test_jit_compile as T
if %(cache)r:
    dfx.jit_cache_dir(%(cache)r)
c = dfx.Context(device=-1, window_size=16)
getattr(T, %(fn)r)(c)
failed = c.jit_precompile()
print(json.dumps({"failed": failed, **dfx.jit_info()}))
"""


def _child(fn, cache=""):
    code = _CHILD % {"root": ROOT, "tests": HERE, "cache": cache, "fn": fn}
    env = dict(os.environ)
    env.pop("DFX_JIT_CACHE", None)
    env["DFX_JIT_ALL"] = "1"
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def _bs(c, dtype, n=1 << 12):
    S, K, T = (c.store_create([n], dtype) for _ in range(3))
    r, sig, rv = (c.store_create([], dtype) for _ in range(3))
    dfx.apps.black_scholes(c, S, K, T, r, sig, rv, n, dtype, 1)
    c.flush()


def small_streams(c):
    """Black-Scholes FP64 and a CG iteration."""
    _bs(c, "f64")
    m = 64
    rp, col = c.store_create([m + 1], "i32"), c.store_create([5 * m], "i32")
    val, b = c.store_create([5 * m], "f64"), c.store_create([m], "f64")
    cg = dfx.apps.CG(c, rp, col, val, b, m)
    cg.iteration()
    c.flush()


def spmv_two_dtypes(c):
    """The same SpMV-only pass (an empty op list) in FP64 and in FP32."""
    for dt in ("f64", "f32"):
        n = 1000
        hr, hc = c.store_create([n + 1], "i32"), c.store_create([5 * n], "i32")
        hv, hx, hy = c.store_create([5 * n], dt), c.store_create([n], dt), c.store_create([n], dt)
        N, T = c.part_none(), c.part_tiling([n])
        c.submit("spmv_csr", [1], [(hr, N, "R"), (hc, N, "R"), (hv, N, "R"), (hx, c.part_image(hc, N), "R"),
                                   (hy, T, "W")])
        c.flush()


def all_streams(c):
    """Black-Scholes (FP64 and FP32), CG, BiCGSTAB, Jacobi and one GMG
    iteration over 3 levels."""
    from test_plan_cache import _streams
    _streams(c)
    _bs(c, "f32")
    import synth
    m, nlev = 15, 3

    def st(a):
        return c.store_create(list(a.shape), "i32" if a.dtype.kind == "i" else "f64")
    lev = [(tuple(st(a) for a in A), diag, None if R is None else tuple(st(a) for a in R),
            None if P is None else tuple(st(a) for a in P)) for A, diag, R, P in synth.gmg_levels(m, nlev)]
    sizes = [A[0].size - 1 for A, _, _, _ in synth.gmg_levels(m, nlev)]
    g = dfx.apps.GMG(c, lev, sizes, c.store_create([m * m], "f64"))
    g.iteration()
    c.flush()


def test_every_pass_compiles(monkeypatch):
    monkeypatch.setenv("DFX_JIT_ALL", "1")
    c = dfx.Context(device=-1, window_size=16)
    all_streams(c)
    before = dfx.jit_info()
    assert c.jit_precompile() == 0
    after = dfx.jit_info()
    assert after["failed"] == before["failed"]
    assert after["compiled"] + after["disk_hits"] > before["compiled"] + before["disk_hits"]
    # a second precompile finds every kernel in the process's cache
    assert c.jit_precompile() == 0
    assert dfx.jit_info()["compiled"] == after["compiled"]
    c.close()


def test_one_program_two_dtypes_two_kernels():
    r = _child("spmv_two_dtypes")
    assert r["failed"] == 0 and r["compiled"] == 2


def test_disk_cache_serves_another_process(tmp_path):
    cache = str(tmp_path)
    first = _child("small_streams", cache)
    second = _child("small_streams", cache)
    assert first["failed"] == 0 and second["failed"] == 0
    assert first["compiled"] > 0 and first["disk_hits"] == 0
    assert second["compiled"] == 0 and second["disk_hits"] == first["compiled"]
    files = sorted(f for f in os.listdir(cache) if f.endswith(".co"))
    assert len(files) == first["compiled"]
    # a file whose key or code bytes are damaged is compiled again
    for where in (9, -12):
        path = os.path.join(cache, files[0])
        data = bytearray(open(path, "rb").read())
        data[where] ^= 0xFF
        open(path, "wb").write(bytes(data))
        again = _child("small_streams", cache)
        assert again["failed"] == 0 and again["compiled"] == 1
        assert again["disk_hits"] == first["compiled"] - 1
