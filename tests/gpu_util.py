"""Helpers shared by the GPU tests: contexts, uploads, tolerance checks."""
import sys

import numpy as np

import paper_2406_18109_amd as dfx
import synth
from oracle import workloads as wl


def note(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def ctx(fuse=True, window=64, memo=True):
    return dfx.Context(device=0, window_size=window, fuse=fuse, memo=memo)


def upload(c, arr, dtype=None):
    arr = np.asarray(arr)
    dt = dtype or {np.dtype(np.float64): "f64", np.dtype(np.float32): "f32",
                   np.dtype(np.int32): "i32", np.dtype(np.int64): "i64"}[arr.dtype]
    s = c.store_create(list(arr.shape), dt)
    c.store_write(s, arr)
    return s


def rel_err_floor(g, o):
    """max |g-o| / max(|o|, 1): the elementwise tolerance metric."""
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    if g.size == 0:
        return 0.0
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), 1.0)))


def rel_err(g, o):
    return abs(float(g) - float(o)) / max(abs(float(o)), 1e-300)


def bs_run(c, n, dtype="f64", passes=1, points=1):
    npdt = np.float64 if dtype == "f64" else np.float32
    S, K, T = synth.bs_inputs(n, npdt)
    # the oracle's own scalars; the device forms rv = r + sigma^2/2 itself
    r, sig, rv = wl.bs_scalars(synth.BS_RATE, synth.BS_VOL, npdt)
    hS, hK, hT = upload(c, S), upload(c, K), upload(c, T)
    hr, hs = (upload(c, np.array(v, dtype=npdt)) for v in (synth.BS_RATE, synth.BS_VOL))
    hv = dfx.apps.bs_drift(c, hr, hs, dtype)
    got_rv = float(c.store_read(hv, [], dtype))
    assert got_rv == rv, (got_rv, rv)
    c.stats_reset()
    out = None
    for _ in range(passes):
        if out:
            c.store_release(out[0])
            c.store_release(out[1])
        out = dfx.apps.black_scholes(c, hS, hK, hT, hr, hs, hv, n, dtype, points)
        c.flush()
    call = c.store_read(out[0], [n], dtype)
    put = c.store_read(out[1], [n], dtype)
    return (S, K, T, r, sig, rv), call, put
