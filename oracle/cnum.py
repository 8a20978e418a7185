"""ctypes loader for the oracle's plain C numerics (oracle/cnum.c).

Test infrastructure only.  `build()` compiles cnum.c with gcc at -O2 and
-ffp-contract=off, no fast-math; `lib()` loads it, building it first when the
shared object is missing or older than its source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cnum.c")
_SO = os.path.join(_HERE, "libcnum.so")
_lib = None


def build() -> str:
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-std=c99", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    L = ctypes.CDLL(_SO)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    i64 = ctypes.c_int64
    for name in ("or_log", "or_exp", "or_erf"):
        getattr(L, name).argtypes = [dp, dp, i64]
        getattr(L, name).restype = None
    L.or_pow.argtypes = [dp, dp, dp, i64]
    L.or_pow.restype = None
    L.or_spmv.argtypes = [i64, ip, ip, dp, dp, dp]
    L.or_spmv.restype = None
    L.or_fsum.argtypes = [dp, i64]
    L.or_fsum.restype = ctypes.c_double
    L.or_fsum_prod.argtypes = [dp, dp, i64]
    L.or_fsum_prod.restype = ctypes.c_double
    _lib = L
    return L


def _d(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _unary(name, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    getattr(lib(), name)(_d(x), _d(y), x.size)
    return y


def log(x):
    return _unary("or_log", x)


def exp(x):
    return _unary("or_exp", x)


def erf(x):
    return _unary("or_erf", x)


def power(x, e):
    x = np.ascontiguousarray(x, dtype=np.float64)
    e = np.ascontiguousarray(np.broadcast_to(e, x.shape), dtype=np.float64)
    y = np.empty_like(x)
    lib().or_pow(_d(x), _d(e), _d(y), x.size)
    return y


def spmv(rowptr, col, val, x):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = rowptr.size - 1
    y = np.empty(n, dtype=np.float64)
    lib().or_spmv(n, _i(rowptr), _i(col), _d(val), _d(x), _d(y))
    return y


def fsum(x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    return float(lib().or_fsum(_d(x), x.size))


def fsum_prod(x, y) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    y = np.ascontiguousarray(y, dtype=np.float64).ravel()
    assert x.size == y.size
    return float(lib().or_fsum_prod(_d(x), _d(y), x.size))
