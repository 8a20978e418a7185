"""ctypes binding of libdfx.so: the C-ABI calls with the same names, argument
marshalling only.  Every computation runs inside the library's kernels; this
module fails loudly when the library is missing.

PyTorch supplies device memory (its caching allocator, plugged in through the
allocation callbacks) and the HIP stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DFX_LIB names another build of the same library (the sanitizer build of
# the host code that the CPU tests use); by default the in-tree libdfx.so
LIB_PATH = os.environ.get("DFX_LIB") or os.path.join(_HERE, "libdfx.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE, ENOMEM_BUDGET, EBREAKDOWN, EMAXITER, ENOTFOUND, EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9
F32, F64, I32, I64 = 0, 1, 2, 3
R, W, RW, RD = 1, 2, 3, 4
PRIV = {"R": R, "W": W, "RW": RW, "Rd": RD, "RD": RD}
DTYPES = {"f32": F32, "f64": F64, "i32": I32, "i64": I64}
NP_DTYPE = {F32: np.float32, F64: np.float64, I32: np.int32, I64: np.int64}
OPS = {
    "neg": 1, "abs": 2, "sqrt": 3, "exp": 4, "log": 5, "erf": 6, "square": 7, "copy": 8,
    "add": 16, "sub": 17, "mul": 18, "div": 19, "pow": 20, "max": 21, "min": 22,
    "add_imm": 32, "sub_imm": 33, "rsub_imm": 34, "mul_imm": 35, "div_imm": 36, "rdiv_imm": 37,
    "fill": 48, "axpy": 49,
    "sum": 64, "sumsq": 65, "dot": 66,
    "spmv_csr": 80,
}
MAX_DIM = 4
INFO_MAX = 64

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class dfx_config(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("alloc", ALLOC_FN),
                ("dealloc", FREE_FN), ("alloc_user", C.c_void_p), ("window_size", C.c_int32),
                ("fuse", C.c_int32), ("memo", C.c_int32), ("tune", C.c_int32), ("auto_window", C.c_int32),
                ("jit", C.c_int32), ("reserved", C.c_int32 * 6)]


class dfx_arg(C.Structure):
    _fields_ = [("store", C.c_int64), ("part", C.c_int32), ("priv", C.c_int32)]


class dfx_task(C.Structure):
    _fields_ = [("op", C.c_uint32), ("ndim", C.c_int32), ("launch", C.POINTER(C.c_int64)),
                ("nargs", C.c_int32), ("args", C.POINTER(dfx_arg)), ("nimm", C.c_int32),
                ("imm", C.POINTER(C.c_double))]


class dfx_stats(C.Structure):
    _fields_ = [("tasks_submitted", C.c_int64), ("tasks_dispatched", C.c_int64),
                ("groups_dispatched", C.c_int64), ("launches", C.c_int64),
                ("temporaries_eliminated", C.c_int64), ("memo_hits", C.c_int64),
                ("memo_misses", C.c_int64), ("graph_replays", C.c_int64),
                ("alg_bytes", C.c_int64), ("analysis_seconds", C.c_double),
                ("compiled_launches", C.c_int64)]


class dfx_jit_info(C.Structure):
    _fields_ = [("compiled", C.c_int64), ("failed", C.c_int64), ("disk_hits", C.c_int64),
                ("pending", C.c_int32), ("reserved", C.c_int32), ("compile_seconds", C.c_double)]


class dfx_group_info(C.Structure):
    _fields_ = [("first_task", C.c_int64), ("prefix_len", C.c_int32), ("memo_hit", C.c_int32),
                ("n_passes", C.c_int32), ("pass_kind", C.c_int32 * 8), ("n_temporaries", C.c_int32),
                ("temporaries", C.c_int64 * INFO_MAX), ("alg_bytes", C.c_int64)]


class dfx_serve_cfg(C.Structure):
    _fields_ = [("hbm_budget", C.c_uint64), ("max_slots", C.c_int32), ("max_iter", C.c_int32),
                ("tol", C.c_double), ("iters_per_round", C.c_int32), ("reserved", C.c_int32 * 7)]


class dfx_csr_desc(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p)]


class dfx_solve_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("rel_residual", C.c_double),
                ("t_arrive", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


class dfx_serve_counters(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("rounds", C.c_int64), ("launches", C.c_int64), ("iterations", C.c_int64),
                ("row_updates", C.c_int64), ("peak_bytes", C.c_uint64), ("resident_bytes", C.c_uint64),
                ("queued", C.c_int64)]


SOLVE_QUEUED, SOLVE_RUNNING, SOLVE_CONVERGED, SOLVE_MAXITER, SOLVE_BREAKDOWN = 0, 1, 2, 3, 4

_lib = None

# name -> (restype, argtypes) for every exported call
SIGNATURES = {
    "dfx_version": (C.c_char_p, []),
    "dfx_last_error": (C.c_char_p, [C.c_void_p]),
    "dfx_create": (C.c_int, [C.POINTER(dfx_config), C.POINTER(C.c_void_p)]),
    "dfx_destroy": (C.c_int, [C.c_void_p]),
    "dfx_store_create": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int64)]),
    "dfx_store_wrap": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int64)]),
    "dfx_store_write": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_size_t]),
    "dfx_store_read": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_size_t]),
    "dfx_store_device_ptr": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_void_p)]),
    "dfx_store_release": (C.c_int, [C.c_void_p, C.c_int64]),
    "dfx_proj_identity": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "dfx_proj_drop": (C.c_int, [C.c_void_p, C.c_int32, C.c_uint32, C.POINTER(C.c_int32)]),
    "dfx_part_none": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "dfx_part_tiling": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32)]),
    "dfx_part_image": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.POINTER(C.c_int32)]),
    "dfx_submit": (C.c_int, [C.c_void_p, C.POINTER(dfx_task)]),
    "dfx_flush": (C.c_int, [C.c_void_p]),
    "dfx_flush_noalloc": (C.c_int, [C.c_void_p]),
    "dfx_sync": (C.c_int, [C.c_void_p]),
    "dfx_graph_begin": (C.c_int, [C.c_void_p]),
    "dfx_graph_end": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "dfx_graph_launch": (C.c_int, [C.c_void_p, C.c_int32]),
    "dfx_graph_destroy": (C.c_int, [C.c_void_p, C.c_int32]),
    "dfx_stats_get": (C.c_int, [C.c_void_p, C.POINTER(dfx_stats)]),
    "dfx_stats_reset": (C.c_int, [C.c_void_p]),
    "dfx_window_size": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "dfx_jit_wait": (C.c_int, []),
    "dfx_jit_info_get": (C.c_int, [C.POINTER(dfx_jit_info)]),
    "dfx_jit_cache_dir": (C.c_int, [C.c_char_p]),
    "dfx_jit_precompile": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "dfx_plan_cache_save": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_int64)]),
    "dfx_plan_cache_load": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_int64)]),
    "dfx_group_count": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "dfx_group_get": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(dfx_group_info)]),
    "dfx_serve_start": (C.c_int, [C.c_void_p, C.POINTER(dfx_serve_cfg)]),
    "dfx_serve_submit": (C.c_int, [C.c_void_p, C.POINTER(dfx_csr_desc), C.c_void_p, C.POINTER(C.c_uint64)]),
    "dfx_serve_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(dfx_solve_result)]),
    "dfx_serve_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.c_double, C.POINTER(dfx_solve_result)]),
    "dfx_serve_read_x": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_size_t]),
    "dfx_serve_release": (C.c_int, [C.c_void_p, C.c_uint64]),
    "dfx_serve_stats": (C.c_int, [C.c_void_p, C.POINTER(dfx_serve_counters)]),
    "dfx_serve_stop": (C.c_int, [C.c_void_p]),
    "dfx_batch_create": (C.c_int, [C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "dfx_batch_destroy": (C.c_int, [C.c_void_p]),
    "dfx_batch_last_error": (C.c_char_p, [C.c_void_p]),
    "dfx_batch_record_begin": (C.c_int, [C.c_void_p, C.c_void_p]),
    "dfx_batch_loop_begin": (C.c_int, [C.c_void_p, C.c_void_p]),
    "dfx_batch_record_end": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_double,
                                       C.POINTER(C.c_int32)]),
    "dfx_batch_run": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "dfx_batch_wait": (C.c_int, [C.c_void_p]),
    "dfx_batch_stream_info": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "dfx_batch_counts": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
}


def lib():
    """Load libdfx.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdfx.so is not built (run paper_2406_18109_amd.build.build()); "
                           "there is no fallback path")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def jit_wait():
    """Block until no pass kernel is queued or compiling (process-wide)."""
    lib().dfx_jit_wait()


def jit_info() -> dict:
    s = dfx_jit_info()
    rc = lib().dfx_jit_info_get(C.byref(s))
    if rc != 0:
        raise DfxError(rc, "dfx_jit_info_get failed")
    return {k: getattr(s, k) for k, _ in dfx_jit_info._fields_ if k != "reserved"}


def jit_cache_dir(path):
    """Directory of compiled code objects shared across processes (None: off)."""
    lib().dfx_jit_cache_dir(os.fsencode(path) if path else None)


class DfxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("dfx error %d: %s" % (code, msg))
        self.code = code


def _i64(seq):
    seq = list(seq)
    return (C.c_int64 * max(1, len(seq)))(*seq)


def _dt(dtype):
    if isinstance(dtype, int):
        return dtype
    if isinstance(dtype, str):
        return DTYPES[dtype]
    d = np.dtype(dtype)
    return {np.dtype(np.float32): F32, np.dtype(np.float64): F64,
            np.dtype(np.int32): I32, np.dtype(np.int64): I64}[d]


class _TorchAlloc:
    """Device memory from PyTorch's caching allocator."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device

        def alloc(nbytes, stream, user):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0)))
            except Exception:
                return None

        def free(ptr, nbytes, stream, user):
            torch.cuda.caching_allocator_delete(int(ptr))

        self.alloc_fn = ALLOC_FN(alloc)
        self.free_fn = FREE_FN(free)


class Context:
    """One dfx context (dfx_create ... dfx_destroy)."""

    def __init__(self, device: int = 0, window_size: int = 16, fuse: bool = True, memo: bool = True,
                 stream=None, allocator: str = "torch", tune: bool = False, auto_window: int = 0, jit: int = 0):
        self.L = lib()
        cfg = dfx_config()
        cfg.device = device
        cfg.window_size = window_size
        cfg.fuse = 1 if fuse else 0
        cfg.memo = 1 if memo else 0
        cfg.tune = 1 if tune else 0
        cfg.auto_window = auto_window
        cfg.jit = int(jit)
        self._alloc = None
        self.torch_stream = None
        if device >= 0:
            import torch
            if stream is None:
                self.torch_stream = torch.cuda.Stream(device=device)
                stream = self.torch_stream.cuda_stream
            cfg.stream = C.c_void_p(int(stream))
            if allocator == "torch":
                self._alloc = _TorchAlloc(device)
                cfg.alloc = self._alloc.alloc_fn
                cfg.dealloc = self._alloc.free_fn
        h = C.c_void_p()
        rc = self.L.dfx_create(C.byref(cfg), C.byref(h))
        if rc != 0:
            raise DfxError(rc, "dfx_create failed")
        self.h = h
        self.device = device

    # -- helpers ------------------------------------------------------------
    def _chk(self, rc):
        if rc != 0:
            raise DfxError(rc, self.L.dfx_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            rc = self.L.dfx_destroy(self.h)
            self.h = None
            if rc != 0:
                raise DfxError(rc, "dfx_destroy failed")

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.L.dfx_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # -- stores --------------------------------------------------------------
    def store_create(self, shape, dtype="f64") -> int:
        out = C.c_int64()
        self._chk(self.L.dfx_store_create(self.h, len(shape), _i64(shape), _dt(dtype), C.byref(out)))
        return out.value

    def store_wrap(self, dptr: int, shape, dtype) -> int:
        out = C.c_int64()
        self._chk(self.L.dfx_store_wrap(self.h, C.c_void_p(dptr), len(shape), _i64(shape), _dt(dtype), C.byref(out)))
        return out.value

    def store_write(self, s: int, arr: np.ndarray):
        a = np.ascontiguousarray(arr)
        self._chk(self.L.dfx_store_write(self.h, s, a.ctypes.data_as(C.c_void_p), a.nbytes))

    def store_read(self, s: int, shape, dtype) -> np.ndarray:
        out = np.empty(shape, dtype=NP_DTYPE[_dt(dtype)])
        self._chk(self.L.dfx_store_read(self.h, s, out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out

    def store_device_ptr(self, s: int) -> int:
        p = C.c_void_p()
        self._chk(self.L.dfx_store_device_ptr(self.h, s, C.byref(p)))
        return p.value or 0

    def store_release(self, s: int):
        self._chk(self.L.dfx_store_release(self.h, s))

    # -- projections / partitions ---------------------------------------------
    def proj_identity(self, ndim: int) -> int:
        out = C.c_int32()
        self._chk(self.L.dfx_proj_identity(self.h, ndim, C.byref(out)))
        return out.value

    def proj_drop(self, ndim_in: int, keep_mask: int) -> int:
        out = C.c_int32()
        self._chk(self.L.dfx_proj_drop(self.h, ndim_in, keep_mask, C.byref(out)))
        return out.value

    def part_none(self) -> int:
        out = C.c_int32()
        self._chk(self.L.dfx_part_none(self.h, C.byref(out)))
        return out.value

    def part_tiling(self, tile, offset=None, proj=None) -> int:
        if offset is None:
            offset = [0] * len(tile)
        if proj is None:
            proj = self.proj_identity(len(tile))
        out = C.c_int32()
        self._chk(self.L.dfx_part_tiling(self.h, len(tile), _i64(tile), _i64(offset), proj, C.byref(out)))
        return out.value

    def part_image(self, src: int, src_part: int) -> int:
        out = C.c_int32()
        self._chk(self.L.dfx_part_image(self.h, src, src_part, C.byref(out)))
        return out.value

    # -- tasks ---------------------------------------------------------------
    def submit(self, op, launch, args, imm=()):
        """args: [(store, part, priv)] with priv in R/W/RW/Rd (int or name)."""
        opc = OPS[op] if isinstance(op, str) else int(op)
        A = (dfx_arg * max(1, len(args)))()
        for i, (s, p, pr) in enumerate(args):
            A[i].store = s
            A[i].part = p
            A[i].priv = PRIV[pr] if isinstance(pr, str) else int(pr)
        imm = list(imm)
        Im = (C.c_double * max(1, len(imm)))(*imm)
        t = dfx_task(opc, len(launch), _i64(launch), len(args), A, len(imm), Im)
        self._chk(self.L.dfx_submit(self.h, C.byref(t)))

    def flush(self):
        self._chk(self.L.dfx_flush(self.h))

    def flush_noalloc(self):
        self._chk(self.L.dfx_flush_noalloc(self.h))

    def sync(self):
        self._chk(self.L.dfx_sync(self.h))

    # -- graphs ---------------------------------------------------------------
    def graph_begin(self):
        self._chk(self.L.dfx_graph_begin(self.h))

    def graph_end(self) -> int:
        g = C.c_int32()
        self._chk(self.L.dfx_graph_end(self.h, C.byref(g)))
        return g.value

    def graph_launch(self, g: int):
        self._chk(self.L.dfx_graph_launch(self.h, g))

    def graph_destroy(self, g: int):
        self._chk(self.L.dfx_graph_destroy(self.h, g))

    # -- introspection ----------------------------------------------------------
    def stats(self) -> dict:
        s = dfx_stats()
        self._chk(self.L.dfx_stats_get(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in dfx_stats._fields_}

    def stats_reset(self):
        self._chk(self.L.dfx_stats_reset(self.h))

    # -- serving ------------------------------------------------------------------
    def serve_start(self, hbm_budget: int, max_slots: int = 256, tol: float = 1e-8, max_iter: int = 100000,
                    iters_per_round: int = 0):
        cfg = dfx_serve_cfg(hbm_budget, max_slots, max_iter, tol, iters_per_round)
        self._chk(self.L.dfx_serve_start(self.h, C.byref(cfg)))
        self._serve_keep = {}

    def serve_submit(self, rowptr, col, val, b) -> int:
        """Queue one CG solve; the CSR arrays are kept referenced until admission."""
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        n = rowptr.size - 1
        d = dfx_csr_desc(n, col.size, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data)
        t = C.c_uint64()
        self._chk(self.L.dfx_serve_submit(self.h, C.byref(d), b.ctypes.data, C.byref(t)))
        self._serve_keep[t.value] = (rowptr, col, val)
        return t.value

    @staticmethod
    def _res(r):
        return {"status": r.status, "iterations": r.iterations, "rel_residual": r.rel_residual,
                "t_arrive": r.t_arrive, "t_admit": r.t_admit, "t_done": r.t_done}

    def serve_poll(self, ticket: int) -> dict:
        r = dfx_solve_result()
        self._chk(self.L.dfx_serve_poll(self.h, ticket, C.byref(r)))
        if r.status != SOLVE_QUEUED:
            self._serve_keep.pop(ticket, None)
        return self._res(r)

    def serve_wait(self, ticket: int, timeout: float = 600.0) -> dict:
        r = dfx_solve_result()
        self._chk(self.L.dfx_serve_wait(self.h, ticket, timeout, C.byref(r)))
        self._serve_keep.pop(ticket, None)
        return self._res(r)

    def serve_read_x(self, ticket: int, n: int) -> np.ndarray:
        x = np.empty(n, dtype=np.float64)
        self._chk(self.L.dfx_serve_read_x(self.h, ticket, x.ctypes.data, n))
        return x

    def serve_release(self, ticket: int):
        self._chk(self.L.dfx_serve_release(self.h, ticket))

    def serve_stats(self) -> dict:
        s = dfx_serve_counters()
        self._chk(self.L.dfx_serve_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in dfx_serve_counters._fields_}

    def serve_stop(self):
        self._chk(self.L.dfx_serve_stop(self.h))
        self._serve_keep = {}

    def plan_cache_save(self, path) -> int:
        n = C.c_int64()
        self._chk(self.L.dfx_plan_cache_save(self.h, os.fsencode(path), C.byref(n)))
        return n.value

    def plan_cache_load(self, path) -> int:
        n = C.c_int64()
        self._chk(self.L.dfx_plan_cache_load(self.h, os.fsencode(path), C.byref(n)))
        return n.value

    def jit_precompile(self) -> int:
        """Compile every memoised pass's kernel now; returns how many failed."""
        n = C.c_int64()
        self._chk(self.L.dfx_jit_precompile(self.h, C.byref(n)))
        return n.value

    def window_size(self) -> int:
        n = C.c_int32()
        self._chk(self.L.dfx_window_size(self.h, C.byref(n)))
        return n.value

    def groups(self) -> list:
        n = C.c_int64()
        self._chk(self.L.dfx_group_count(self.h, C.byref(n)))
        out = []
        gi = dfx_group_info()
        for i in range(n.value):
            self._chk(self.L.dfx_group_get(self.h, i, C.byref(gi)))
            out.append({"first_task": gi.first_task, "prefix_len": gi.prefix_len,
                        "memo_hit": bool(gi.memo_hit), "n_passes": gi.n_passes,
                        "pass_kind": list(gi.pass_kind[:gi.n_passes]),
                        "temporaries": sorted(gi.temporaries[:gi.n_temporaries]),
                        "alg_bytes": gi.alg_bytes})
        return out


class Batch:
    """A batch of independent task streams run in one persistent launch
    (dfx_batch_*): each stream is what one context dispatches between
    record_begin and record_end."""

    RUNNING, DONE, PAUSED = 0, 1, 2

    def __init__(self, device: int = 0, stream=None):
        self.L = lib()
        self.torch_stream = None
        if stream is None:
            import torch
            self.torch_stream = torch.cuda.Stream(device=device)
            stream = self.torch_stream.cuda_stream
        h = C.c_void_p()
        rc = self.L.dfx_batch_create(device, C.c_void_p(int(stream)), C.byref(h))
        if rc != 0:
            raise DfxError(rc, "dfx_batch_create failed")
        self.h = h

    def _chk(self, rc):
        if rc != 0:
            raise DfxError(rc, self.L.dfx_batch_last_error(self.h).decode())
        return rc

    def record_begin(self, ctx: Context):
        self._chk(self.L.dfx_batch_record_begin(self.h, ctx.h))

    def loop_begin(self, ctx: Context):
        self._chk(self.L.dfx_batch_loop_begin(self.h, ctx.h))

    def record_end(self, ctx: Context, max_iter: int = 0, conv_a: int = 0, conv_b: int = 0, tol: float = 0.0) -> int:
        sid = C.c_int32()
        self._chk(self.L.dfx_batch_record_end(self.h, ctx.h, max_iter, conv_a, conv_b, tol, C.byref(sid)))
        return sid.value

    def run(self, round_limit: int = 0, restart: bool = True):
        self._chk(self.L.dfx_batch_run(self.h, round_limit, 1 if restart else 0))

    def wait(self):
        self._chk(self.L.dfx_batch_wait(self.h))

    def stream_info(self, sid: int):
        it, st = C.c_int32(), C.c_int32()
        self._chk(self.L.dfx_batch_stream_info(self.h, sid, C.byref(it), C.byref(st)))
        return it.value, st.value

    def counts(self):
        a, b, g = C.c_int32(), C.c_int32(), C.c_int32()
        self._chk(self.L.dfx_batch_counts(self.h, C.byref(a), C.byref(b), C.byref(g)))
        return {"streams": a.value, "passes": b.value, "grid": g.value}

    def close(self):
        if getattr(self, "h", None):
            self.L.dfx_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
