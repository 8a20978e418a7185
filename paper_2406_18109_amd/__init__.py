"""dfx: fused execution of NumPy/SciPy-sparse-style task windows on AMD MI355X.

The compute path is libdfx.so (include/dfx.h): the fusion analysis of
"Composing Distributed Computations Through Task and Kernel Fusion" on the
host and hand-written gfx950 HIP kernels on the device.  `_binding` is the
ctypes layer with the C-ABI's names; `apps` issues the workloads' task
streams through it.
"""
from ._binding import Batch, Context, DfxError, jit_cache_dir, jit_info, jit_wait, lib  # noqa: F401
from . import apps  # noqa: F401
