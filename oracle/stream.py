"""Unfused, op-by-op FP64 evaluation of a task stream (the meaning of the stream).

Test infrastructure only.  Each index task runs as its point tasks, one
point at a time, each on its sub-stores (section 3.2, computational model),
and every store -- temporaries included -- is a materialised array.  This is
the stream's plain definition: what any fused execution must reproduce up to
rounding order.

Arithmetic: + - * / sqrt neg abs max min are single IEEE double operations
(numpy float64); log, exp, erf and pow call the host C library element by
element (oracle/cnum.c); reductions are exactly rounded sums (cnum.fsum), and
dot products sum the rounded products x_i*y_i exactly rounded; a reduction
with the init flag set stores the sum, otherwise it adds the sum to the
store's previous value in one rounding.  The CSR product sums each row
sequentially in CSR order.

Float32 stores are held as float64 arrays of their exact float32 values; the
evaluation itself is always in float64.

Op table (arguments in order; k = imm[0]):
  unary   neg abs sqrt exp log erf square           (a R, out W)
  binary  add sub mul div pow max min               (a R, b R, out W)
  immediate  add_imm sub_imm rsub_imm mul_imm div_imm rdiv_imm   (a R, out W)
          a+k, a-k, k-a, a*k, a/k, k/a
  copy    (a R, out W)          out = a
  fill    (out W)               out = k
  axpy    (alpha R, x R, y RW)  y = y + alpha*x  (k=+1) | y = y - alpha*x (k=-1)
  sum     (x R, s Rd)           s (+)= sum x_i
  sumsq   (x R, s Rd)           s (+)= sum x_i*x_i
  dot     (x R, y R, s Rd)      s (+)= sum x_i*y_i         init flag = imm[0]
  spmv    (rowptr R, col R, val R, x R, y W)   y = A x over y's rows
"""
from __future__ import annotations

import numpy as np

from . import cnum
from .ir import Image, NoneP, Tiling, points

UNARY = {
    "neg": lambda a: -a,
    "abs": np.abs,
    "sqrt": np.sqrt,
    "exp": cnum.exp,
    "log": cnum.log,
    "erf": cnum.erf,
    "square": lambda a: a * a,
}
BINARY = {
    "add": lambda a, b: a + b,
    "sub": lambda a, b: a - b,
    "mul": lambda a, b: a * b,
    "div": lambda a, b: a / b,
    "pow": lambda a, b: cnum.power(np.broadcast_to(a, np.broadcast(a, b).shape), b),
    "max": np.maximum,
    "min": np.minimum,
}
IMMEDIATE = {
    "add_imm": lambda a, k: a + k,
    "sub_imm": lambda a, k: a - k,
    "rsub_imm": lambda a, k: k - a,
    "mul_imm": lambda a, k: a * k,
    "div_imm": lambda a, k: a / k,
    "rdiv_imm": lambda a, k: k / a,
}
REDUCE = {"sum": 1, "sumsq": 1, "dot": 2}


def _region(arr, part, p, rank):
    """Sub-store S[P, p] as a numpy view broadcastable over the task's element
    index (dropped launch dims become size-1 axes)."""
    if isinstance(part, NoneP) or isinstance(part, Image):
        return arr
    assert isinstance(part, Tiling)
    shape = arr.shape
    q = part.proj(p)
    q1 = part.proj(tuple(c + 1 for c in p))
    sl = tuple(slice(max(0, a * t + o), min(s, b * t + o))
               for a, b, t, o, s in zip(q, q1, part.tile, part.offset, shape))
    v = arr[sl]
    keep = part.proj.keep
    if keep is not None and rank > 0 and v.ndim < rank:
        newshape = [1] * rank
        for store_dim, launch_dim in enumerate(keep):
            newshape[launch_dim] = v.shape[store_dim]
        v = v.reshape(newshape)
    return v


def evaluate(tasks, stores: dict) -> dict:
    """Apply `tasks` in program order to `stores` (name -> numpy array).

    Arrays are modified in place (float arrays must be float64); the dict is
    returned for convenience."""
    for t in tasks:
        _run(t, stores)
    return stores


def _run(t, st):
    rank = len(t.domain)
    pts = points(t.domain)
    op = t.op
    args = t.args
    if op in REDUCE:
        nin = REDUCE[op]
        s_name = args[nin][0]
        contrib_x, contrib_y = [], []
        for p in pts:
            xs = [_region(st[a[0]], a[1], p, rank) for a in args[:nin]]
            if op == "sum":
                contrib_x.append(np.asarray(xs[0], dtype=np.float64).ravel())
            elif op == "sumsq":
                x = np.asarray(xs[0], dtype=np.float64).ravel()
                contrib_x.append(x)
                contrib_y.append(x)
            else:
                x, y = np.broadcast_arrays(xs[0], xs[1])
                contrib_x.append(np.asarray(x, dtype=np.float64).ravel())
                contrib_y.append(np.asarray(y, dtype=np.float64).ravel())
        xcat = np.concatenate(contrib_x) if contrib_x else np.zeros(0)
        if op == "sum":
            total = cnum.fsum(xcat)
        else:
            total = cnum.fsum_prod(xcat, np.concatenate(contrib_y))
        init = bool(t.imm[0]) if t.imm else False
        old = 0.0 if init else float(st[s_name])
        st[s_name][...] = total if init else old + total
        return
    if op == "spmv":
        rp, col, val, x = (st[a[0]] for a in args[:4])
        y_name, y_part = args[4][0], args[4][1]
        for p in pts:
            if isinstance(y_part, Tiling):
                lo = max(0, y_part.proj(p)[0] * y_part.tile[0] + y_part.offset[0])
                hi = min(st[y_name].shape[0],
                         y_part.proj(tuple(c + 1 for c in p))[0] * y_part.tile[0] + y_part.offset[0])
            else:
                lo, hi = 0, st[y_name].shape[0]
            if hi <= lo:
                continue
            sub_rp = rp[lo:hi + 1]
            st[y_name][lo:hi] = cnum.spmv(sub_rp - sub_rp[0], col[sub_rp[0]:sub_rp[-1]],
                                          val[sub_rp[0]:sub_rp[-1]], x)
        return
    # Elementwise ops: compute every point's result before writing any, so
    # a task reading and writing the same sub-store sees its inputs.
    results = []
    for p in pts:
        vals = [_region(st[a[0]], a[1], p, rank) for a in args]
        if op in UNARY:
            r = UNARY[op](np.asarray(vals[0], dtype=np.float64))
            out = 1
        elif op in BINARY:
            r = BINARY[op](np.asarray(vals[0], dtype=np.float64), np.asarray(vals[1], dtype=np.float64))
            out = 2
        elif op in IMMEDIATE:
            r = IMMEDIATE[op](np.asarray(vals[0], dtype=np.float64), float(t.imm[0]))
            out = 1
        elif op == "copy":
            r = np.array(vals[0], dtype=np.float64, copy=True)
            out = 1
        elif op == "fill":
            r = np.float64(t.imm[0])
            out = 0
        elif op == "axpy":
            alpha, x, y = (np.asarray(v, dtype=np.float64) for v in vals[:3])
            prod = alpha * x
            r = y + prod if float(t.imm[0]) > 0 else y - prod
            out = 2
        else:
            raise ValueError("unknown op " + op)
        results.append((p, out, r))
    for p, out, r in results:
        a = args[out]
        dst = _region(st[a[0]], a[1], p, rank)
        dst[...] = np.broadcast_to(r, dst.shape)
