"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle.

This module holds input generation only: counter-based random numbers, the
structure and coefficients of the Poisson test matrices, the Jacobi grid's
boundary data and the serving workload's request list.  It holds none of the
arithmetic of the fused-execution method (no task evaluation, no reductions,
no solver steps).

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: value(key, c) = mix(key + (c + 1) * GAMMA), where mix is the
SplitMix64 finaliser.  A uniform double in [0, 1) is (value >> 11) * 2**-53.
The key of (seed, stream) is mix(seed * GAMMA2 + stream); streams of one seed
are independent sequences.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
GAMMA2 = np.uint64(0xD1B54A32D192ED03)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int = 0) -> np.uint64:
    with np.errstate(over="ignore"):
        k = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * GAMMA2 + np.uint64(stream)
    return _mix(np.array([k], dtype=np.uint64))[0]


def raw64(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """n raw 64-bit values of (seed, stream) starting at counter `start`."""
    key = stream_key(seed, stream)
    c = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(key + c * GAMMA)


def uniform01(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """n doubles uniform in [0, 1): (value >> 11) * 2**-53."""
    v = raw64(seed, stream, n, start) >> np.uint64(11)
    return v.astype(np.float64) * (2.0 ** -53)


def uniform(seed: int, stream: int, n: int, lo: float, hi: float,
            dtype=np.float64, start: int = 0) -> np.ndarray:
    """n values uniform in [lo, hi), computed in float64 then rounded to dtype."""
    u = uniform01(seed, stream, n, start)
    x = lo + (hi - lo) * u
    return x.astype(dtype)


# --------------------------------------------------------------------------
# Black-Scholes option batch: spot and strike uniform in [10, 100), expiry
# uniform in [0.25, 2) years; rate 0.02 and volatility 0.3 are scalars.
# --------------------------------------------------------------------------
BS_SEED = 1001
BS_RATE = 0.02
BS_VOL = 0.3


def bs_inputs(n: int, dtype=np.float64, seed: int = BS_SEED):
    S = uniform(seed, 0, n, 10.0, 100.0, dtype)
    K = uniform(seed, 1, n, 10.0, 100.0, dtype)
    T = uniform(seed, 2, n, 0.25, 2.0, dtype)
    return S, K, T


# --------------------------------------------------------------------------
# Jacobi grid: the full array includes the boundary ring.  Row 0 is 1.0,
# every other cell (boundary and interior) starts at 0.
# --------------------------------------------------------------------------
def jacobi_grid(n: int, dtype=np.float64) -> np.ndarray:
    g = np.zeros((n, n), dtype=dtype)
    g[0, :] = 1.0
    return g


# --------------------------------------------------------------------------
# Poisson matrices in CSR with 32-bit indices.  Unknowns are numbered
# lexicographically with x fastest; Dirichlet boundary rows are eliminated,
# so a row holds the diagonal (2*dim) and -1 for each in-grid neighbour.
# Columns inside a row are sorted ascending.
# --------------------------------------------------------------------------
def poisson_csr(m: int, dim: int):
    """Return (rowptr int32[n+1], col int32[nnz], val float64[nnz])."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    n = m ** dim
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx
    for _ in range(dim):
        coords.append(rem % m)
        rem = rem // m
    # neighbour offsets sorted ascending: -m^(d-1) ... -1, 0, +1 ... +m^(d-1)
    offs = []
    for axis in reversed(range(dim)):
        offs.append((axis, -1))
    offs.append((None, 0))
    for axis in range(dim):
        offs.append((axis, +1))
    valid = []
    for axis, s in offs:
        if axis is None:
            valid.append(np.ones(n, dtype=bool))
        elif s < 0:
            valid.append(coords[axis] > 0)
        else:
            valid.append(coords[axis] < m - 1)
    counts = np.zeros(n, dtype=np.int64)
    for v in valid:
        counts += v
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    nnz = int(rowptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    pos = rowptr[:-1].copy()
    for (axis, s), v in zip(offs, valid):
        rows = idx[v]
        p = pos[v]
        if axis is None:
            col[p] = rows
            val[p] = 2.0 * dim
        else:
            col[p] = rows + s * (m ** axis)
            val[p] = -1.0
        pos[v] += 1
    return rowptr.astype(np.int32), col, val



def injection_csr(mc: int):
    """Injection from the (2 mc + 1)^2 interior grid to the mc^2 one (x
    fastest, Dirichlet boundary): coarse point (I, J) takes the value of fine
    point (2I+1, 2J+1).  Shape mc^2 x (2 mc + 1)^2, one entry of 1 per row."""
    mf = 2 * mc + 1
    J, I = np.divmod(np.arange(mc * mc, dtype=np.int64), mc)
    col = ((2 * J + 1) * mf + 2 * I + 1).astype(np.int32)
    rowptr = np.arange(mc * mc + 1, dtype=np.int32)
    return rowptr, col, np.ones(mc * mc)


def bilinear_csr(mc: int):
    """Bilinear interpolation from the mc^2 grid to the (2 mc + 1)^2 one,
    zero outside the grid: a fine point on a coarse point takes its value
    (weight 1), one between two coarse points along a line their mean
    (1/2 each), one at a cell centre the mean of the four corners (1/4 each).
    Columns ascending."""
    mf = 2 * mc + 1
    j, i = np.divmod(np.arange(mf * mf, dtype=np.int64), mf)

    def axis(k):
        # coarse neighbours along one axis and their weights: odd fine index
        # 2K+1 sits on coarse K; even 2K lies between coarse K-1 and K
        odd = (k % 2) == 1
        lo = np.where(odd, (k - 1) // 2, k // 2 - 1)
        hi = np.where(odd, -1, k // 2)
        wl = np.where(odd, 1.0, 0.5)
        wh = np.where(odd, 0.0, 0.5)
        return (lo, wl), (hi, wh)

    cols, vals = [], []
    for (cj, wj) in axis(j):            # ascending coarse row J first,
        for (ci, wi) in axis(i):        # then coarse column I: ascending index
            ok = (cj >= 0) & (cj < mc) & (ci >= 0) & (ci < mc) & (wj > 0) & (wi > 0)
            cols.append(np.where(ok, cj * mc + ci, -1))
            vals.append(np.where(ok, wj * wi, 0.0))
    col = np.stack(cols, axis=1)
    val = np.stack(vals, axis=1)
    keep = col >= 0
    rowptr = np.zeros(mf * mf + 1, dtype=np.int64)
    np.cumsum(keep.sum(axis=1), out=rowptr[1:])
    return rowptr.astype(np.int32), col[keep].astype(np.int32), val[keep]


def gmg_levels(m0: int, nlev: int):
    """The multigrid hierarchy of the m0^2 Poisson problem (m0 = 2^k - 1):
    level l has side m_l = (m_{l-1} - 1) / 2 and operator poisson_csr(m_l)
    scaled by 4^-l (the 5-point operator rediscretised on the coarser grid,
    in units of the finest h^2; every value stays exact), whose diagonal is
    4 * 4^-l, and the transfers to and from level l+1 (injection and
    bilinear interpolation).  Returns [(A, diag, R, P)] with R = P = None on
    the coarsest level."""
    out, m = [], m0
    for l in range(nlev):
        rp, col, val = poisson_csr(m, 2)
        A = (rp, col, val * 0.25 ** l)
        diag = 4.0 * 0.25 ** l
        if l < nlev - 1:
            if m % 2 == 0 or m < 3:
                raise ValueError("side must be 2^k - 1 on every level but the last")
            mc = (m - 1) // 2
            out.append((A, diag, injection_csr(mc), bilinear_csr(mc)))
            m = mc
        else:
            out.append((A, diag, None, None))
    return out


def convdiff_csr(m: int, dim: int, c: float = 0.5):
    """A nonsymmetric variant of poisson_csr: first-order upwind convection
    along x, so the diagonal is 2*dim + c and the west neighbour -1 - c (c
    exactly representable keeps every value exact).  Weakly diagonally
    dominant and irreducible, hence nonsingular.  Same CSR layout."""
    rowptr, col, val = poisson_csr(m, dim)
    rows = np.repeat(np.arange(rowptr.size - 1, dtype=np.int64), np.diff(rowptr))
    val = val.copy()
    val[col == rows] += c
    val[col == rows - 1] -= c   # x fastest: column i-1 is the west neighbour when it exists
    return rowptr, col, val

def rhs(n: int, seed: int, stream: int = 0) -> np.ndarray:
    """Right-hand side uniform in [-1, 1)."""
    return uniform(seed, stream, n, -1.0, 1.0)


CG64_SEED = 2001
CG256_SEED = 2002
BICG256_SEED = 2003   # BiCGSTAB on the 256^3 convection-diffusion system
GMG_SEED = 2004       # multigrid on the 1023^2 Poisson problem


# --------------------------------------------------------------------------
# Serving workload: independent 2-D Poisson solves with grid side uniform in
# {lo..hi}, right-hand sides from seed 3002 + request id, Poisson arrivals.
# --------------------------------------------------------------------------
SERVE_SIDE_SEED = 3001
SERVE_RHS_SEED = 3002
SERVE_ARRIVAL_SEED = 3003


def serve_sides(count: int, lo: int = 32, hi: int = 512, seed: int = SERVE_SIDE_SEED) -> np.ndarray:
    u = uniform01(seed, 0, count)
    return (lo + np.floor(u * (hi - lo + 1))).astype(np.int64)


def serve_rhs(req_id: int, n: int) -> np.ndarray:
    return rhs(n, SERVE_RHS_SEED + req_id)


def serve_arrivals(count: int, rate: float, seed: int = SERVE_ARRIVAL_SEED) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    u = uniform01(seed, 0, count)
    gaps = -np.log1p(-u) / rate
    return np.cumsum(gaps)
