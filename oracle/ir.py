"""The paper's IR (section 3, the syntax figure) as plain Python values.

Test infrastructure only.  Stores, projection functions, partitions,
privileges and index tasks exactly as the grammar defines them, plus the
sub-store construct used for reasoning:

  Store       S ::= Store(id, shape)
  Projection  F ::= Projection(id, Point -> Point)      (here: keep a subset of dims)
  Partition   P ::= None | Tiling(tile, offset, F) | Image(src, src_part)
  Privilege   Pr ::= R | W | Rd | RW
  IndexTask   T ::= IndexTask(domain, [(S, P, Pr)])

`Image` is the one partition kind added beyond None and Tiling (section 3.1
allows more kinds as long as two partitions can be compared in O(1)): the
sub-store of point p is the set of coordinates stored in src[src_part, p],
which is how a CSR matrix-vector product names the gathered entries of x.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from typing import Optional, Tuple

R, W, RD, RW = "R", "W", "Rd", "RW"


def reads(pr: str) -> bool:
    return pr in (R, RW)


def writes(pr: str) -> bool:
    return pr in (W, RW)


def reduces(pr: str) -> bool:
    return pr == RD


@dataclass(frozen=True)
class Proj:
    """Projection keeping launch dims `keep` (in order) as the store's dims.

    keep=None is the identity.  Dropping a launch dim makes several points
    map to the same sub-store (aliasing / replication, section 3.1)."""
    keep: Optional[Tuple[int, ...]] = None

    def __call__(self, p):
        if self.keep is None:
            return tuple(p)
        return tuple(p[k] for k in self.keep)


@dataclass(frozen=True)
class NoneP:
    pass


@dataclass(frozen=True)
class Tiling:
    tile: Tuple[int, ...]
    offset: Tuple[int, ...]
    proj: Proj = field(default_factory=Proj)


@dataclass(frozen=True)
class Image:
    src: str
    src_part: object


@dataclass
class Task:
    op: str
    domain: Tuple[int, ...]          # () is a single task
    args: list                       # [(store name, partition, privilege)]
    imm: tuple = ()


def points(domain):
    """All points of a rectangular launch domain; () has the single point ()."""
    return list(itertools.product(*[range(d) for d in domain]))


def tiling_box(part: Tiling, p, shape):
    """Sub-store bounds of a Tiling partition at point p (section 3.1, the
    sub-store-bounds formula): [proj(p)*tile, proj(p+1)*tile) + offset,
    intersected with the store's extent."""
    q = part.proj(p)
    q1 = part.proj(tuple(c + 1 for c in p))
    lo = tuple(max(0, min(s, a * t + o)) for a, t, o, s in zip(q, part.tile, part.offset, shape))
    hi = tuple(max(0, min(s, b * t + o)) for b, t, o, s in zip(q1, part.tile, part.offset, shape))
    return lo, hi


def substore_points(shape, part, p, data=None):
    """The set of store points in S[P, p] (small stores only)."""
    if isinstance(part, NoneP):
        return set(itertools.product(*[range(s) for s in shape]))
    if isinstance(part, Tiling):
        lo, hi = tiling_box(part, p, shape)
        return set(itertools.product(*[range(a, b) for a, b in zip(lo, hi)]))
    if isinstance(part, Image):
        if data is None or part.src not in data:
            raise ValueError("Image partition needs the source store's values")
        src = data[part.src]
        src_pts = substore_points(src.shape, part.src_part, p, data)
        return {(int(src[q]),) for q in src_pts}
    raise TypeError(part)
