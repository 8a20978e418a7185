"""Brute-force and definitional statement of the fusion analysis (sections 4 and 5).

Test infrastructure only.  Everything here enumerates points and sub-stores
explicitly, so it is meant for tiny launch domains (a few points) and tiny
stores (a few hundred elements).

  dep(...)            Definition 1 (true-, anti- and reduction-dependence)
  dependence_map(...) the dependence map D(T1, T2) of section 4.1
  fusible(...)        the fusibility definition: D[p] is a subset of {p}
  constraints(...)    the four fusion constraints of section 4.2 (figure of
                      fusion constraints), each quantified over pairs exactly
                      as stated
  longest_prefix(...) largest f such that window[:f] meets all constraints
  covers(...)         covers(S, P): P's sub-stores hold every point of S
  temporaries(...)    the temporary-store definition of section 5.1
  canonical(...)      the De Bruijn-like renaming of section 5.2
"""
from __future__ import annotations

import itertools

from .ir import (Image, NoneP, Tiling, points, reads, reduces, substore_points,
                 writes)


def _args_by_store(task):
    out = {}
    for (s, p, pr) in task.args:
        out.setdefault(s, []).append((p, pr))
    return out


def dep(t1, p, t2, p2, shapes, data=None) -> bool:
    """Definition 1: T2^p2 depends on T1^p (T1 issued before T2)."""
    a1 = _args_by_store(t1)
    a2 = _args_by_store(t2)
    for s in set(a1) & set(a2):
        for (P1, pr1) in a1[s]:
            sub1 = substore_points(shapes[s], P1, p, data)
            if not sub1:
                continue
            for (P2, pr2) in a2[s]:
                true_dep = writes(pr1) and (reads(pr2) or writes(pr2) or reduces(pr2))
                anti_dep = reads(pr1) and (writes(pr2) or reduces(pr2))
                red_dep = reduces(pr1) and (reads(pr2) or writes(pr2))
                if not (true_dep or anti_dep or red_dep):
                    continue
                sub2 = substore_points(shapes[s], P2, p2, data)
                if sub1 & sub2:
                    return True
    return False


def dependence_map(t1, t2, shapes, data=None):
    """D(T1, T2)[p] = { p' in domain(T2) : dep(T1^p, T2^p') }."""
    return {p: {p2 for p2 in points(t2.domain) if dep(t1, p, t2, p2, shapes, data)}
            for p in points(t1.domain)}


def fusible(t1, t2, shapes, data=None) -> bool:
    D = dependence_map(t1, t2, shapes, data)
    return all(D[p] <= {p} for p in D)


def legal(task, shapes, data=None) -> bool:
    """Non-interference of one index task: no two distinct points access
    overlapping data where one of them writes, and no point reads or writes
    data another point reduces to.  The fusion constraints identify
    point-wise dependence only for streams of such tasks (a write through
    the same partition is point-wise only if that partition's sub-stores
    are disjoint across written points)."""
    pts = points(task.domain)
    for ia, (s1, P1, pr1) in enumerate(task.args):
        for (s2, P2, pr2) in task.args:
            if s1 != s2:
                continue
            conflict = (writes(pr1) and (reads(pr2) or writes(pr2) or reduces(pr2))) or \
                       (reduces(pr1) and (reads(pr2) or writes(pr2)))
            if not conflict:
                continue
            for p in pts:
                a = substore_points(shapes[s1], P1, p, data)
                for p2 in pts:
                    if p2 != p and a & substore_points(shapes[s2], P2, p2, data):
                        return False
    return True


def prefix_fusible(tasks, shapes, data=None) -> bool:
    """Every pair T_i, T_j (i < j) of the sequence is fusible."""
    return all(fusible(tasks[i], tasks[j], shapes, data)
               for i in range(len(tasks)) for j in range(i + 1, len(tasks)))


# --- The four fusion constraints (section 4.2) -----------------------------

def launch_domain_equivalence(ts) -> bool:
    return all(t.domain == ts[0].domain for t in ts)


def true_dependence(ts) -> bool:
    for i, ti in enumerate(ts):
        for (S, P, pr) in ti.args:
            if not writes(pr):
                continue
            for tj in ts[i + 1:]:
                for (S2, P2, pr2) in tj.args:
                    if S2 == S and (reads(pr2) or writes(pr2)) and P2 != P:
                        return False
    return True


def anti_dependence(ts) -> bool:
    for i, ti in enumerate(ts):
        for (S, P, pr) in ti.args:
            if not reads(pr):
                continue
            for tj in ts[i + 1:]:
                for (S2, P2, pr2) in tj.args:
                    if S2 == S and writes(pr2) and P2 != P:
                        return False
    return True


def reduction(ts) -> bool:
    for i, ti in enumerate(ts):
        for (S, P, pr) in ti.args:
            if not reduces(pr):
                continue
            for j, tj in enumerate(ts):
                if j == i:
                    continue
                for (S2, P2, pr2) in tj.args:
                    if S2 == S and (reads(pr2) or writes(pr2)):
                        return False
    return True


def constraints(ts) -> bool:
    return (launch_domain_equivalence(ts) and true_dependence(ts)
            and anti_dependence(ts) and reduction(ts))


def longest_prefix(window) -> int:
    """Largest f >= 1 with constraints(window[:f]); 0 for an empty window."""
    f = 0
    for k in range(1, len(window) + 1):
        if constraints(window[:k]):
            f = k
    return f


# --- Temporary stores (section 5.1) -----------------------------------------

def covers(shape, part, domain, data=None) -> bool:
    """True when the sub-stores of `part` over `domain` hold every point of the store."""
    if isinstance(part, NoneP):
        return True
    allpts = set(itertools.product(*[range(s) for s in shape]))
    got = set()
    for p in points(domain):
        got |= substore_points(shape, part, p, data)
    return allpts <= got


def temporaries(window, f, app_live, shapes, data=None):
    """Stores temporary in the fusion of window[:f]:
      (1) every read of S through P in the prefix follows a write of S
          through the same P in an earlier prefix task, and that P covers S;
      (2) no task after f reads or reduces S;
      (3) S has no live application reference.
    """
    prefix, rest = window[:f], window[f:]
    stores = []
    for t in prefix:
        for (s, _, _) in t.args:
            if s not in stores:
                stores.append(s)
    temps = set()
    for s in stores:
        ok = True
        for j, tj in enumerate(prefix):
            for (S, P, pr) in tj.args:
                if S != s or not reads(pr):
                    continue
                found = any(S2 == s and writes(pr2) and P2 == P
                            and covers(shapes[s], P, ti.domain, data)
                            for ti in prefix[:j] for (S2, P2, pr2) in ti.args)
                if not found:
                    ok = False
        if not ok:
            continue
        if any(S == s and (reads(pr) or reduces(pr)) for tk in rest for (S, _, pr) in tk.args):
            continue
        if s in app_live:
            continue
        temps.add(s)
    return temps


# --- Canonical form (section 5.2) --------------------------------------------

def canonical(window):
    """Rename stores by order of first appearance (alpha-equivalence).

    Returns, per task, its op, launch domain, immediates and the list of
    (canonical store index, partition, privilege); Image partitions name
    their source by canonical index too."""
    names = {}

    def idx(s):
        if s not in names:
            names[s] = len(names)
        return names[s]

    out = []
    for t in window:
        args = []
        for (s, P, pr) in t.args:
            i = idx(s)
            if isinstance(P, Image):
                P = ("Image", idx(P.src), P.src_part)
            args.append((i, P, pr))
        out.append((t.op, tuple(t.domain), tuple(t.imm), tuple(args)))
    return tuple(out)


def store_pattern(window):
    """Only the store/privilege pattern of the canonical form (the paper's
    printed representation)."""
    return tuple(tuple((i, pr) for (i, _, pr) in t[3]) for t in canonical(window))
