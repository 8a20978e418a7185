"""The order of additions of the block-sum reduction (fin_sums in
csrc/vm_exec.h), modelled in numpy and compared with the canonical pairwise
tree it must equal: chunks of 1024 block sums, each a complete subtree
(pairwise, level by level), then the chunk sums by the same tree.  The
device code reduces a chunk by aligned quarters of 256 (four values per
lane, then a lane tree: block_tree) and joins the quarters as the chunk
tree's two top levels, with 4 or 16 waves per block and the chunk sums by
quarters when there are more than 256.  Float32 sums of random values give
different bits under almost any change of association, so equal bits pin the
model to the canonical tree at every size, including ragged chunks, more than
256 chunks (beyond what the GPU tests can allocate) and the four-wave form's
64-chunk limit."""
import numpy as np
import pytest


def pairwise(a):
    a = list(a)
    n, h = len(a), 1
    while h < n:
        for i in range(0, n, 2 * h):
            if i + h < n:
                a[i] = np.float32(a[i] + a[i + h])
        h *= 2
    return a[0] if n else np.float32(0)


def canonical(p):
    cs = [pairwise(p[c:c + 1024]) for c in range(0, len(p), 1024)]
    return pairwise(cs) if cs else np.float32(0)


def block_tree(a, cnt):
    v = []
    for j in range(0, cnt, 4):
        c = min(4, cnt - j)
        v01 = np.float32(a[j] + a[j + 1]) if c > 1 else a[j]
        v.append(np.float32(v01 + np.float32(a[j + 2] + a[j + 3])) if c == 4 else
                 np.float32(v01 + a[j + 2]) if c == 3 else v01)
    n, h = len(v), 1
    while h < n:
        for i in range(0, n, 2 * h):
            if i + h < n:
                v[i] = np.float32(v[i] + v[i + h])
        h *= 2
    return v[0]


def top(s4, n):
    a, b = s4[0], s4[2]
    if 256 < n:
        a = np.float32(a + s4[1])
    if 768 < n:
        b = np.float32(b + s4[3])
    if 512 < n:
        a = np.float32(a + b)
    return a


def quarters(a, n):
    return [block_tree(a[q * 256:], min(n - q * 256, 256)) if n > q * 256 else np.float32(0) for q in range(4)]


def fin_sums(p, nw):
    n = len(p)
    nch = (n + 1023) // 1024
    fcs = [None] * nch
    for c0 in range(0, nch, nw // 4):
        for c in range(c0, min(c0 + nw // 4, nch)):
            L = min(1024, n - c * 1024)
            fcs[c] = top(quarters(p[c * 1024:], L), L)
    if nch == 0:
        return np.float32(0)
    if nch <= 256:
        return block_tree(fcs, nch)
    return top(quarters(fcs, nch), nch)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 255, 256, 257, 1023, 1024, 1025, 2049, 4097, 65536, 65537, 262145, 300000])
def test_block_sum_order_is_canonical(n):
    p = np.random.default_rng(n).standard_normal(n).astype(np.float32) * np.float32(1e3)
    ref = canonical(p)
    assert fin_sums(p, 16) == ref
    if (n + 1023) // 1024 <= 64:
        assert fin_sums(p, 4) == ref


def test_a_changed_order_is_detected():
    """The check has teeth: a quarter tree that pairs its lanes' groups left
    to right instead of pairwise changes the bits."""
    p = np.random.default_rng(9).standard_normal(4096).astype(np.float32) * np.float32(1e3)
    ref = canonical(p)

    def seq_tree(a, cnt):
        acc = np.float32(0)
        for j in range(0, cnt, 4):
            acc = np.float32(acc + pairwise(a[j:min(j + 4, cnt)]))
        return acc
    chunks = []
    for c in range(0, 4096, 1024):
        qs = [seq_tree(p[c + k * 256:], 256) for k in range(4)]
        chunks.append(top(qs, 1024))
    assert pairwise(chunks) != ref
