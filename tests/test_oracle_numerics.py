"""Pins for the oracle's plain C numerics (exact sums, CSR SpMV, libm loops)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import cnum
import synth


def _exact_round(fr: Fraction) -> float:
    # float(Fraction) rounds to nearest-even exactly.
    return float(fr)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fsum_is_exactly_rounded(seed):
    rng = np.random.default_rng(seed)
    # Heavy cancellation across magnitudes.
    x = rng.standard_normal(4000) * np.exp2(rng.integers(-60, 60, 4000))
    x = np.concatenate([x, -x[:1500] * 0.999999, [1e300, -1e300, 3.0]])
    exact = sum((Fraction(float(v)) for v in x), Fraction(0))
    assert cnum.fsum(x) == _exact_round(exact)
    assert cnum.fsum(x) == math.fsum(x)


def test_fsum_half_even_and_edges():
    assert cnum.fsum(np.array([])) == 0.0
    assert cnum.fsum(np.array([1.0, 1e100, 1.0, -1e100])) == 2.0
    # 1 + 2^-53 + 2^-53*2^-60: the tail breaks the tie upward.
    x = np.array([1.0, 2.0 ** -53, 2.0 ** -113])
    assert cnum.fsum(x) == 1.0 + 2.0 ** -52
    # exact tie 1 + 2^-53 rounds to even (1.0)
    assert cnum.fsum(np.array([1.0, 2.0 ** -53])) == 1.0


def test_fsum_prod_rounds_each_product_then_sums_exactly():
    rng = np.random.default_rng(7)
    x = rng.standard_normal(3000)
    y = rng.standard_normal(3000)
    prods = [float(a) * float(b) for a, b in zip(x, y)]
    exact = sum((Fraction(p) for p in prods), Fraction(0))
    assert cnum.fsum_prod(x, y) == float(exact)


def test_spmv_sequential_row_order_brute_force():
    rowptr, col, val = synth.poisson_csr(5, 2)
    x = synth.rhs(25, 11)
    y = cnum.spmv(rowptr, col, val, x)
    for i in range(25):
        s = None
        for k in range(rowptr[i], rowptr[i + 1]):
            t = float(val[k]) * float(x[col[k]])
            s = t if s is None else s + t
        assert y[i] == s


def test_spmv_equals_dense_product_on_integers():
    # Integer data: every partial sum is exact, so any order must agree.
    rowptr, col, val = synth.poisson_csr(6, 3)
    n = 216
    A = np.zeros((n, n))
    for i in range(n):
        for k in range(rowptr[i], rowptr[i + 1]):
            A[i, col[k]] = val[k]
    xs = np.arange(n, dtype=np.float64) % 17 - 8
    assert np.array_equal(cnum.spmv(rowptr, col, val, xs), A @ xs)


def test_libm_loops_match_python_math():
    x = np.linspace(0.01, 30, 1001)
    assert all(cnum.log(x)[i] == math.log(x[i]) for i in range(0, 1001, 7))
    assert all(cnum.exp(-x)[i] == math.exp(-x[i]) for i in range(0, 1001, 7))
    z = np.linspace(-6, 6, 1001)
    assert all(cnum.erf(z)[i] == math.erf(z[i]) for i in range(0, 1001, 7))
    assert cnum.power(np.array([2.0, 9.0]), np.array([10.0, 0.5])).tolist() == [1024.0, 3.0]


def test_poisson_structure():
    rowptr, col, val = synth.poisson_csr(64, 2)
    assert rowptr[-1] == 5 * 64 * 64 - 4 * 64 == 20224
    rowptr3, col3, val3 = synth.poisson_csr(8, 3)
    assert rowptr3[-1] == 7 * 8 ** 3 - 6 * 8 ** 2
    # columns sorted within rows, symmetric matrix, diagonally dominant
    for rp, c, v, m, d in ((rowptr, col, val, 64, 2), (rowptr3, col3, val3, 8, 3)):
        n = m ** d
        for i in range(0, n, max(1, n // 50)):
            cols = c[rp[i]:rp[i + 1]]
            assert np.all(np.diff(cols) > 0)
            assert v[rp[i]:rp[i + 1]][list(cols).index(i)] == 2 * d


def test_synth_generator_is_deterministic_and_uniform():
    a = synth.uniform01(5, 0, 100000)
    b = synth.uniform01(5, 0, 100000)
    assert np.array_equal(a, b)
    assert 0.0 <= a.min() and a.max() < 1.0
    assert abs(a.mean() - 0.5) < 0.005
    c = synth.uniform01(5, 1, 100000)
    assert abs(np.corrcoef(a, c)[0, 1]) < 0.01
    # the counter-based stream can be read from any offset
    assert np.array_equal(synth.uniform01(5, 0, 10, start=100), a[100:110])
    S, K, T = synth.bs_inputs(1000)
    assert S.min() >= 10 and S.max() < 100 and T.min() >= 0.25 and T.max() < 2
