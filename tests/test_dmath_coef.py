"""The FP64 log/exp/erf constants the kernels use are the ones their
generator derives, and every fit is inside its error budget (well below
half an ulp of the result, so the final roundings dominate)."""
import importlib.util
import os

import pytest

mp = pytest.importorskip("mpmath")

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_2406_18109_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_dmath", os.path.join(CSRC, "gen_dmath.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_committed_header_is_the_generated_one():
    g = _gen()
    text, _ = g.render()
    with open(os.path.join(CSRC, "dmath_coef.h")) as fh:
        assert fh.read() == text


def test_fit_errors_within_budget():
    _, errors = _gen().render()
    # relative errors for log and small-range erf; absolute for the erfc tail (erf is
    # 1 - erfc there, |erf| > 0.77) and for exp(r) in [0.70, 1.42]
    assert errors["log"] < 2.0 ** -56
    assert errors["erf_small"] < 2.0 ** -55
    assert errors["erfc_tail"] < 2.0 ** -56
    assert errors["exp"] < 2.0 ** -60


def test_ln2_split():
    g = _gen()
    hi = mp.mpf(g.LN2_HI)
    # k * LN2_HI is exact for every exponent a double can have
    assert hi * 2 ** 42 == int(hi * 2 ** 42)
    assert abs(hi + mp.mpf(g.LN2_LO) - mp.log(2)) < mp.mpf(2) ** -95
