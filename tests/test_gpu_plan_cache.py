"""Plans loaded from the on-disk cache execute with no analysis and give the
same bits as the plans the saving context built (Black-Scholes, CG,
BiCGSTAB)."""
import numpy as np
import pytest

import paper_2406_18109_amd as dfx
import synth
from gpu_util import bs_run, note, upload

pytestmark = pytest.mark.gpu


def _run(c):
    _, call, put = bs_run(c, 3 * 4096 + 77, passes=2)
    m = 48
    rowptr, col, val = synth.convdiff_csr(m, 2)
    b = synth.rhs(m * m, 4130)
    hs = [upload(c, a) for a in (rowptr, col, val, b)]
    res = [call, put]
    for cls in (dfx.apps.CG, dfx.apps.BiCGSTAB):
        s = cls(c, *hs, m * m)
        for _ in range(5):
            s.iteration()
        res.append(c.store_read(s.x, [m * m], "f64"))
    return res


def test_loaded_plans_bit_identical(tmp_path):
    path = str(tmp_path / "plans.bin")
    note("plan cache: save")
    a = dfx.Context(device=0, window_size=64)
    ra = _run(a)
    n = a.plan_cache_save(path)
    a.close()
    note("plan cache: load %d plans" % n)
    b = dfx.Context(device=0, window_size=64)
    assert b.plan_cache_load(path) == n
    rb = _run(b)
    st = b.stats()
    b.close()
    assert st["memo_misses"] == 0
    for x, y in zip(ra, rb):
        assert np.array_equal(x, y)
