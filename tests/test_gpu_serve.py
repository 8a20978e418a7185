"""Continuous-batching CG server: each result is the same alone and in the mix,
matches the unbatched task-stream CG bit for bit, and agrees with the oracle;
admission respects the HBM budget; error paths are reported."""
import math
import time

import numpy as np
import pytest

import paper_2406_18109_amd as dfx
from paper_2406_18109_amd import _binding as B
import synth
from oracle import cnum
from oracle import workloads as wl

from gpu_util import ctx, note, rel_err, rel_err_floor, upload

pytestmark = pytest.mark.gpu
TOL = 1e-8


def _task_stream_cg(rowptr, col, val, b, iters):
    c = ctx()
    n = b.size
    hs = [upload(c, a) for a in (rowptr, col, val, b)]
    cg = dfx.apps.CG(c, *hs, n)
    for _ in range(iters):
        cg.iteration()
    x = c.store_read(cg.x, [n], "f64")
    c.close()
    return x


def test_alone_equals_mix_and_matches_oracle():
    c = ctx()
    c.serve_start(hbm_budget=1 << 30, max_slots=6, tol=TOL, max_iter=4000)
    sides = [40, 17, 64, 23, 33, 50, 8, 64, 31, 45]
    mats = {s: synth.poisson_csr(s, 2) for s in set(sides)}
    A = 40
    rpA, colA, valA = mats[A]
    bA = synth.serve_rhs(0, A * A)
    note("serve alone")
    t = c.serve_submit(rpA, colA, valA, bA)
    rA = c.serve_wait(t, 120)
    xA = c.serve_read_x(t, A * A)
    assert rA["status"] == B.SOLVE_CONVERGED
    note("serve mix")
    tickets = []
    for i, s in enumerate(sides):
        rp, col, val = mats[s]
        b = bA if i == 4 else synth.serve_rhs(i + 1, s * s)
        if i == 4:
            assert s == 33
            rp, col, val = mats[A]
        tickets.append((c.serve_submit(rp, col, val, b), s if i != 4 else A, b))
        time.sleep(0.002 * (i % 3))
    res = [(c.serve_wait(t, 300), s, b, t) for (t, s, b) in tickets]
    st = c.serve_stats()
    assert st["completed"] == len(sides) + 1
    for r, s, b, t in res:
        assert r["status"] == B.SOLVE_CONVERGED, (s, r)
        x = c.serve_read_x(t, s * s)
        rp, col, val = mats[s]
        # recursive and true residual
        assert r["rel_residual"] <= TOL
        true_res = np.linalg.norm(b - cnum.spmv(rp, col, val, x)) / np.linalg.norm(b)
        assert true_res <= 2 * TOL
        if t == tickets[4][0]:
            assert np.array_equal(x, xA) and r["iterations"] == rA["iterations"]
    # the oracle's CG for the same number of iterations
    xo, ho = wl.cg(rpA, colA, valA, bA, rA["iterations"])
    assert rel_err_floor(xA, xo) <= 1e-9
    assert abs(rA["rel_residual"] - math.sqrt(ho[-1] / ho[0])) <= 1e-9 * math.sqrt(ho[-1] / ho[0])
    # same arithmetic as the unbatched task-stream executor
    xt = _task_stream_cg(rpA, colA, valA, bA, rA["iterations"])
    assert np.array_equal(xA, xt)
    c.serve_stop()
    c.close()


def test_multi_tile_alone_equals_mix_and_matches_oracle():
    """Solves of several tiles (one tile holds 4096 unknowns): sides 129, 300
    and 512 (5, 22 and 64 tiles) alone, then inside a mix of 16 uneven solves
    that also holds one-tile ones.  Each multi-tile result is bit-identical
    alone and in the mix, bit-identical to the task-stream CG run for the
    same number of iterations, and within tolerance of the oracle's CG."""
    big = [129, 300, 512]
    mix = [129, 40, 300, 64, 512, 23, 96, 200, 33, 257, 50, 150, 8, 380, 70, 450]
    mats = {s: synth.poisson_csr(s, 2) for s in set(mix)}
    rhs = {s: synth.serve_rhs(600 + s, s * s) for s in set(mix)}
    alone = {}
    for s in big:
        c = ctx()
        c.serve_start(hbm_budget=1 << 30, max_slots=4, tol=TOL, max_iter=20 * s)
        note("serve alone side=%d" % s)
        t = c.serve_submit(*mats[s], rhs[s])
        r = c.serve_wait(t, 300)
        assert r["status"] == B.SOLVE_CONVERGED, (s, r)
        alone[s] = (r, c.serve_read_x(t, s * s))
        c.serve_stop()
        c.close()
    c = ctx()
    c.serve_start(hbm_budget=1 << 30, max_slots=8, tol=TOL, max_iter=20 * max(mix))
    note("serve mix of %d solves" % len(mix))
    tickets = []
    for i, s in enumerate(mix):
        tickets.append((c.serve_submit(*mats[s], rhs[s]), s))
        time.sleep(0.003 * (i % 4))
    inmix = {}
    for t, s in tickets:
        r = c.serve_wait(t, 600)
        assert r["status"] == B.SOLVE_CONVERGED, (s, r)
        x = c.serve_read_x(t, s * s)
        rp, col, val = mats[s]
        true_res = np.linalg.norm(rhs[s] - cnum.spmv(rp, col, val, x)) / np.linalg.norm(rhs[s])
        assert r["rel_residual"] <= TOL and true_res <= 2 * TOL, (s, r, true_res)
        inmix[s] = (r, x)
    c.serve_stop()
    c.close()
    for s in big:
        (ra, xa), (rm, xm) = alone[s], inmix[s]
        assert ra["iterations"] == rm["iterations"] and ra["rel_residual"] == rm["rel_residual"], s
        assert np.array_equal(xa, xm), s
        note("serve side=%d: task-stream CG, %d iterations" % (s, ra["iterations"]))
        assert np.array_equal(xa, _task_stream_cg(*mats[s], rhs[s], ra["iterations"])), s
        note("serve side=%d: oracle CG" % s)
        xo, ho = wl.cg(*mats[s], rhs[s], ra["iterations"])
        assert rel_err_floor(xa, xo) <= 1e-9, s
        ro = math.sqrt(ho[-1] / ho[0])
        assert abs(ra["rel_residual"] - ro) <= 1e-9 * ro, s


def test_iterations_per_round_do_not_change_results():
    """A solve that converges inside a multi-iteration round stops on the
    device: x, the iteration count and the residual are those of one
    iteration per round."""
    sides = [40, 23, 8, 57]
    mats = {s: synth.poisson_csr(s, 2) for s in sides}
    out = {}
    for ipr in (1, 7):
        c = ctx()
        c.serve_start(hbm_budget=1 << 30, max_slots=4, tol=TOL, max_iter=4000, iters_per_round=ipr)
        note("serve iters_per_round=%d" % ipr)
        tickets = [(c.serve_submit(*mats[s], synth.serve_rhs(50 + i, s * s)), s) for i, s in enumerate(sides)]
        out[ipr] = [(c.serve_wait(t, 300), c.serve_read_x(t, s * s)) for t, s in tickets]
        rounds = c.serve_stats()["rounds"]
        out[ipr].append(rounds)
        c.serve_stop()
        c.close()
    for (r1, x1), (r7, x7) in zip(out[1][:-1], out[7][:-1]):
        assert r1["status"] == r7["status"] == B.SOLVE_CONVERGED
        assert r1["iterations"] == r7["iterations"]
        assert r1["rel_residual"] == r7["rel_residual"]
        assert np.array_equal(x1, x7)
    assert out[7][-1] < out[1][-1]


def test_admission_binds_to_budget():
    c = ctx()
    s = 96
    rp, col, val = synth.poisson_csr(s, 2)
    n = s * s
    fp_est = 12 * col.size + 4 * (n + 1) + 5 * 8 * n
    budget = int(2.5 * fp_est)
    c.serve_start(hbm_budget=budget, max_slots=16, tol=TOL, max_iter=4000)
    ts = [c.serve_submit(rp, col, val, synth.serve_rhs(100 + i, n)) for i in range(6)]
    rs = [c.serve_wait(t, 300) for t in ts]
    assert all(r["status"] == B.SOLVE_CONVERGED for r in rs)
    st = c.serve_stats()
    assert st["peak_bytes"] <= budget
    # at most two fit at once: admissions are staggered
    admits = sorted(r["t_admit"] for r in rs)
    dones = sorted(r["t_done"] for r in rs)
    assert admits[2] >= dones[0] - 1e-6
    c.serve_stop()


def test_error_paths():
    c = ctx()
    with pytest.raises(B.DfxError) as e:
        c.serve_start(hbm_budget=1 << 20, max_slots=2, tol=TOL, max_iter=7, iters_per_round=-1)
    assert e.value.code == B.EINVAL
    c.serve_start(hbm_budget=1 << 20, max_slots=2, tol=TOL, max_iter=7)
    rp, col, val = synth.poisson_csr(200, 2)   # ~2.4 MB footprint
    with pytest.raises(B.DfxError) as e:
        c.serve_submit(rp, col, val, np.ones(200 * 200))
    assert e.value.code == B.ENOMEM_BUDGET
    rp, col, val = synth.poisson_csr(16, 2)
    bad = col.copy()
    bad[5] = 10 ** 6
    with pytest.raises(B.DfxError) as e:
        c.serve_submit(rp, bad, val, np.ones(256))
    assert e.value.code == B.EINVAL
    # iteration limit
    t = c.serve_submit(rp, col, val, synth.serve_rhs(7, 256))
    r = c.serve_wait(t, 60)
    assert r["status"] == B.SOLVE_MAXITER and r["iterations"] == 7
    # zero right-hand side: converged at x = 0 without iterating
    t = c.serve_submit(rp, col, val, np.zeros(256))
    r = c.serve_wait(t, 60)
    assert r["status"] == B.SOLVE_CONVERGED and r["iterations"] == 0
    assert not np.any(c.serve_read_x(t, 256))
    # non-finite right-hand side: breakdown is reported, nothing hangs
    b = np.ones(256)
    b[3] = np.nan
    t = c.serve_submit(rp, col, val, b)
    r = c.serve_wait(t, 60)
    assert r["status"] == B.SOLVE_BREAKDOWN
    c.serve_stop()
