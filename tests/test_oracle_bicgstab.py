"""Pins for the oracle's BiCGSTAB (van der Vorst 1992; the further Krylov
method of the evaluation's task-count table).

Independent checks: SciPy's bicgstab (the same published recurrence, its own
code) iterate by iterate, convergence to SciPy's direct solve on a
nonsymmetric system, and the recurrence residual against b - A x at every
step (a dropped or mis-signed update of x or r breaks it)."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import workloads as wl


def _mat(rowptr, col, val):
    n = rowptr.size - 1
    return sp.csr_matrix((val, col, rowptr), shape=(n, n))


def _systems():
    yield "convdiff 2-D 12", synth.convdiff_csr(12, 2), synth.rhs(144, 4001)
    yield "poisson 3-D 6", synth.poisson_csr(6, 3), synth.rhs(216, 4002)
    yield "convdiff 3-D 5", synth.convdiff_csr(5, 3, 1.25), synth.rhs(125, 4003)


def test_matches_scipy_iterates():
    k = 6
    for name, (rowptr, col, val), b in _systems():
        its = []
        _, info = spla.bicgstab(_mat(rowptr, col, val), b, rtol=0.0, atol=0.0, maxiter=k,
                                callback=lambda xk: its.append(xk.copy()))
        assert info == k and len(its) == k, name
        for j in range(1, k + 1):
            x, _ = wl.bicgstab(rowptr, col, val, b, j)
            err = np.max(np.abs(x - its[j - 1])) / np.max(np.abs(its[j - 1]))
            assert err <= 1e-11, (name, j, err)


def test_converges_to_direct_solve_nonsymmetric():
    m = 16
    rowptr, col, val = synth.convdiff_csr(m, 2)
    A = _mat(rowptr, col, val)
    assert abs(A - A.T).max() > 0
    b = synth.rhs(m * m, 4004)
    x, hist = wl.bicgstab(rowptr, col, val, b, 60)
    xd = spla.spsolve(A.tocsc(), b)
    assert np.sqrt(hist[-1]) <= 1e-14 * np.sqrt(hist[0])
    assert np.max(np.abs(x - xd)) <= 1e-9 * np.max(np.abs(xd))


def test_recurrence_residual_is_true_residual():
    rowptr, col, val = synth.convdiff_csr(10, 2)
    A = _mat(rowptr, col, val)
    b = synth.rhs(100, 4005)
    _, hist = wl.bicgstab(rowptr, col, val, b, 8)
    assert hist[0] == float(np.dot(b, b)) or abs(hist[0] - np.dot(b, b)) <= 1e-15 * np.dot(b, b)
    for k in range(1, 9):
        xk, _ = wl.bicgstab(rowptr, col, val, b, k)
        true = b - A @ xk
        assert abs(hist[k] - np.dot(true, true)) <= 1e-9 * hist[k] + 1e-28 * hist[0], k


def _planted(old, new):
    """The oracle's bicgstab with one plausible mistake written into it."""
    import inspect
    import textwrap
    from oracle import cnum
    src = textwrap.dedent(inspect.getsource(wl.bicgstab))
    assert src.count(old) == 1, old
    ns = {"np": np, "cnum": cnum}
    exec(compile(src.replace(old, new), "<planted>", "exec"), ns)
    return ns["bicgstab"]


def test_pins_catch_planted_mistakes():
    """Each mistake (a dropped term, a wrong sign, a dropped factor, a
    swapped operand) makes the SciPy-iterate pin fail."""
    rowptr, col, val = synth.convdiff_csr(12, 2)
    b = synth.rhs(144, 4001)
    its = []
    spla.bicgstab(_mat(rowptr, col, val), b, rtol=0.0, atol=0.0, maxiter=4,
                  callback=lambda xk: its.append(xk.copy()))
    mistakes = [("x = (x + alpha * p) + omega * s", "x = x + alpha * p"),
                ("r = s - omega * t", "r = s + omega * t"),
                ("beta = (rho_new / rho) * (alpha / omega)", "beta = rho_new / rho"),
                ("omega = cnum.fsum_prod(t, s) / cnum.fsum_prod(t, t)",
                 "omega = cnum.fsum_prod(t, s) / cnum.fsum_prod(s, s)")]
    for old, new in mistakes:
        bad = _planted(old, new)
        errs = []
        for j in range(1, 5):
            x, _ = bad(rowptr, col, val, b, j)
            errs.append(np.max(np.abs(x - its[j - 1])) / np.max(np.abs(its[j - 1])))
        assert max(errs) > 1e-6, (new, errs)
