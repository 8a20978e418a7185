"""The persistent batched executor (dfx_batch_*): many independent task
streams of uneven sizes in one launch.  Each stream is recorded from its own
context (Black-Scholes passes, Jacobi sweeps, CG iterations on Poisson
systems of different sizes) and must give bit for bit what the same stream
gives through the ordinary flush, and match the oracle at the elementwise and
reduction tolerances."""
import numpy as np
import pytest

import paper_2406_18109_amd as dfx
import synth
from gpu_util import note, rel_err_floor, upload
from oracle import workloads as wl

pytestmark = pytest.mark.gpu
TOL_ELEM = 1e-12
TOL_RED = 1e-10


class Job:
    """One task stream: set-up in a fresh context (ordinary flush), then the
    recorded (or solo-run) part, then the results read back."""

    def __init__(self, kind, size, reps):
        self.kind, self.size, self.reps = kind, size, reps

    def setup(self):
        c = dfx.Context(device=0, window_size=64 if self.kind == "bs" else 16)
        self.c = c
        if self.kind == "bs":
            n = self.size
            S, K, T = synth.bs_inputs(n)
            self.inp = (S, K, T)
            self.h = [upload(c, a) for a in (S, K, T)] + [upload(c, np.array(v)) for v in
                                                          (synth.BS_RATE, synth.BS_VOL)]
            self.h.append(dfx.apps.bs_drift(c, self.h[3], self.h[4]))
        elif self.kind == "jacobi":
            N = self.size
            self.grid0 = synth.jacobi_grid(N)
            self.G = upload(c, self.grid0)
            self.J = dfx.apps.Jacobi(c, self.G, N)
        else:
            m = self.size
            self.sysm = synth.poisson_csr(m, 2)
            self.b = synth.rhs(m * m, 6100 + m)
            self.cg = dfx.apps.CG(c, *[upload(c, a) for a in self.sysm + (self.b,)], m * m)
        c.flush()
        c.sync()

    def body(self, batch=None):
        """The stream proper: Black-Scholes passes, Jacobi sweeps (the
        program rebinds its names each sweep, so only the last residual
        stays readable), or CG iterations (recorded once as a repeated body
        when batched)."""
        c = self.c
        if self.kind == "bs":
            S, K, T, r, sig, rv = self.h
            for _ in range(self.reps):
                self.out = dfx.apps.black_scholes(c, S, K, T, r, sig, rv, self.size)
                c.flush()
        elif self.kind == "jacobi":
            self.res = [self.J.sweep() for _ in range(self.reps)]
        else:
            if batch is None:
                for _ in range(self.reps):
                    self.cg.iteration()
            else:
                batch.loop_begin(c)
                self.cg.iteration()

    def results(self):
        c = self.c
        if self.kind == "bs":
            n = self.size
            return [c.store_read(self.out[0], [n], "f64"), c.store_read(self.out[1], [n], "f64")]
        if self.kind == "jacobi":
            N = self.size
            return [c.store_read(self.G, [N, N], "f64"), c.store_read(self.res[-1], [], "f64")]
        n = self.size ** 2
        return [c.store_read(self.cg.x, [n], "f64"), c.store_read(self.cg.rho, [], "f64")]

    def oracle_check(self, got):
        if self.kind == "bs":
            S, K, T = self.inp
            oc, op = wl.black_scholes(S, K, T, *wl.bs_scalars(synth.BS_RATE, synth.BS_VOL))
            assert rel_err_floor(got[0], oc) <= TOL_ELEM and rel_err_floor(got[1], op) <= TOL_ELEM
        elif self.kind == "jacobi":
            g = self.grid0.copy()
            ss = [wl.jacobi_sweep(g) for _ in range(self.reps)]
            assert np.array_equal(got[0], g)
            assert abs(float(got[1]) - np.sqrt(ss[-1])) <= TOL_RED * np.sqrt(ss[-1])
        else:
            xo, ho = wl.cg(*self.sysm, self.b, self.reps)
            assert rel_err_floor(got[0], xo) <= TOL_ELEM
            assert abs(float(got[1]) - ho[-1]) <= TOL_RED * ho[-1]


def _jobs():
    # 72 streams of uneven sizes: Black-Scholes from one partial tile to 75
    # tiles, Jacobi grids from 10^2 to 300^2, CG from 5^2 to 150^2 (1 to 6
    # tiles per pass, 4 to 40 iterations)
    jobs = []
    for i in range(24):
        jobs.append(Job("bs", [77, 4096, 5000, 40000, 123457, 300001][i % 6] + 13 * i, 1 + i % 2))
    for i in range(24):
        jobs.append(Job("jacobi", [10, 35, 66, 130, 200, 300][i % 6] + i, 1 + i % 3))
    for i in range(24):
        jobs.append(Job("cg", [5, 16, 40, 64, 100, 150][i % 6] + i, 4 + (7 * i) % 37))
    return jobs


def test_batch_streams_equal_solo_and_oracle():
    jobs = _jobs()
    note("batch: solo runs of %d streams" % len(jobs))
    solo = []
    for j in jobs:
        j.setup()
        j.body()
        solo.append(j.results())
        j.c.close()
    note("batch: recording")
    b = dfx.Batch(device=0)
    sids = []
    for j in jobs:
        j.setup()
        b.record_begin(j.c)
        j.body(b)
        sids.append(b.record_end(j.c, max_iter=j.reps if j.kind == "cg" else 0))
    cnt = b.counts()
    assert cnt["streams"] == len(jobs)
    note("batch: one launch, %s" % cnt)
    b.run()
    b.wait()
    for j, sid, ref in zip(jobs, sids, solo):
        it, st = b.stream_info(sid)
        assert st == dfx.Batch.DONE
        if j.kind == "cg":
            assert it == j.reps
        got = j.results()
        for g, r in zip(got, ref):
            assert np.array_equal(g, r), (j.kind, j.size)
        j.oracle_check(got)
    b.close()
    for j in jobs:
        j.c.close()


def test_batch_cg_stops_at_tolerance():
    """A repeated CG body with a convergence test stops each stream at its own
    iteration count: the first k with rho_k <= tol^2 rho_0, as the oracle's
    CG with the same rule."""
    sides = [12, 20, 33, 47]
    b = dfx.Batch(device=0)
    ctxs, cgs, sids, rho0 = [], [], [], []
    for m in sides:
        c = dfx.Context(device=0, window_size=16)
        sysm = synth.poisson_csr(m, 2)
        bb = synth.rhs(m * m, 6300 + m)
        cg = dfx.apps.CG(c, *[upload(c, a) for a in sysm + (bb,)], m * m)
        r0 = c.store_create([], "f64")
        c.submit("copy", [], [(cg.rho, c.part_none(), "R"), (r0, c.part_none(), "W")])
        c.flush()
        c.sync()
        b.record_begin(c)
        b.loop_begin(c)
        cg.iteration()
        sids.append(b.record_end(c, max_iter=2000, conv_a=cg.rho, conv_b=r0, tol=1e-16))
        ctxs.append((c, sysm, bb))
        cgs.append(cg)
    b.run()
    b.wait()
    for (c, sysm, bb), cg, sid in zip(ctxs, cgs, sids):
        it, st = b.stream_info(sid)
        assert st == dfx.Batch.DONE
        _, ho = wl.cg(*sysm, bb, 2000, tol=1e-8)
        k_oracle = len(ho) - 1
        assert abs(it - k_oracle) <= 1, (it, k_oracle)
        xo, _ = wl.cg(*sysm, bb, it)
        n = sysm[0].size - 1
        assert rel_err_floor(c.store_read(cg.x, [n], "f64"), xo) <= TOL_ELEM
        c.close()
    b.close()
