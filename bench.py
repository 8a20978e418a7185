#!/usr/bin/env python3
"""Benchmark of the fused task-window executor on one MI355X.

Headline workload: Black-Scholes over 2^26 options in FP64.  A step is one
pass of the whole hot path over that batch: 28 index tasks submitted through
the C ABI, the window analysed (memoised after the first pass), and the fused
group executed as one kernel.  Inputs are resident in HBM before timing.

Printed: one JSON line with the headline (fused algorithmic HBM GB/s), the
roofline of the dominant kernel, the CPU oracle timed on a bounded sample,
and the other legs of the metric (unfused GB/s, FP32, Jacobi stencil, CG
and BiCGSTAB iterations/s, multigrid-preconditioned CG iterations/s, and the continuous-batching server: its closed-loop saturation
solves/s, then p50/p99 latency with Poisson arrivals at 0.5, 0.8 and 0.95 of
saturation, the 0.8 point over the whole 4096-request stream) under "legs".
Progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


# --tune: contexts time launch-shape candidates on each plan's first
# executions (then every leg warms up for at least 8 executions)
TUNE = False
# compiled passes: 1 = background compilation (the default), 0 = every pass
# interpreted.  Legs wait for the compiler before their timed region and
# report its time (compile_s) apart from the first iteration.
JIT = 1


def jit_settle(dfx, step):
    """Wait for queued kernel compilation, then run one more untimed step so
    every compiled kernel is loaded before timing; returns the compile
    seconds spent so far in this process."""
    if JIT:
        dfx.jit_wait()
        step()
    return dfx.jit_info()["compile_seconds"] if JIT else 0.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("paper_2406_18109_amd/csrc/kernels.hip", "paper_2406_18109_amd/csrc/vm.h",
              "paper_2406_18109_amd/csrc/vm_exec.h", "paper_2406_18109_amd/csrc/dev_common.h",
              "paper_2406_18109_amd/csrc/vm_tier0.hip", "paper_2406_18109_amd/csrc/vm_tier1.hip",
              "paper_2406_18109_amd/csrc/vm_tier2.hip", "paper_2406_18109_amd/csrc/vm_tier3.hip",
              "paper_2406_18109_amd/csrc/dmath.h", "paper_2406_18109_amd/csrc/dmath_coef.h",
              "paper_2406_18109_amd/csrc/vm_instr.inc", "paper_2406_18109_amd/csrc/jit.cpp"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name, per_launch_alg):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    e = d.get(name)
    if not e or e.get("kernel_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def timed_steps(torch, stream, step, K):
    """Run K steps between synchronisations; return (wall ms per step, list of
    per-step event ms on the executor's stream)."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        evs[i][0].record(stream)
        step()
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / K
    return wall, [a.elapsed_time(b) for a, b in evs]


# FP64 VALU issue peak: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz lane-
# instructions per second (an FMA is one instruction, two flops: 78.6 TFLOP/s)
VALU_PEAK_LANE_INSTR = 256 * 4 * 16 * 2.4e9


def alu_roof(n, kernel_s):
    """The ALU roof of the Black-Scholes FP64 pass from the committed counter
    summary (profiles/traffic.json, taken on the current kernel source):
    `valu_per_option` is what the dominant kernel, the compiled pass, executes
    (SQ_INSTS_VALU x 64 / options).  A compiled pass runs the chain as
    straight-line code, so this is the pass's own arithmetic plus the tiling's
    address and mask work.  Floor at the VALU issue peak, and the achieved
    issue rate.  None without a current summary."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        e = json.load(fh).get("bs_f64_fused")
    if not e or e.get("kernel_hash") != kernel_source_hash() or "valu_per_option" not in e:
        return None
    cnt = e["valu_per_option"]
    ach = cnt * n / kernel_s
    out = {"unit": "T lane-instr/s", "peak": round(VALU_PEAK_LANE_INSTR / 1e12, 2),
           "valu_per_option": cnt, "valu_floor_ms": round(cnt * n / VALU_PEAK_LANE_INSTR * 1e3, 4),
           "achieved": round(ach / 1e12, 3), "frac": round(ach / VALU_PEAK_LANE_INSTR, 4)}
    if "salu_per_option" in e:
        out["salu_per_option"] = e["salu_per_option"]
    return out


class BSBench:
    def __init__(self, dfx, synth, np, n, dtype, fuse):
        self.np = np
        npdt = np.float64 if dtype == "f64" else np.float32
        self.ctx = dfx.Context(device=0, window_size=64, fuse=fuse, tune=TUNE, jit=JIT)
        self.dfx, self.n, self.dtype = dfx, n, dtype
        S, K, T = synth.bs_inputs(n, npdt)
        c = self.ctx
        self.h = []
        for a in (S, K, T):
            s = c.store_create([n], dtype)
            c.store_write(s, a)
            self.h.append(s)
        for v in (synth.BS_RATE, synth.BS_VOL):
            s = c.store_create([], dtype)
            c.store_write(s, np.array(v, dtype=npdt))
            self.h.append(s)
        # rv = r + sigma^2/2 as single tasks, once, before the pricing steps
        self.h.append(dfx.apps.bs_drift(c, self.h[3], self.h[4], dtype))
        c.flush()
        self.out = None
        del S, K, T

    def step(self):
        c = self.ctx
        if self.out:
            c.store_release(self.out[0])
            c.store_release(self.out[1])
        S, K, T, r, sig, rv = self.h
        self.out = self.dfx.apps.black_scholes(c, S, K, T, r, sig, rv, self.n, self.dtype)
        c.flush()

    def close(self):
        self.ctx.close()


def paper_mean(times):
    """The paper's timing method: drop the fastest and the slowest run,
    average the rest (12 runs -> mean of 10)."""
    t = sorted(times)
    if len(t) > 2:
        t = t[1:-1]
    return sum(t) / len(t)


def counts(st, units):
    """Per-unit task and group counts (the paper's task-count table: tasks per
    iteration issued, fused tasks dispatched) and launches."""
    return {"tasks_per_iter": st["tasks_dispatched"] / units, "groups_per_iter": st["groups_dispatched"] / units,
            "launches_per_iter": st["launches"] / units}


def bs_leg(torch, dfx, synth, np, n, dtype, fuse, K, W, runs=0):
    t0 = time.perf_counter()
    b = BSBench(dfx, synth, np, n, dtype, fuse)
    setup = time.perf_counter() - t0
    # the first pass: analysis, lowering and the plan's first launch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step()
    torch.cuda.synchronize()
    first = time.perf_counter() - t0
    analysis = b.ctx.stats()["analysis_seconds"]
    for _ in range(max(W, 8) if TUNE else W):
        b.step()
    c0 = dfx.jit_info()["compile_seconds"]
    compile_s = jit_settle(dfx, b.step) - c0 if JIT else 0.0
    b.ctx.stats_reset()
    wall, ev = timed_steps(torch, b.ctx.torch_stream, b.step, K)
    st = b.ctx.stats()
    bytes_per_step = st["alg_bytes"] / K
    launches = st["launches"] / K
    paper = None
    if runs:
        paper = paper_mean([timed_steps(torch, b.ctx.torch_stream, b.step, 10)[0] for _ in range(runs)])
    b.close()
    ev_ms = sum(ev) / len(ev)
    out = {"ms_per_step": wall, "event_ms_per_step": ev_ms, "alg_bytes_per_step": bytes_per_step,
           "launches_per_step": launches, "gbs": bytes_per_step / (wall * 1e-3) / 1e9,
           "kernel_gbs": bytes_per_step / (ev_ms * 1e-3) / 1e9, "first_pass_ms": first * 1e3,
           "analysis_s": analysis, "tasks_per_pass": st["tasks_dispatched"] / K,
           "groups_per_pass": st["groups_dispatched"] / K, "jit": JIT, "compile_s": compile_s,
           "compiled_launches_per_pass": st["compiled_launches"] / K}
    if paper is not None:
        out["paper_method_ms_per_step"] = paper
    return out


def jacobi_leg(torch, dfx, synth, np, N, sweeps, fuse):
    c = dfx.Context(device=0, window_size=16, fuse=fuse, tune=TUNE, jit=JIT)
    c0 = dfx.jit_info()["compile_seconds"]
    G = c.store_create([N, N], "f64")
    c.store_write(G, synth.jacobi_grid(N))
    J = dfx.apps.Jacobi(c, G, N)
    c.sync()
    t0 = time.perf_counter()
    J.sweep()
    c.sync()
    first = time.perf_counter() - t0
    for _ in range(8 if TUNE else 2):
        J.sweep()
    compile_s = jit_settle(dfx, J.sweep) - c0 if JIT else 0.0
    c.sync()
    c.stats_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(sweeps):
        J.sweep()
    c.sync()
    dt = (time.perf_counter() - t0) / sweeps
    st = c.stats()
    out = {"sweeps": sweeps, "ms_per_sweep": dt * 1e3, "alg_bytes_per_sweep": st["alg_bytes"] / sweeps,
           "gbs": st["alg_bytes"] / sweeps / dt / 1e9, "launches_per_sweep": st["launches"] / sweeps,
           "first_sweep_ms": first * 1e3, "jit": JIT, "compile_s": compile_s,
           "compiled_launches_per_sweep": st["compiled_launches"] / sweeps}
    out.update(counts(st, sweeps))
    c.close()
    return out


def cg_leg(torch, dfx, synth, np, m, dim, iters, fuse, graph, solver="cg", runs=0):
    """CG on the Poisson matrix, or BiCGSTAB (solver="bicgstab") on the
    nonsymmetric convection-diffusion matrix of the same shape.  With
    `runs`, the timed region is repeated that many times and the paper's
    method (drop fastest and slowest, mean of the rest) gives ms_per_iter."""
    c = dfx.Context(device=0, window_size=16, fuse=fuse, tune=TUNE, jit=JIT)
    c0 = dfx.jit_info()["compile_seconds"]
    if solver == "cg":
        rowptr, col, val = synth.poisson_csr(m, dim)
        seed = synth.CG64_SEED if dim == 2 else synth.CG256_SEED
    else:
        rowptr, col, val = synth.convdiff_csr(m, dim)
        seed = synth.BICG256_SEED
    n = m ** dim
    b = synth.rhs(n, seed)
    hs = []
    for a, dt in ((rowptr, "i32"), (col, "i32"), (val, "f64"), (b, "f64")):
        s = c.store_create(list(a.shape), dt)
        c.store_write(s, a)
        hs.append(s)
    del rowptr, col, val
    cg = (dfx.apps.CG if solver == "cg" else dfx.apps.BiCGSTAB)(c, *hs, n)
    c.sync()
    # first iteration: analysis and lowering of every window (memo misses),
    # workspaces, first launches
    t0 = time.perf_counter()
    cg.iteration()
    c.sync()
    first = time.perf_counter() - t0
    analysis = c.stats()["analysis_seconds"]
    for _ in range(8 if TUNE else 1):
        cg.iteration()
    compile_s = jit_settle(dfx, cg.iteration) - c0 if JIT else 0.0
    c.sync()
    g = None
    capture = None
    if graph:
        t0 = time.perf_counter()
        c.graph_begin()
        cg.iteration()
        g = c.graph_end()
        capture = time.perf_counter() - t0
    c.sync()

    def region():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(iters):
            if g is not None:
                c.graph_launch(g)
            else:
                cg.iteration()
        c.sync()
        return (time.perf_counter() - t0) / iters

    c.stats_reset()
    dt = region()
    st = c.stats()
    out = {"iters": iters, "iters_per_s": 1.0 / dt, "ms_per_iter": dt * 1e3,
           "alg_bytes_per_iter": st["alg_bytes"] / iters,
           "gbs": st["alg_bytes"] / iters / dt / 1e9, "first_iter_ms": first * 1e3, "analysis_s": analysis,
           "jit": JIT, "compile_s": compile_s, "compiled_launches_per_iter": st["compiled_launches"] / iters}
    out.update(counts(st, iters))
    if capture is not None:
        out["capture_ms"] = capture * 1e3
        # graph replays do not submit tasks: take the counts from one eager iteration
        c.stats_reset()
        cg.iteration()
        c.sync()
        st1 = c.stats()
        out["tasks_per_iter"] = st1["tasks_dispatched"]
        out["groups_per_iter"] = st1["groups_dispatched"]
    if runs:
        times = [region() for _ in range(runs)]
        out["paper_method_ms_per_iter"] = paper_mean(times) * 1e3
        out["paper_method_iters_per_s"] = 1.0 / paper_mean(times)
    if g is not None:
        c.graph_destroy(g)
    c.close()
    return out


def gmg_leg(torch, dfx, synth, np, m, nlev, iters, fuse, graph, runs=0):
    """The GMG solver (CG preconditioned by one V(2,2) cycle, injection
    restriction, weighted Jacobi) on the m^2 Poisson problem over nlev
    levels; with graph, one whole iteration is recorded and replayed."""
    c = dfx.Context(device=0, window_size=16, fuse=fuse, tune=TUNE, jit=JIT)
    c0 = dfx.jit_info()["compile_seconds"]
    levels = synth.gmg_levels(m, nlev)

    def up(a):
        s = c.store_create(list(a.shape), "i32" if a.dtype == np.int32 else "f64")
        c.store_write(s, a)
        return s
    lev = [(tuple(up(a) for a in A), diag, None if R is None else tuple(up(a) for a in R),
            None if P is None else tuple(up(a) for a in P)) for A, diag, R, P in levels]
    sizes = [A[0].size - 1 for A, _, _, _ in levels]
    del levels
    g = dfx.apps.GMG(c, lev, sizes, up(synth.rhs(m * m, synth.GMG_SEED)))
    c.sync()
    t0 = time.perf_counter()
    g.iteration()
    c.sync()
    first = time.perf_counter() - t0
    compile_s = jit_settle(dfx, g.iteration) - c0 if JIT else 0.0
    gid = None
    capture = None
    if graph:
        t0 = time.perf_counter()
        c.graph_begin()
        g.iteration()
        gid = c.graph_end()
        capture = time.perf_counter() - t0
    c.sync()

    def region():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(iters):
            if gid is not None:
                c.graph_launch(gid)
            else:
                g.iteration()
        c.sync()
        return (time.perf_counter() - t0) / iters

    c.stats_reset()
    dt = region()
    st = c.stats()
    out = {"iters": iters, "iters_per_s": 1.0 / dt, "ms_per_iter": dt * 1e3,
           "alg_bytes_per_iter": st["alg_bytes"] / iters,
           "gbs": st["alg_bytes"] / iters / dt / 1e9, "first_iter_ms": first * 1e3,
           "jit": JIT, "compile_s": compile_s, "compiled_launches_per_iter": st["compiled_launches"] / iters}
    out.update(counts(st, iters))
    if capture is not None:
        out["capture_ms"] = capture * 1e3
        c.stats_reset()
        g.iteration()
        c.sync()
        st1 = c.stats()
        out["tasks_per_iter"] = st1["tasks_dispatched"]
        out["groups_per_iter"] = st1["groups_dispatched"]
    if runs:
        times = [region() for _ in range(runs)]
        out["paper_method_ms_per_iter"] = paper_mean(times) * 1e3
    if gid is not None:
        c.graph_destroy(gid)
    c.close()
    return out


def breakeven(fused, unfused, key_ms, first_key):
    """One-time cost of fusion (first fused iteration, which analyses and
    lowers every window, plus the graph capture, less one steady fused
    iteration), and the iterations after which the fused run is ahead of
    the unfused one, which pays its own first-iteration cost (the paper's
    warm-up and breakeven table)."""
    f_ss, u_ss = fused[key_ms], unfused[key_ms]
    extra = (fused[first_key] + fused.get("capture_ms", 0.0) - f_ss) - (unfused[first_key] - u_ss)
    gain = u_ss - f_ss
    out = {"one_time_ms_fused": fused[first_key] + fused.get("capture_ms", 0.0) - f_ss,
           "one_time_ms_unfused": unfused[first_key] - u_ss,
           "gain_ms_per_iter": gain,
           "breakeven_iters": (max(0.0, extra) / gain) if gain > 0 else None}
    # kernel compilation runs on a host thread while the passes run
    # interpreted; counted as one-time cost it moves the breakeven to
    cf, cu = fused.get("compile_s", 0.0) * 1e3, unfused.get("compile_s", 0.0) * 1e3
    if cf or cu:
        out["compile_ms_fused"], out["compile_ms_unfused"] = cf, cu
        out["breakeven_iters_with_compile"] = (max(0.0, extra + cf - cu) / gain) if gain > 0 else None
    return out


def serve_leg(dfx, synth, np, count, rate, budget, slots, ipr=0, mats=None):
    """Continuous-batching server on the first `count` requests of the serving
    stream: 2-D Poisson solves, side uniform in [32, 512], tol 1e-8, Poisson
    arrivals at `rate` per second (None: every request submitted at once, the
    closed-loop saturation run).  Latency = completion - arrival."""
    import threading
    sides = synth.serve_sides(count)
    arrivals = np.zeros(count) if rate is None else synth.serve_arrivals(count, rate)
    if mats is None:
        mats = {int(s): synth.poisson_csr(int(s), 2) for s in set(sides.tolist())}
    c = dfx.Context(device=0)
    c.serve_start(hbm_budget=budget, max_slots=slots, tol=1e-8, max_iter=20000, iters_per_round=ipr)
    tickets = [None] * count

    def feeder():
        t0 = time.perf_counter()
        for i in range(count):
            side = int(sides[i])
            b = synth.serve_rhs(i, side * side)
            d = arrivals[i] - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            rp, col, val = mats[side]
            tickets[i] = c.serve_submit(rp, col, val, b)

    t_start = time.perf_counter()
    th = threading.Thread(target=feeder)
    th.start()
    th.join()
    res = []
    for i, t in enumerate(tickets):
        res.append(c.serve_wait(t, 3600))
        c.serve_release(t)
        if i % 256 == 255 or i == count - 1:
            log("serve: %d of %d requests done" % (i + 1, count))
    wall = time.perf_counter() - t_start
    st = c.serve_stats()
    c.serve_stop()
    c.close()
    lat = np.array([r["t_done"] - r["t_arrive"] for r in res])
    its = np.array([r["iterations"] for r in res])
    ok = sum(1 for r in res if r["status"] == 2)
    return {"requests": count, "converged": ok, "arrival_rate_per_s": rate, "solves_per_s": count / wall,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_iterations": float(its.mean()), "rounds": st["rounds"], "launches": st["launches"],
            "iters_per_round": ipr,
            "peak_bytes": st["peak_bytes"], "hbm_budget": budget, "max_slots": slots, "wall_s": wall}


SERVE_LOADS = (0.5, 0.8, 0.95)


def batch_leg(dfx, synth, np, count, slots, budget):
    """The serving stream's first `count` solves run as task streams of the
    persistent batched executor: each solve's CG set-up in its own context,
    one CG iteration recorded as a repeated body that stops at
    rho_k <= 1e-16 rho_0 (||r_k|| <= 1e-8 ||b||), every stream in one
    launch.  Beside it the round-based server on the same requests, all
    submitted at once (closed loop)."""
    sides = synth.serve_sides(count)
    mats = {int(s): synth.poisson_csr(int(s), 2) for s in set(sides.tolist())}
    b = dfx.Batch(device=0)
    ctxs = []
    t0 = time.perf_counter()
    for i in range(count):
        side = int(sides[i])
        c = dfx.Context(device=0, window_size=16)
        rp, col, val = mats[side]
        hs = []
        for a, dt in ((rp, "i32"), (col, "i32"), (val, "f64"), (synth.serve_rhs(i, side * side), "f64")):
            h = c.store_create(list(a.shape), dt)
            c.store_write(h, a)
            hs.append(h)
        cg = dfx.apps.CG(c, *hs, side * side)
        r0 = c.store_create([], "f64")
        none = c.part_none()
        c.submit("copy", [], [(cg.rho, none, "R"), (r0, none, "W")])
        c.flush()
        b.record_begin(c)
        b.loop_begin(c)
        cg.iteration()
        b.record_end(c, max_iter=20000, conv_a=cg.rho, conv_b=r0, tol=1e-16)
        ctxs.append((c, cg))
    setup = time.perf_counter() - t0
    cnt = b.counts()
    t0 = time.perf_counter()
    b.run()   # one launch solves every stream (a second run would resume from the solutions)
    b.wait()
    wall = time.perf_counter() - t0
    its = [b.stream_info(i)[0] for i in range(count)]
    done = sum(1 for i in range(count) if b.stream_info(i)[1] == dfx.Batch.DONE)
    b.close()
    for c, _ in ctxs:
        c.close()
    out = {"requests": count, "converged": done, "solves_per_s": count / wall, "wall_s": wall,
           "mean_iterations": float(np.mean(its)), "max_iterations": int(np.max(its)),
           "record_s": setup, "streams": cnt["streams"], "passes": cnt["passes"], "grid": cnt["grid"]}
    log("batch", out)
    srv = serve_leg(dfx, synth, np, count, None, budget, slots, 0, mats)
    out["server_closed_loop_solves_per_s"] = srv["solves_per_s"]
    out["speedup_vs_server"] = out["solves_per_s"] / srv["solves_per_s"]
    return out


def serve_sweep(dfx, synth, np, count, budget, slots, ipr=0):
    """Saturation throughput from a closed-loop run (all requests at once),
    then Poisson arrivals at 0.5, 0.8 and 0.95 of it; the leg's p50/p99 are
    those at 0.8, over the whole stream.  The saturation run and the 0.5 and
    0.95 points use the stream's first 1024 requests (GPU time)."""
    sides = synth.serve_sides(count)
    mats = {int(s): synth.poisson_csr(int(s), 2) for s in set(sides.tolist())}
    short = min(count, 1024)
    log("serve: closed loop, %d requests" % short)
    sat = serve_leg(dfx, synth, np, short, None, budget, slots, ipr, mats)
    out = {"saturation_solves_per_s": sat["solves_per_s"], "closed_loop": sat, "loads": {}}
    for f in SERVE_LOADS:
        rate = f * sat["solves_per_s"]
        n = count if f == 0.8 else short
        log("serve: %d requests, arrivals at %.2f of saturation (%.1f/s)" % (n, f, rate))
        out["loads"]["%.2f" % f] = serve_leg(dfx, synth, np, n, rate, budget, slots, ipr, mats)
    main = out["loads"]["0.80"]
    for k in ("requests", "converged", "arrival_rate_per_s", "solves_per_s", "p50_latency_s", "p99_latency_s",
              "mean_iterations", "hbm_budget", "max_slots", "peak_bytes"):
        out[k] = main[k]
    out["load"] = 0.8
    return out


def copy_leg(dfx, np, torch, n, K):
    """One COPY task over n doubles per step (reads and writes 8n bytes each):
    the streaming reference, and the known-size kernel that calibrates the
    HBM traffic counters."""
    c = dfx.Context(device=0, window_size=4, tune=TUNE)
    a = c.store_create([n], "f64")
    c.store_write(a, np.zeros(n))
    b = c.store_create([n], "f64")
    T = c.part_tiling([n])

    def step():
        c.submit("copy", [1], [(a, T, "R"), (b, T, "W")])
        c.flush()
    for _ in range(8 if TUNE else 2):
        step()
    wall, ev = timed_steps(torch, c.torch_stream, step, K)
    c.close()
    ev_ms = sum(ev) / len(ev)
    return {"elements": n, "ms_per_step": wall, "event_ms_per_step": ev_ms,
            "gbs": 16.0 * n / (ev_ms * 1e-3) / 1e9}


# ---- the oracle on the host's cores ------------------------------------------
# Timed before anything touches the GPU.  Single-thread: the oracle as it
# stands.  All-core: the same oracle functions run unchanged by a pool of
# forked workers over fixed chunks of the same workload (elementwise work
# split by index ranges, Jacobi by row blocks with their halo rows, CG's SpMV
# by row blocks); the chunk results are not combined, only timed.
_POOL_DATA = {}


def _host_info():
    import platform
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return n, model


def _bs_chunk(i):
    from oracle import workloads as wl
    S, K, T, sc, P = (_POOL_DATA[k] for k in ("S", "K", "T", "sc", "P"))
    m = S.size // P
    sl = slice(i * m, (i + 1) * m)
    wl.black_scholes(S[sl], K[sl], T[sl], *sc)
    return i


def _jac_chunk(i):
    from oracle import workloads as wl
    G, P = _POOL_DATA["G"], _POOL_DATA["P"]
    N = G.shape[0]
    rows = (N - 2 + P - 1) // P
    r0 = 1 + i * rows
    r1 = min(N - 1, r0 + rows)
    sub = G[r0 - 1:r1 + 1].copy()   # the block's interior rows and one halo row each side
    wl.jacobi_sweep(sub)
    return i


def _spmv_chunk(i):
    from oracle import cnum
    rp, col, val, x, P = (_POOL_DATA[k] for k in ("rp", "col", "val", "x", "P"))
    n = rp.size - 1
    rows = (n + P - 1) // P
    r0, r1 = i * rows, min(n, (i + 1) * rows)
    lo, hi = int(rp[r0]), int(rp[r1])
    cnum.spmv((rp[r0:r1 + 1] - lo).astype(np.int32), col[lo:hi], val[lo:hi], x)
    return i


def _timed(fn, reps):
    """Median wall time of `reps` calls after one untimed call."""
    fn()
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        t.append(time.perf_counter() - t0)
    t.sort()
    return t[len(t) // 2]


def cpu_baselines(quick=False):
    """The oracle timed on this host: Black-Scholes (GB/s of the fused pass's
    algorithmic bytes), one Jacobi sweep of the 8192^2 grid, one CG
    iteration on 256^3; single-thread and all-core (at most 16 workers, the
    box's CPU share for one GPU)."""
    import multiprocessing as mp
    import numpy as _np
    global np
    np = _np
    import synth
    from oracle import cnum
    from oracle import workloads as wl
    ncpu, model = _host_info()
    P = max(1, min(16, ncpu))
    out = {"host_cpus": ncpu, "cpu_model": model, "workers": P}
    # Black-Scholes: 2^21 options single-thread; P chunks of 2^21 all-core
    n1 = 1 << 21
    S, K, T = synth.bs_inputs(n1 * P)
    sc = wl.bs_scalars(synth.BS_RATE, synth.BS_VOL)
    reps = 2 if quick else 5
    t1 = _timed(lambda: wl.black_scholes(S[:n1], K[:n1], T[:n1], *sc), reps)
    ctx = mp.get_context("fork")

    def all_core(fn):
        # workers forked after the workload's data is in place (copy on write)
        with ctx.Pool(P) as pool:
            return _timed(lambda: pool.map(fn, range(P)), reps_big)

    reps_big = 1 if quick else 2
    _POOL_DATA.update(S=S, K=K, T=T, sc=sc, P=P)
    with ctx.Pool(P) as pool:
        tp = _timed(lambda: pool.map(_bs_chunk, range(P)), reps)
    out["bs_f64"] = {"options_single": n1, "gbs_single": 40.0 * n1 / t1 / 1e9,
                     "options_all": n1 * P, "gbs_all": 40.0 * n1 * P / tp / 1e9}
    log("cpu: black-scholes", out["bs_f64"])
    del S, K, T
    _POOL_DATA.clear()
    # Jacobi: one sweep of 8192^2 (each timed call starts from a copy of the grid)
    N = 1024 if quick else 8192
    G = synth.jacobi_grid(N)
    tj1 = _timed(lambda: wl.jacobi_sweep(G.copy()), reps_big)
    _POOL_DATA.update(G=G, P=P)
    tjp = all_core(_jac_chunk)
    out["jacobi_sweep"] = {"grid": N, "ms_single": tj1 * 1e3, "ms_all": tjp * 1e3}
    log("cpu: jacobi", out["jacobi_sweep"])
    del G
    _POOL_DATA.clear()
    # CG on 256^3: the set-up and first iteration single-thread; its SpMV
    # single-thread and all-core
    m = 64 if quick else 256
    rp, col, val = synth.poisson_csr(m, 3)
    b = synth.rhs(m ** 3, synth.CG256_SEED)
    tc1 = _timed(lambda: wl.cg(rp, col, val, b, 1), reps_big)
    ts1 = _timed(lambda: cnum.spmv(rp, col, val, b), reps_big)
    _POOL_DATA.update(rp=rp, col=col, val=val, x=b, P=P)
    tsp = all_core(_spmv_chunk)
    out["cg256_iteration"] = {"side": m, "setup_and_first_iteration_ms_single": tc1 * 1e3,
                              "spmv_ms_single": ts1 * 1e3, "spmv_ms_all": tsp * 1e3}
    log("cpu: cg", out["cg256_iteration"])
    _POOL_DATA.clear()
    return out


def serve_main(dfx, synth, np, args):
    budget = int(args.serve_budget_gb * (1 << 30))
    if args.serve_rate is None:
        return serve_sweep(dfx, synth, np, args.serve_requests, budget, args.serve_slots, args.serve_iters_per_round)
    return serve_leg(dfx, synth, np, args.serve_requests, args.serve_rate, budget, args.serve_slots,
                     args.serve_iters_per_round)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--tune", action="store_true",
                    help="enable the library's launch-shape tuner (warm-ups extended to 8 executions)")
    ap.add_argument("--legs", default="all",
                    help="all | headline | serve | copy | comma-separated bs_f64,bs_f32,jacobi,cg64,cg256,bicgstab256,gmg,batch,serve")
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--batch-requests", type=int, default=256,
                    help="serving solves run by the batched executor in one launch")
    ap.add_argument("--serve-rate", type=float, default=None,
                    help="fixed Poisson arrival rate; default: a saturation run, then 0.5/0.8/0.95 of it")
    ap.add_argument("--serve-slots", type=int, default=256)
    ap.add_argument("--serve-budget-gb", type=float, default=4.0)
    ap.add_argument("--serve-iters-per-round", type=int, default=0,
                    help="CG iterations per scheduling round (0: the library default)")
    ap.add_argument("--log2n", type=int, default=26)
    ap.add_argument("--jacobi-sweeps", type=int, default=200, help="fused Jacobi sweeps timed (the config's 200)")
    ap.add_argument("--cg256-iters", type=int, default=500, help="CG 256^3 iterations timed (the config's 500)")
    ap.add_argument("--jit", type=int, default=1, choices=[0, 1],
                    help="1: passes compiled in the background (timed once ready); 0: interpreted")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timings on the host")
    ap.add_argument("--quick-cpu", action="store_true", help="small oracle samples (a smoke run of the bench)")
    args = ap.parse_args()
    global TUNE, JIT
    TUNE = args.tune
    JIT = args.jit
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported (the executor runs on "
              "a single device)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np

    n = 1 << args.log2n
    K, W = args.steps, args.warmup
    cpu = None
    if args.legs not in ("copy", "serve") and not args.no_cpu:
        # before anything touches the GPU: the pool's workers are forked
        log("cpu oracle on the host's cores")
        cpu = cpu_baselines(quick=args.quick_cpu)

    import torch

    import paper_2406_18109_amd as dfx
    import synth

    if args.legs == "copy":
        print(json.dumps(copy_leg(dfx, np, torch, n, K)))
        return
    if args.legs == "serve":
        out = serve_main(dfx, synth, np, args)
        print(json.dumps(out))
        return
    # legs: "all" (the default line), "headline", or a comma-separated list of
    # bs_f64, bs_f32, jacobi, cg64, cg256, bicgstab256, gmg, batch, serve
    if args.legs == "all":
        sel = {"bs_f64", "bs_f32", "jacobi", "cg64", "cg256", "bicgstab256", "gmg", "batch", "serve"}
    elif args.legs == "headline":
        sel = set()
    else:
        sel = set(args.legs.split(","))
    log("black-scholes f64 fused n=2^%d" % args.log2n)
    fused = bs_leg(torch, dfx, synth, np, n, "f64", True, K, W, runs=12 if "bs_f64" in sel else 0)
    log("fused", fused)
    legs = {"bs_f64_fused": fused}
    log("copy 2^%d doubles (the streaming ceiling)" % args.log2n)
    copy = copy_leg(dfx, np, torch, n, max(K, 20))
    legs["copy"] = copy
    if "bs_f64" in sel:
        log("black-scholes f64 unfused")
        legs["bs_f64_unfused"] = bs_leg(torch, dfx, synth, np, n, "f64", False, max(2, K // 5), 1)
        u = legs["bs_f64_unfused"]
        fused["speedup_vs_unfused"] = u["ms_per_step"] / fused["ms_per_step"]
        fused["breakeven"] = breakeven(fused, u, "ms_per_step", "first_pass_ms")
    if "bs_f32" in sel:
        log("black-scholes f32 fused / unfused")
        legs["bs_f32_fused"] = bs_leg(torch, dfx, synth, np, n, "f32", True, K, W)
        legs["bs_f32_unfused"] = bs_leg(torch, dfx, synth, np, n, "f32", False, max(2, K // 5), 1)
        legs["bs_f32_fused"]["speedup_vs_unfused"] = (legs["bs_f32_unfused"]["ms_per_step"] /
                                                     legs["bs_f32_fused"]["ms_per_step"])
    if "jacobi" in sel:
        log("jacobi 8192^2 fused (%d sweeps) / unfused" % args.jacobi_sweeps)
        legs["jacobi_fused"] = jacobi_leg(torch, dfx, synth, np, 8192, args.jacobi_sweeps, True)
        legs["jacobi_unfused"] = jacobi_leg(torch, dfx, synth, np, 8192, 10, False)
        jf, ju = legs["jacobi_fused"], legs["jacobi_unfused"]
        jf["speedup_vs_unfused"] = ju["ms_per_sweep"] / jf["ms_per_sweep"]
        jf["breakeven"] = breakeven(jf, ju, "ms_per_sweep", "first_sweep_ms")
    if "cg64" in sel:
        log("cg 64^2 (12 runs of 100 iterations each)")
        legs["cg64_unfused"] = cg_leg(torch, dfx, synth, np, 64, 2, 100, False, False, runs=12)
        legs["cg64_fused"] = cg_leg(torch, dfx, synth, np, 64, 2, 100, True, False, runs=12)
        legs["cg64_fused_graph"] = cg_leg(torch, dfx, synth, np, 64, 2, 100, True, True, runs=12)
        legs["cg64_fused_graph"]["breakeven"] = breakeven(legs["cg64_fused_graph"], legs["cg64_unfused"],
                                                          "ms_per_iter", "first_iter_ms")
    if "cg256" in sel:
        log("cg 256^3 (%d iterations)" % args.cg256_iters)
        legs["cg256_fused_graph"] = cg_leg(torch, dfx, synth, np, 256, 3, args.cg256_iters, True, True)
        legs["cg256_unfused"] = cg_leg(torch, dfx, synth, np, 256, 3, 20, False, False)
        cf, cu = legs["cg256_fused_graph"], legs["cg256_unfused"]
        cf["speedup_vs_unfused"] = cu["ms_per_iter"] / cf["ms_per_iter"]
        cf["breakeven"] = breakeven(cf, cu, "ms_per_iter", "first_iter_ms")
    if "bicgstab256" in sel:
        log("bicgstab 256^3")
        legs["bicgstab256_fused_graph"] = cg_leg(torch, dfx, synth, np, 256, 3, 50, True, True, "bicgstab")
        legs["bicgstab256_unfused"] = cg_leg(torch, dfx, synth, np, 256, 3, 10, False, False, "bicgstab")
        bf, bu = legs["bicgstab256_fused_graph"], legs["bicgstab256_unfused"]
        bf["speedup_vs_unfused"] = bu["ms_per_iter"] / bf["ms_per_iter"]
        bf["breakeven"] = breakeven(bf, bu, "ms_per_iter", "first_iter_ms")
    if "gmg" in sel:
        log("gmg 1023^2, 9 levels (12 runs of 5 iterations)")
        legs["gmg1023_fused_graph"] = gmg_leg(torch, dfx, synth, np, 1023, 9, 5, True, True, runs=12)
        legs["gmg1023_unfused"] = gmg_leg(torch, dfx, synth, np, 1023, 9, 5, False, False)
        gf, gu = legs["gmg1023_fused_graph"], legs["gmg1023_unfused"]
        gf["speedup_vs_unfused"] = gu["ms_per_iter"] / gf["ms_per_iter"]
        gf["breakeven"] = breakeven(gf, gu, "ms_per_iter", "first_iter_ms")
    if "batch" in sel:
        log("batched executor: %d serving solves in one launch, against the server" % args.batch_requests)
        legs["batch"] = batch_leg(dfx, synth, np, args.batch_requests, args.serve_slots,
                                  int(args.serve_budget_gb * (1 << 30)))
    if "serve" in sel:
        log("serving: %d CG solves, %s" % (args.serve_requests, "load sweep" if args.serve_rate is None
                                              else "Poisson arrivals at %.0f/s" % args.serve_rate))
        legs["serve"] = serve_main(dfx, synth, np, args)

    per_launch = fused["alg_bytes_per_step"] / max(1.0, fused["launches_per_step"])
    kernel_s = fused["event_ms_per_step"] * 1e-3 / max(1.0, fused["launches_per_step"])
    achieved = per_launch / kernel_s / 1e9
    traffic = measured_traffic("bs_f64_fused", per_launch)
    hbm_floor = per_launch / (HBM_PEAK_GBS * 1e9)
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "frac_of_copy": round(achieved / copy["gbs"], 4), "copy_gbs": round(copy["gbs"], 1),
            "hbm_floor_ms": round(hbm_floor * 1e3, 4)}
    alu = alu_roof(n, kernel_s)
    if alu is not None:
        roof["alu"] = alu
        if alu["valu_floor_ms"] * 1e-3 > hbm_floor:
            # the op list's own arithmetic takes longer at the VALU peak than
            # its bytes at the HBM peak: the pass is ALU-bound
            roof.update(bound="alu", achieved=alu["achieved"], peak=alu["peak"], unit=alu["unit"],
                        frac=alu["frac"], hbm_frac=round(achieved / HBM_PEAK_GBS, 4))
    line = {
        "metric": "fused vs unfused HBM GB/s (% of peak) and CG iters/s on 1 MI355X; p99 solve latency",
        "value": round(fused["gbs"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(fused["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "black-scholes fused pass, 2^%d options FP64 (28 index tasks -> 1 kernel)" % args.log2n,
                   "options": n, "tasks_per_pass": 28, "parallelism": "1 GPU",
                   "kernel": "compiled pass (hiprtc, op list as constants)" if JIT else "op-list interpreter"},
        "roofline": roof,
        "legs": legs,
    }
    if cpu is not None:
        bs = cpu["bs_f64"]
        line["cpu_baseline"] = {
            "value": round(bs["gbs_all"], 4), "unit": "GB/s", "cores": cpu["workers"], "kind": "oracle",
            "sample": "Black-Scholes FP64, %d options in %d fixed chunks (one forked worker each, the oracle "
                      "unchanged: numpy + libm, unfused op by op); host %s, %d CPUs" %
                      (bs["options_all"], cpu["workers"], cpu["cpu_model"], cpu["host_cpus"]),
            "single_thread": {"value": round(bs["gbs_single"], 4), "unit": "GB/s", "cores": 1,
                              "sample": "%d options" % bs["options_single"]},
            "jacobi_sweep_8192": cpu["jacobi_sweep"], "cg256_iteration": cpu["cg256_iteration"]}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
