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


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("paper_2406_18109_amd/csrc/kernels.hip", "paper_2406_18109_amd/csrc/vm.h",
              "paper_2406_18109_amd/csrc/vm_exec.h", "paper_2406_18109_amd/csrc/dev_common.h",
              "paper_2406_18109_amd/csrc/vm_tier0.hip", "paper_2406_18109_amd/csrc/vm_tier1.hip",
              "paper_2406_18109_amd/csrc/vm_tier2.hip", "paper_2406_18109_amd/csrc/vm_tier3.hip",
              "paper_2406_18109_amd/csrc/dmath.h", "paper_2406_18109_amd/csrc/dmath_coef.h"):
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


class BSBench:
    def __init__(self, dfx, synth, np, n, dtype, fuse):
        self.np = np
        npdt = np.float64 if dtype == "f64" else np.float32
        self.ctx = dfx.Context(device=0, window_size=64, fuse=fuse, tune=TUNE)
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


def bs_leg(torch, dfx, synth, np, n, dtype, fuse, K, W):
    b = BSBench(dfx, synth, np, n, dtype, fuse)
    for _ in range(max(W, 8) if TUNE else W):
        b.step()
    b.ctx.stats_reset()
    wall, ev = timed_steps(torch, b.ctx.torch_stream, b.step, K)
    st = b.ctx.stats()
    bytes_per_step = st["alg_bytes"] / K
    launches = st["launches"] / K
    b.close()
    ev_ms = sum(ev) / len(ev)
    return {"ms_per_step": wall, "event_ms_per_step": ev_ms, "alg_bytes_per_step": bytes_per_step,
            "launches_per_step": launches, "gbs": bytes_per_step / (wall * 1e-3) / 1e9,
            "kernel_gbs": bytes_per_step / (ev_ms * 1e-3) / 1e9}


def jacobi_leg(torch, dfx, synth, np, N, sweeps, fuse):
    c = dfx.Context(device=0, window_size=16, fuse=fuse, tune=TUNE)
    G = c.store_create([N, N], "f64")
    c.store_write(G, synth.jacobi_grid(N))
    J = dfx.apps.Jacobi(c, G, N)
    for _ in range(8 if TUNE else 3):
        J.sweep()
    c.sync()
    c.stats_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(sweeps):
        J.sweep()
    c.sync()
    dt = (time.perf_counter() - t0) / sweeps
    st = c.stats()
    out = {"ms_per_sweep": dt * 1e3, "alg_bytes_per_sweep": st["alg_bytes"] / sweeps,
           "gbs": st["alg_bytes"] / sweeps / dt / 1e9, "launches_per_sweep": st["launches"] / sweeps}
    c.close()
    return out


def cg_leg(torch, dfx, synth, np, m, dim, iters, fuse, graph, solver="cg"):
    """CG on the Poisson matrix, or BiCGSTAB (solver="bicgstab") on the
    nonsymmetric convection-diffusion matrix of the same shape."""
    c = dfx.Context(device=0, window_size=16, fuse=fuse, tune=TUNE)
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
    for _ in range(8 if TUNE else 2):
        cg.iteration()
    c.sync()
    g = None
    if graph:
        c.graph_begin()
        cg.iteration()
        g = c.graph_end()
    c.sync()
    c.stats_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        if g is not None:
            c.graph_launch(g)
        else:
            cg.iteration()
    c.sync()
    dt = (time.perf_counter() - t0) / iters
    st = c.stats()
    out = {"iters_per_s": 1.0 / dt, "ms_per_iter": dt * 1e3,
           "alg_bytes_per_iter": st["alg_bytes"] / iters,
           "gbs": st["alg_bytes"] / iters / dt / 1e9, "launches_per_iter": st["launches"] / iters}
    if g is not None:
        c.graph_destroy(g)
    c.close()
    return out


def gmg_leg(torch, dfx, synth, np, m, nlev, iters, fuse, graph):
    """The GMG solver (CG preconditioned by one V(2,2) cycle, injection
    restriction, weighted Jacobi) on the m^2 Poisson problem over nlev
    levels; with graph, one whole iteration is recorded and replayed."""
    c = dfx.Context(device=0, window_size=16, fuse=fuse, tune=TUNE)
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
    g.iteration()
    c.sync()
    gid = None
    if graph:
        c.graph_begin()
        g.iteration()
        gid = c.graph_end()
    c.sync()
    c.stats_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        if gid is not None:
            c.graph_launch(gid)
        else:
            g.iteration()
    c.sync()
    dt = (time.perf_counter() - t0) / iters
    st = c.stats()
    out = {"iters_per_s": 1.0 / dt, "ms_per_iter": dt * 1e3, "alg_bytes_per_iter": st["alg_bytes"] / iters,
           "gbs": st["alg_bytes"] / iters / dt / 1e9, "launches_per_iter": st["launches"] / iters}
    if gid is not None:
        c.graph_destroy(gid)
    c.close()
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


def cpu_baseline(synth, wl, np, sample):
    S, K, T = synth.bs_inputs(sample)
    r, sig, rv = wl.bs_scalars(synth.BS_RATE, synth.BS_VOL)
    wl.black_scholes(S[:1000], K[:1000], T[:1000], r, sig, rv)
    t0 = time.perf_counter()
    reps = 0
    while True:
        wl.black_scholes(S, K, T, r, sig, rv)
        reps += 1
        if time.perf_counter() - t0 > 10.0:
            break
    dt = (time.perf_counter() - t0) / reps
    return sample * 40 / dt / 1e9, reps, dt


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
                    help="all | headline | serve | copy | comma-separated bs_f64,bs_f32,jacobi,cg64,cg256,bicgstab256,gmg,serve")
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--serve-rate", type=float, default=None,
                    help="fixed Poisson arrival rate; default: a saturation run, then 0.5/0.8/0.95 of it")
    ap.add_argument("--serve-slots", type=int, default=256)
    ap.add_argument("--serve-budget-gb", type=float, default=4.0)
    ap.add_argument("--serve-iters-per-round", type=int, default=0,
                    help="CG iterations per scheduling round (0: the library default)")
    ap.add_argument("--log2n", type=int, default=26)
    args = ap.parse_args()
    global TUNE
    TUNE = args.tune
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported (the executor runs on "
              "a single device)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2406_18109_amd as dfx
    import synth
    from oracle import workloads as wl

    n = 1 << args.log2n
    K, W = args.steps, args.warmup
    if args.legs == "copy":
        print(json.dumps(copy_leg(dfx, np, torch, n, K)))
        return
    if args.legs == "serve":
        out = serve_main(dfx, synth, np, args)
        print(json.dumps(out))
        return
    # legs: "all" (the default line), "headline", or a comma-separated list of
    # bs_f64, bs_f32, jacobi, cg64, cg256, bicgstab256, gmg, serve
    if args.legs == "all":
        sel = {"bs_f64", "bs_f32", "jacobi", "cg64", "cg256", "bicgstab256", "gmg", "serve"}
    elif args.legs == "headline":
        sel = set()
    else:
        sel = set(args.legs.split(","))
    log("black-scholes f64 fused n=2^%d" % args.log2n)
    fused = bs_leg(torch, dfx, synth, np, n, "f64", True, K, W)
    log("fused", fused)
    legs = {"bs_f64_fused": fused}
    if "bs_f64" in sel:
        log("black-scholes f64 unfused")
        legs["bs_f64_unfused"] = bs_leg(torch, dfx, synth, np, n, "f64", False, max(2, K // 5), 1)
        legs["bs_f64_fused"]["speedup_vs_unfused"] = legs["bs_f64_unfused"]["ms_per_step"] / fused["ms_per_step"]
    if "bs_f32" in sel:
        log("black-scholes f32 fused / unfused")
        legs["bs_f32_fused"] = bs_leg(torch, dfx, synth, np, n, "f32", True, K, W)
        legs["bs_f32_unfused"] = bs_leg(torch, dfx, synth, np, n, "f32", False, max(2, K // 5), 1)
        legs["bs_f32_fused"]["speedup_vs_unfused"] = (legs["bs_f32_unfused"]["ms_per_step"] /
                                                     legs["bs_f32_fused"]["ms_per_step"])
    if "jacobi" in sel:
        log("jacobi 8192^2 fused / unfused")
        legs["jacobi_fused"] = jacobi_leg(torch, dfx, synth, np, 8192, 20, True)
        legs["jacobi_unfused"] = jacobi_leg(torch, dfx, synth, np, 8192, 5, False)
        legs["jacobi_fused"]["speedup_vs_unfused"] = (legs["jacobi_unfused"]["ms_per_sweep"] /
                                                     legs["jacobi_fused"]["ms_per_sweep"])
    if "cg64" in sel:
        log("cg 64^2")
        legs["cg64_unfused"] = cg_leg(torch, dfx, synth, np, 64, 2, 100, False, False)
        legs["cg64_fused"] = cg_leg(torch, dfx, synth, np, 64, 2, 100, True, False)
        legs["cg64_fused_graph"] = cg_leg(torch, dfx, synth, np, 64, 2, 100, True, True)
    if "cg256" in sel:
        log("cg 256^3")
        legs["cg256_fused_graph"] = cg_leg(torch, dfx, synth, np, 256, 3, 30, True, True)
        legs["cg256_unfused"] = cg_leg(torch, dfx, synth, np, 256, 3, 10, False, False)
    if "bicgstab256" in sel:
        log("bicgstab 256^3")
        legs["bicgstab256_fused_graph"] = cg_leg(torch, dfx, synth, np, 256, 3, 20, True, True, "bicgstab")
        legs["bicgstab256_unfused"] = cg_leg(torch, dfx, synth, np, 256, 3, 6, False, False, "bicgstab")
        legs["bicgstab256_fused_graph"]["speedup_vs_unfused"] = (legs["bicgstab256_unfused"]["ms_per_iter"] /
                                                                 legs["bicgstab256_fused_graph"]["ms_per_iter"])
    if "gmg" in sel:
        log("gmg 1023^2, 9 levels")
        legs["gmg1023_fused_graph"] = gmg_leg(torch, dfx, synth, np, 1023, 9, 10, True, True)
        legs["gmg1023_unfused"] = gmg_leg(torch, dfx, synth, np, 1023, 9, 3, False, False)
        legs["gmg1023_fused_graph"]["speedup_vs_unfused"] = (legs["gmg1023_unfused"]["ms_per_iter"] /
                                                             legs["gmg1023_fused_graph"]["ms_per_iter"])
    if "serve" in sel:
        log("serving: %d CG solves, %s" % (args.serve_requests, "load sweep" if args.serve_rate is None
                                              else "Poisson arrivals at %.0f/s" % args.serve_rate))
        legs["serve"] = serve_main(dfx, synth, np, args)

    log("cpu oracle sample")
    sample = 1 << 21
    cpu_gbs, reps, dt = cpu_baseline(synth, wl, np, sample)
    per_launch = fused["alg_bytes_per_step"] / max(1.0, fused["launches_per_step"])
    achieved = per_launch / (fused["event_ms_per_step"] * 1e-3) / 1e9
    traffic = measured_traffic("bs_f64_fused", per_launch)
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
                   "options": n, "tasks_per_pass": 28, "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
        "cpu_baseline": {"value": round(cpu_gbs, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
                         "sample": "%d options x %d reps, FP64 numpy + libm, unfused op by op" % (sample, reps)},
        "legs": legs,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
