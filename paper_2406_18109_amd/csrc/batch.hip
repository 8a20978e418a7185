// The persistent batched executor (see batch.h): one launch runs many
// independent task streams of fused passes.  Each wave is an independent
// worker.  It claims a work item (stream, current pass, run of tiles) with an
// atomic on the stream's claim word, executes the run with the op-list step
// of the ordinary kernel, writes one sum per tile and reduction, and counts
// the run done.  The wave that finishes a pass's last run reduces the tile
// sums with the canonical pairwise tree (the same tree the two-launch path
// evaluates, so every result is bit-identical to a solo run), writes the 0-d
// results, and advances the stream to its next pass.  A stream runs on one
// XCD; its passes are ordered by agent-scope release/acquire (xcd_release,
// xcd_acquire); values written inside the launch (0-d results, tile sums)
// are read with vector or atomic loads, never through the scalar cache.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch.h"
#include "dev_common.h"
#include "vm_exec.h"

namespace dfx {

namespace {

// One instantiation serves every pass of a batch: FP64, 8 registers, up to
// 6 input streams, the SpMV prologue taken when the pass has one, one row
// per step; with the transcendental op set (HV 1) when any pass needs it,
// else the arithmetic one (HV 0, fewer registers).
typedef double BT;
constexpr int BNR = VM_NREG_LIGHT, BNINB = 6;

// Synchronisation.  Streams are pinned to XCDs, so every wave that reads a
// stream's data runs on the XCD whose L2 holds it.  A run's stores are
// released by waiting for their completion (s_waitcnt: they have reached
// the L2), without writing the L2 back to memory as an agent-scope release
// would; a claim or a completed count is followed by the agent-scope
// acquire (it invalidates the CU's caches above the L2).  Control words are
// agent-scope atomics.  A message-passing test between waves of one XCD on
// MI355X (writer: plain stores, wait, flag; reader: flag, acquire, loads)
// saw no stale value over 8 x 10^5 messages with this pair, and stale values
// with an L1-only invalidate (buffer_inv sc0) as the acquire.
__device__ __forceinline__ void xcd_release() {
  __builtin_amdgcn_s_waitcnt(0);
  asm volatile("" ::: "memory");
}
__device__ __forceinline__ void xcd_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
template <typename U> __device__ __forceinline__ U xload(U* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename U> __device__ __forceinline__ void xstore(U* p, U v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename U> __device__ __forceinline__ U xadd(U* p, U v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// A data word written inside the launch (a 0-d result), read after an
// acquire: an atomic load, never the scalar cache.
__device__ __forceinline__ double load_data_f64(const double* p) {
  return __builtin_bit_cast(double, __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT));
}

__device__ __forceinline__ unsigned long long bcast64(unsigned long long v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// Pass index (into the batch's pass table) of the g-th pass a stream runs;
// -1 past the end of a stream without a repeated body.
__device__ __forceinline__ int pass_of(const BatchStream& st, uint32_t g) {
  if ((int64_t)g < st.n_pre) return st.pass0 + (int)g;
  if (st.n_body == 0) return -1;
  return st.pass0 + st.n_pre + (int)((g - (uint32_t)st.n_pre) % (uint32_t)st.n_body);
}

// Run index a settled (done or paused) stream's claim word holds: never
// claimable, and far from carrying into the pass count.
constexpr unsigned long long CLAIM_CLOSED = 0x80000000ull;

// The canonical tree over a[0..n) (any n >= 1) evaluated by one wave:
// aligned chunks of 256 are complete subtrees (block_tree), their sums are
// written to `scratch` and reduced the same way until one chunk remains.
// `a` and `scratch` are global; the result is valid in every lane.
__device__ double wave_tree(const double* a, int64_t n, double* scratch, int lane) {
  const double* src = a;
  double* dst = scratch;
  while (n > 4 * WAVE) {
    const int64_t m = (n + 4 * WAVE - 1) / (4 * WAVE);
    for (int64_t c = 0; c < m; ++c) {
      const int cnt = (int)min((int64_t)4 * WAVE, n - c * 4 * WAVE);
      const double v = block_tree(src + c * 4 * WAVE, cnt, lane);
      if (lane == 0) dst[c] = v;
    }
    __threadfence_block();
    src = dst;
    dst = (dst == scratch) ? scratch + ((m + 255) & ~(int64_t)255) : scratch;
    n = m;
  }
  const double v = block_tree(src, (int)n, lane);
  return __shfl(v, 0, WAVE);
}

// Execute run r of pass B for stream st: tiles [r * tpw, min(n_tiles, (r+1) * tpw)).
template <int BHV>
__device__ void run_tiles(const BatchPass& B, const BatchStream& st, int64_t r, int32_t* scol, double* sval) {
  typedef Shape<BT, BHV, true, BNR, 0> BS;
  typedef typename GVec<BT, BS::GS>::type bgvec;
  const VmParams& P = B.P;
  constexpr int V = BS::V, U = BS::U, TW = BS::TW, E = BS::E;
  const int lane = threadIdx.x & (WAVE - 1);
  bgvec R0[BNR], R1[BNR], R2[BNR], R3[BNR];
  VmState<BT, BS::NG, BS::GS> G;
  // broadcast operands: 0-d stores, possibly written earlier in this launch
  for (int k = 0; k < P.n_bc; ++k) {
    const bgvec v = (bgvec)load_data_f64((const double*)P.bc[k]);
    const int rr = P.bc_reg[k];
    constexpr int NG = BS::NG;
    FOR_G(Rg[rr] = v;)
  }
#pragma unroll
  for (int g = 0; g < BS::NG; ++g) G.z[g] = (bgvec)0.0;
  BT L[BNINB][E];
  const int64_t t_begin = r * P.tiles_per_wave;
  const int64_t t_end = min(t_begin + P.tiles_per_wave, P.n_tiles);
  for (int64_t t = t_begin; t < t_end; ++t) {
    const int64_t tr = t / P.strips;
    const int64_t ts = t - tr * P.strips;
    const int64_t cbase = ts * TW;
    const int64_t c0 = cbase + (int64_t)lane * V;
    G.acc0 = G.acc1 = G.acc2 = G.acc3 = 0.0;
    for (int rw = 0; rw < RED_TH; rw += U) {
      const int64_t row0 = tr * RED_TH + rw;
      if (row0 >= P.rows) break;
      const bool interior = P.is1d ? ((row0 + U) * TW <= P.n1d) : (row0 + U <= P.rows && cbase + TW <= P.cols);
      int mode = MODE_FAST;
      unsigned vmask = (1u << E) - 1;
      if (!(P.unit_cols && interior)) {
        mode = P.vec_cols ? MODE_CLAMP : MODE_SLOW;
        vmask = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int64_t row = row0 + e / V, col = c0 + e % V;
          const bool ok = P.is1d ? (row * TW + col < P.n1d) : (row < P.rows && col < P.cols);
          vmask |= (ok ? 1u : 0u) << e;
        }
      }
      if (mode != MODE_SLOW) vm_load<BT, V, U, E, BNINB>(P, L, row0, c0, vmask, mode, cbase);
      vm_step<BT, BHV, true, BNR, BNINB, true, 0, true>(P, R0, R1, R2, R3, G, L, row0, c0, vmask, mode, false, 0,
                                                       scol, sval, nullptr, 0, cbase);
    }
    if (P.n_red > 0) {
      const double a0 = wave_sum(G.acc0);
      if (lane == 0) st.tsum[t] = a0;
      if (P.n_red > 1) { const double a1 = wave_sum(G.acc1); if (lane == 0) st.tsum[st.tsum_stride + t] = a1; }
      if (P.n_red > 2) { const double a2 = wave_sum(G.acc2); if (lane == 0) st.tsum[2 * st.tsum_stride + t] = a2; }
      if (P.n_red > 3) { const double a3 = wave_sum(G.acc3); if (lane == 0) st.tsum[3 * st.tsum_stride + t] = a3; }
    }
  }
}

// Stall detector: a wave that finds nothing to claim while no pass of its
// XCD's streams has completed for this many ticks of the 100 MHz constant
// clock (2 s) ends the launch with an error.
#ifndef DFX_BATCH_STALL_TICKS
#define DFX_BATCH_STALL_TICKS 200000000ull
#endif

template <int BHV>
__global__ __launch_bounds__(BLOCK) void batch_kernel(const BatchPass* __restrict__ passes,
                                                     BatchStream* __restrict__ streams, BatchCtl* __restrict__ ctl) {
  __shared__ int32_t sp_col[BLOCK / WAVE][SP_CAP];
  __shared__ double sp_val[BLOCK / WAVE][SP_CAP];
  const int lane = threadIdx.x & (WAVE - 1);
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  // this wave's XCD (hardware register XCC_ID)
  const uint32_t xcc = __builtin_amdgcn_readfirstlane(__builtin_amdgcn_s_getreg((20) | (0 << 6) | (3 << 11)));
  const uint32_t nxcd = ctl->n_xcd;
  if (lane == 0) {
    __hip_atomic_fetch_or(&ctl->xcc_seen, 1u << (xcc & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&ctl->waves[xcc & 15], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (xcc >= nxcd) return;
  BatchXcd& X = ctl->x[xcc];
  const uint32_t ns = X.n_streams;   // streams xcc, xcc + nxcd, ...
  if (ns == 0) return;
  const int gw = blockIdx.x * (BLOCK / WAVE) + wib;
  uint32_t s = ((uint32_t)gw / nxcd) % ns;   // index among this XCD's streams
  uint32_t seen_progress = 0;
  // stream and pass up to which this wave's last acquire made every earlier
  // pass visible (passes before acq_gen of stream acq_sid)
  int acq_sid = -1;
  uint32_t acq_gen = 0;
  unsigned long long since = __builtin_amdgcn_s_memrealtime();
  for (;;) {
    uint32_t settled = 0, prog = 0;
    int err = 0;
    if (lane == 0) {
      settled = xload(&X.n_settled);
      prog = xload(&X.progress);
      err = xload(&X.error);
    }
    settled = __builtin_amdgcn_readfirstlane(settled);
    prog = __builtin_amdgcn_readfirstlane(prog);
    err = __builtin_amdgcn_readfirstlane(err);
    if (settled >= ns || err) break;
    // find a claimable run: the lanes look at 64 of this XCD's streams at
    // once (lane l at stream s + l, so the stream this wave last served comes
    // first); a settled stream's claim word is closed, so one load per stream
    // decides.  Then lane 0 claims from the candidates in lane order.
    int sid = -1, pidx = 0;
    uint32_t run = 0, gen = 0, sl = s;
    for (uint32_t base = 0; base < ns && sid < 0; base += WAVE) {
      const uint32_t j = base + lane;
      uint32_t q = s + j;
      q = q < ns ? q : q - ns;   // s < ns and j < ns below, so one wrap suffices
      bool can = false;
      if (j < ns) {
        const BatchStream& stl = streams[(size_t)q * nxcd + xcc];
        const unsigned long long w = xload(&stl.claim);
        const int p = pass_of(stl, (uint32_t)(w >> 32));
        can = p >= 0 && (uint32_t)w < (uint32_t)passes[p].n_runs;
      }
      unsigned long long m = __ballot(can);
      while (m != 0ull) {
        const int L = (int)__builtin_ctzll(m);
        m &= m - 1ull;
        const uint32_t qL = __builtin_amdgcn_readfirstlane(__shfl(q, L, WAVE));
        BatchStream& st = streams[(size_t)qL * nxcd + xcc];
        unsigned long long w = 0;
        if (lane == 0) w = xadd(&st.claim, 1ull);
        w = bcast64(w);
        const int p = pass_of(st, (uint32_t)(w >> 32));
        if (p >= 0 && (uint32_t)w < (uint32_t)passes[p].n_runs) {
          sid = (int)((size_t)qL * nxcd + xcc);
          sl = qL;
          pidx = p;
          run = (uint32_t)w;
          gen = (uint32_t)(w >> 32);
          break;
        }
      }
    }
    if (sid < 0) {
      // nothing to claim: the stall detector ends the launch with an error
      // instead of waiting forever
      const unsigned long long now = __builtin_amdgcn_s_memrealtime();
      if (prog != seen_progress) {
        seen_progress = prog;
        since = now;
      } else if (now - since > DFX_BATCH_STALL_TICKS) {
        if (lane == 0) xstore(&X.error, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    s = sl;
    BatchStream& st = streams[sid];
    const BatchPass& B = passes[pidx];
    // acquire: the stream's earlier passes are visible to every lane.  A
    // wave whose last acquire already followed the completion of every pass
    // before this one (another run of the same pass, or the next pass after
    // it finished the previous one) skips it.
    if (sid != acq_sid || gen > acq_gen) {
      xcd_acquire();
      acq_sid = sid;
      acq_gen = gen;
    }
    run_tiles<BHV>(B, st, run, sp_col[wib], sp_val[wib]);
    since = __builtin_amdgcn_s_memrealtime();
    // release every lane's stores of this run, then count it
    xcd_release();
    uint32_t d = 0;
    if (lane == 0) d = xadd(&st.done, 1u);
    d = __builtin_amdgcn_readfirstlane(d);
    if (d + 1 != (uint32_t)B.n_runs) continue;
    // ---- the last run of the pass: reductions, then advance the stream ------
    // (the other runs' tile sums and outputs; a one-run pass was all this wave's)
    if (B.n_runs > 1) xcd_acquire();
    acq_sid = sid;
    acq_gen = gen + 1;
    const VmParams& P = B.P;
    double* chunk = st.tsum + (int64_t)VM_MAXRED * st.tsum_stride;
    for (int k = 0; k < P.n_red; ++k) {
      const double v = wave_tree(st.tsum + k * st.tsum_stride, P.n_tiles, chunk, lane);
      if (lane == 0) {
        double* res = (double*)B.result[k];
        const double old = load_data_f64(res);
        *res = B.init[k] ? v : old + v;
      }
    }
    xcd_release();
    int32_t next_status = BS_RUNNING;
    const uint32_t g1 = gen + 1;
    if (st.n_body == 0) {
      if ((int64_t)g1 >= st.n_pre) next_status = BS_DONE;
    } else if ((int64_t)g1 > st.n_pre && ((g1 - (uint32_t)st.n_pre) % (uint32_t)st.n_body) == 0) {
      // a repetition of the body is complete (only this wave touches the
      // counters now: the stream's next pass is not yet published)
      int32_t it = 0, rit = 0;
      if (lane == 0) {
        it = xload(&st.iters) + 1;
        rit = xload(&st.round_iters) + 1;
        xstore(&st.iters, it);
        xstore(&st.round_iters, rit);
      }
      it = __builtin_amdgcn_readfirstlane(it);
      rit = __builtin_amdgcn_readfirstlane(rit);
      bool stop = it >= st.max_iter;
      if (!stop && st.conv_a) {
        const double a = load_data_f64(st.conv_a), b = load_data_f64(st.conv_b);
        stop = a <= st.tol * b;
      }
      if (stop) next_status = BS_DONE;
      else if (ctl->round_limit > 0 && rit >= ctl->round_limit) next_status = BS_PAUSED;
    } else if (st.n_pre > 0 && (int64_t)g1 == st.n_pre && st.max_iter <= 0) {
      next_status = BS_DONE;
    }
    if (lane == 0) {
      xstore(&st.done, 0u);
      if (next_status != BS_RUNNING) xstore(&st.status, next_status);
      xcd_release();
      xstore(&st.claim, ((unsigned long long)g1 << 32) | (next_status != BS_RUNNING ? CLAIM_CLOSED : 0ull));
      if (next_status != BS_RUNNING) xadd(&X.n_settled, 1u);
      xadd(&X.progress, 1u);
    }
  }
}

}  // namespace

// Waves one compute unit holds of the batch kernel (heavy: the
// transcendental variant).
int batch_waves_per_cu(int heavy) {
  int blocks = 0;
  const void* f = heavy ? (const void*)&batch_kernel<1> : (const void*)&batch_kernel<0>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, BLOCK, 0) != hipSuccess) return 0;
  return blocks * (BLOCK / WAVE);
}

int launch_batch(const BatchPass* passes, BatchStream* streams, BatchCtl* ctl, int grid, int heavy,
                 hipStream_t stream) {
  if (heavy) hipLaunchKernelGGL(batch_kernel<1>, dim3(grid), dim3(BLOCK), 0, stream, passes, streams, ctl);
  else hipLaunchKernelGGL(batch_kernel<0>, dim3(grid), dim3(BLOCK), 0, stream, passes, streams, ctl);
  return (int)hipGetLastError();
}

}  // namespace dfx
