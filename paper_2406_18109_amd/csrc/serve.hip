// Batched CG for the continuous-batching server: one launch per CG phase
// covers the tiles of every resident solve (solves of different sizes share a
// launch).  Each (solve, tile) work item is processed by one wave in the
// canonical order of the op-list kernel (lane l owns columns 2l, 2l+1 of each
// 128-element row; 32 rows per tile), so the tile sums -- and, through the
// same pairwise tree, every dot product -- are identical whatever else is in
// the batch.  The last wave to finish a solve's tiles in a phase (device-scope
// ticket) forms that solve's scalars: rho and ||b|| (init), alpha = rho/(p.q),
// or beta = rho'/rho and the convergence test.
#include <hip/hip_runtime.h>
#include <math.h>

#include "dev_common.h"
#include "serve.h"

namespace dfx {

constexpr int S_TW = 128;   // FP64 row width of the canonical tiling
constexpr int S_TH = RED_TH;

__device__ __forceinline__ double csr_row(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                          const double* __restrict__ val, const double* __restrict__ x,
                                          int64_t i) {
  const int32_t b = rowptr[i], e = rowptr[i + 1];
  double s = 0.0;
  int32_t k = b;
  // four nonzeros per round keep several gathers in flight; the sum is
  // still sequential in CSR order
  for (; k + 4 <= e; k += 4) {
    const int32_t c0 = col[k], c1 = col[k + 1], c2 = col[k + 2], c3 = col[k + 3];
    const double a0 = val[k], a1 = val[k + 1], a2 = val[k + 2], a3 = val[k + 3];
    const double t0 = a0 * x[c0], t1 = a1 * x[c1], t2 = a2 * x[c2], t3 = a3 * x[c3];
    s = (k == b) ? t0 : s + t0;
    s = s + t1;
    s = s + t2;
    s = s + t3;
  }
  for (; k < e; ++k) {
    const double t = val[k] * x[col[k]];
    s = (k == b) ? t : s + t;
  }
  return s;
}

__global__ __launch_bounds__(BLOCK) void serve_phase_kernel(const ServeLaunch L) {
  const int lane = threadIdx.x & (WAVE - 1);
  int lb = blockIdx.x;
  if ((L.grid & 7) == 0) lb = (blockIdx.x & 7) * (L.grid >> 3) + (blockIdx.x >> 3);
  const int64_t gw = (int64_t)lb * (BLOCK / WAVE) + threadIdx.x / WAVE;
  const int64_t i0 = gw * L.items_per_wave;
  const int64_t i1 = min(i0 + L.items_per_wave, L.n_items);
  const int phase = L.phase;

  for (int64_t it = i0; it < i1; ++it) {
    const int slot = L.item_slot[it];
    const int tile = L.item_tile[it];
    SolveDev* S = L.solves + slot;
    const int status = __builtin_nontemporal_load(&S->status);
    if (phase == PH_INIT ? status != SOLVE_INIT : status != SOLVE_RUN) continue;
    const int64_t n = S->n;
    const double* __restrict__ b = S->b;
    double* __restrict__ x = S->x;
    double* __restrict__ r = S->r;
    double* __restrict__ p = S->p;
    double* __restrict__ q = S->q;
    const double alpha = S->alpha, beta = S->beta;
    double acc = 0.0;
    for (int rr = 0; rr < S_TH; ++rr) {
      const int64_t base = ((int64_t)tile * S_TH + rr) * S_TW + 2 * lane;
      if (base - 2 * lane >= n) break;
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int64_t i = base + v;
        if (i >= n) continue;
        switch (phase) {
          case PH_INIT: {
            const double bi = b[i];
            r[i] = bi;
            p[i] = bi;
            x[i] = 0.0;
            const double t = bi * bi;
            acc = acc + t;
          } break;
          case PH_SPMV_DOT: {
            const double qi = csr_row(S->rowptr, S->col, S->val, p, i);
            q[i] = qi;
            const double t = p[i] * qi;
            acc = acc + t;
          } break;
          case PH_AXPY_DOT: {
            const double t1 = alpha * p[i];
            x[i] = x[i] + t1;
            const double t2 = alpha * q[i];
            const double ri = r[i] - t2;
            r[i] = ri;
            const double t = ri * ri;
            acc = acc + t;
          } break;
          default: {
            const double t = beta * p[i];
            p[i] = t + r[i];
          } break;
        }
      }
    }
    if (phase == PH_UPDATE_P) continue;
    const double ts = wave_sum(acc);
    if (lane == 0) S->partials[tile] = ts;
    __threadfence();
    unsigned int ticket = 0;
    if (lane == 0) ticket = atomicAdd(&S->counter, 1u);
    ticket = __shfl(ticket, 0, WAVE);
    if (ticket != (unsigned int)S->n_tiles - 1) continue;
    // last tile of this solve in this phase: form its scalars
    __threadfence();
    const double total = wave_tree(S->partials, S->n_tiles);
    if (lane == 0) {
      if (phase == PH_INIT) {
        S->rho = total;
        S->bnorm = sqrt(total);
        S->status = !isfinite(total) ? SOLVE_BREAKDOWN : (total == 0.0 ? SOLVE_CONVERGED : SOLVE_RUN);
      } else if (phase == PH_SPMV_DOT) {
        S->pq = total;
        if (!(total > 0.0) || !isfinite(total)) S->status = SOLVE_BREAKDOWN;
        else S->alpha = S->rho / total;
      } else {
        const double rho_new = total;
        S->beta = rho_new / S->rho;
        S->rho = rho_new;
        S->iters = S->iters + 1;
        if (!isfinite(rho_new)) S->status = SOLVE_BREAKDOWN;
        else if (sqrt(rho_new) <= S->tol * S->bnorm) S->status = SOLVE_CONVERGED;
        else if (S->iters >= S->max_iter) S->status = SOLVE_MAXITER;
      }
      __threadfence();
      atomicExch(&S->counter, 0u);
    }
  }
}

int launch_serve_phase(const ServeLaunch& L, hipStream_t stream) {
  hipLaunchKernelGGL(serve_phase_kernel, dim3(L.grid), dim3(BLOCK), 0, stream, L);
  return (int)hipGetLastError();
}

}  // namespace dfx
