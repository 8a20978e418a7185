// Batched CG for the continuous-batching server: one launch per CG phase
// covers the tiles of every resident solve (solves of different sizes share a
// launch).  Each (solve, tile) work item is processed by one wave in the
// canonical order of the op-list kernel (lane l owns columns 2l, 2l+1 of each
// 128-element row; 32 rows per tile), so the tile sums -- and, through the
// same pairwise tree, every dot product -- are identical whatever else is in
// the batch.  A second launch, one block per solve of the phase, reduces the
// solve's tile sums and forms its scalars: rho and ||b|| (init),
// alpha = rho/(p.q), or beta = rho'/rho and the convergence test.
#include <hip/hip_runtime.h>
#include <math.h>

#include "dev_common.h"
#include "serve.h"

namespace dfx {

constexpr int S_TW = 128;   // FP64 row width of the canonical tiling
constexpr int S_TH = RED_TH;

__global__ __launch_bounds__(BLOCK) void serve_phase_kernel(const ServeLaunch L) {
  const int lane = threadIdx.x & (WAVE - 1);
  int lb = blockIdx.x;
  if ((L.grid & 7) == 0) lb = (blockIdx.x & 7) * (L.grid >> 3) + (blockIdx.x >> 3);
  const int64_t gw = (int64_t)lb * (BLOCK / WAVE) + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
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
    if (phase == PH_SPMV_DOT) {
      // q = A p with consecutive rows on consecutive lanes, then p.q in the
      // canonical order (lane l owns elements 2l, 2l+1 of each row)
      const int32_t nnz = S->rowptr[n];
      for (int rr = 0; rr < S_TH; ++rr) {
        const int64_t sb = ((int64_t)tile * S_TH + rr) * S_TW;
        if (sb >= n) break;
        double y[2], qo[4];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          const int64_t i = sb + m * WAVE + lane;
          y[m] = i < n ? csr_row<double>(S->rowptr, S->col, S->val, p, i, nnz, (uint32_t)n) : 0.0;
          if (i < n) q[i] = y[m];
        }
        rows_to_owners<double, 2>(y, qo);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const int64_t i = sb + 2 * lane + v;
          if (i < n) {
            const double t = p[i] * qo[v];
            acc = acc + t;
          }
        }
      }
    }
    for (int rr = 0; rr < S_TH && phase != PH_SPMV_DOT; ++rr) {
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
  }
}

// One block per listed solve: the pairwise tree over its tile sums (as the
// op-list executor's tile tree), then the phase's scalar update.
__global__ __launch_bounds__(BLOCK) void serve_final_kernel(SolveDev* solves, const int32_t* slots, int phase) {
  __shared__ double sh[S_MAXTILES];
  SolveDev* S = solves + slots[blockIdx.x];
  const int status = S->status;
  if (phase == PH_INIT ? status != SOLVE_INIT : status != SOLVE_RUN) return;
  const int L = S->n_tiles;
  for (int i = threadIdx.x; i < L; i += BLOCK) sh[i] = __builtin_nontemporal_load(S->partials + i);
  __syncthreads();
  lds_tree(sh, L);
  if (threadIdx.x != 0) return;
  const double total = L > 0 ? sh[0] : 0.0;
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
}

int launch_serve_phase(const ServeLaunch& L, hipStream_t stream) {
  hipLaunchKernelGGL(serve_phase_kernel, dim3(L.grid), dim3(BLOCK), 0, stream, L);
  if (L.phase != PH_UPDATE_P && L.n_fin > 0)
    hipLaunchKernelGGL(serve_final_kernel, dim3(L.n_fin), dim3(BLOCK), 0, stream, L.solves, L.fin_slots, L.phase);
  return (int)hipGetLastError();
}

}  // namespace dfx
