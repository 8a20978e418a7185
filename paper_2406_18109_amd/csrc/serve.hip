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
// tile rows whose SpMV groups one csr_rows call walks together
#ifndef DFX_SERVE_SPMV_ROWS
#define DFX_SERVE_SPMV_ROWS 2
#endif
constexpr int SR = DFX_SERVE_SPMV_ROWS;
// 1: the SpMV phase stages each 64-row group's CSR range in LDS (csr_group)
#ifndef DFX_SERVE_SPMV_STAGE
#define DFX_SERVE_SPMV_STAGE 0
#endif

// One instantiation per phase, so the elementwise phases do not carry the
// SpMV phase's registers (and keep more waves per SIMD).
template <int PHASE>
__global__ __launch_bounds__(BLOCK) void serve_phase_kernel(const ServeLaunch L) {
  const int lane = threadIdx.x & (WAVE - 1);
  int lb = blockIdx.x;
  if ((L.grid & 7) == 0) lb = (blockIdx.x & 7) * (L.grid >> 3) + (blockIdx.x >> 3);
  const int64_t gw = (int64_t)lb * (BLOCK / WAVE) + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const int64_t i0 = gw * L.items_per_wave;
  const int64_t i1 = min(i0 + L.items_per_wave, L.n_items);
  constexpr int phase = PHASE;

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
    const int64_t t0 = (int64_t)tile * S_TH * S_TW;
    const int nrows = (int)min((int64_t)S_TH, (n - t0 + S_TW - 1) / S_TW);  // rows of the tile inside n
    double acc = 0.0;
    if constexpr (phase == PH_SPMV_DOT && DFX_SERVE_SPMV_STAGE) {
      // q = A p, one 64-row group at a time with its CSR range staged in
      // LDS, then p.q in the canonical order (lane l owns elements 2l, 2l+1
      // of each row)
      __shared__ int32_t sp_col[BLOCK / WAVE][SP_CAP];
      __shared__ double sp_val[BLOCK / WAVE][SP_CAP];
      const int wib = threadIdx.x / WAVE;
      const int32_t nnz = S->rowptr[n];
      for (int rr = 0; rr < nrows; ++rr) {
        const int64_t rb = t0 + (int64_t)rr * S_TW;
        double y[2], pv[2], qo[4];
#pragma unroll
        for (int v = 0; v < 2; ++v) pv[v] = rb + 2 * lane + v < n ? p[rb + 2 * lane + v] : 0.0;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          const int64_t g0 = rb + m * WAVE;
          y[m] = g0 < n ? csr_group<double>(S->rowptr, S->col, S->val, p, g0, n, nnz, (uint32_t)n, sp_col[wib],
                                            sp_val[wib])
                        : 0.0;
          if (g0 + lane < n) q[g0 + lane] = y[m];
        }
        rows_to_owners<double, 2>(y, qo);
#pragma unroll
        for (int v = 0; v < 2; ++v)
          if (rb + 2 * lane + v < n) {
            const double t = pv[v] * qo[v];
            acc = acc + t;
          }
      }
    } else if constexpr (phase == PH_SPMV_DOT) {
      // q = A p with consecutive rows on consecutive lanes (two tile rows,
      // four 64-row groups, per call), then p.q in the canonical order (lane
      // l owns elements 2l, 2l+1 of each row)
      const int32_t nnz = S->rowptr[n];
      for (int r0 = 0; r0 < nrows; r0 += SR) {
        int64_t gi[2 * SR];
        bool gok[2 * SR];
        double y[2 * SR], pv[SR][2];
#pragma unroll
        for (int m = 0; m < 2 * SR; ++m) {
          gi[m] = t0 + (int64_t)(r0 + m / 2) * S_TW + (m % 2) * WAVE + lane;
          gok[m] = r0 + m / 2 < nrows && gi[m] < n;
        }
#pragma unroll
        for (int h = 0; h < SR; ++h)
#pragma unroll
          for (int v = 0; v < 2; ++v) {
            const int64_t i = t0 + (int64_t)(r0 + h) * S_TW + 2 * lane + v;
            pv[h][v] = r0 + h < nrows && i < n ? p[i] : 0.0;
          }
        csr_rows<double, 2 * SR>(S->rowptr, S->col, S->val, p, gi, gok, nnz, (uint32_t)n, y);
#pragma unroll
        for (int m = 0; m < 2 * SR; ++m)
          if (gok[m]) q[gi[m]] = y[m];
#pragma unroll
        for (int h = 0; h < SR; ++h) {
          if (r0 + h >= nrows) break;
          const double yy[2] = {y[2 * h], y[2 * h + 1]};
          double qo[4];
          rows_to_owners<double, 2>(yy, qo);
#pragma unroll
          for (int v = 0; v < 2; ++v) {
            const int64_t i = t0 + (int64_t)(r0 + h) * S_TW + 2 * lane + v;
            if (i < n) {
              const double t = pv[h][v] * qo[v];
              acc = acc + t;
            }
          }
        }
      }
    } else {
      // RU rows' loads in flight together, then the rows in order
      constexpr int RU = 4;
      for (int r0 = 0; r0 < nrows; r0 += RU) {
        double va[RU][2], vb[RU][2], vc[RU][2], vd[RU][2];
        bool ok[RU][2];
        int64_t ix[RU][2];
#pragma unroll
        for (int u = 0; u < RU; ++u)
#pragma unroll
          for (int v = 0; v < 2; ++v) {
            const int64_t i = t0 + (int64_t)(r0 + u) * S_TW + 2 * lane + v;
            ix[u][v] = i;
            ok[u][v] = r0 + u < nrows && i < n;
            va[u][v] = vb[u][v] = vc[u][v] = vd[u][v] = 0.0;
            if (!ok[u][v]) continue;
            if (phase == PH_INIT) {
              va[u][v] = b[i];
            } else if (phase == PH_AXPY_DOT) {
              va[u][v] = p[i];
              vb[u][v] = x[i];
              vc[u][v] = q[i];
              vd[u][v] = r[i];
            } else {
              va[u][v] = p[i];
              vb[u][v] = r[i];
            }
          }
#pragma unroll
        for (int u = 0; u < RU; ++u)
#pragma unroll
          for (int v = 0; v < 2; ++v) {
            if (!ok[u][v]) continue;
            const int64_t i = ix[u][v];
            if (phase == PH_INIT) {
              const double bi = va[u][v];
              r[i] = bi;
              p[i] = bi;
              x[i] = 0.0;
              const double t = bi * bi;
              acc = acc + t;
            } else if (phase == PH_AXPY_DOT) {
              const double t1 = alpha * va[u][v];
              x[i] = vb[u][v] + t1;
              const double t2 = alpha * vc[u][v];
              const double ri = vd[u][v] - t2;
              r[i] = ri;
              const double t = ri * ri;
              acc = acc + t;
            } else {
              const double t = beta * va[u][v];
              p[i] = t + vb[u][v];
            }
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
  switch (L.phase) {
    case PH_INIT: hipLaunchKernelGGL(serve_phase_kernel<PH_INIT>, dim3(L.grid), dim3(BLOCK), 0, stream, L); break;
    case PH_SPMV_DOT: hipLaunchKernelGGL(serve_phase_kernel<PH_SPMV_DOT>, dim3(L.grid), dim3(BLOCK), 0, stream, L); break;
    case PH_AXPY_DOT: hipLaunchKernelGGL(serve_phase_kernel<PH_AXPY_DOT>, dim3(L.grid), dim3(BLOCK), 0, stream, L); break;
    default: hipLaunchKernelGGL(serve_phase_kernel<PH_UPDATE_P>, dim3(L.grid), dim3(BLOCK), 0, stream, L); break;
  }
  if (L.phase != PH_UPDATE_P && L.n_fin > 0)
    hipLaunchKernelGGL(serve_final_kernel, dim3(L.n_fin), dim3(BLOCK), 0, stream, L.solves, L.fin_slots, L.phase);
  return (int)hipGetLastError();
}

}  // namespace dfx
