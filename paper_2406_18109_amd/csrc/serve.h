// Device-side state of the batched CG executor (continuous-batching server).
#pragma once
#include <stdint.h>

namespace dfx {

// One resident solve.  Vectors follow the canonical 1-D tiling of the
// op-list kernel (rows of 128 FP64 elements, tiles of 32 rows), so every
// reduction is the same tree the unbatched path computes.
struct SolveDev {
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  const double* b;
  double* x;
  double* r;
  double* p;
  double* q;
  double* partials;     // n_tiles tile sums
  int64_t n;
  int32_t n_tiles;
  int32_t max_iter;
  double tol;
  double rho, pq, alpha, beta, bnorm;
  int32_t iters;
  int32_t status;       // SOLVE_* below
};

constexpr int S_MAXTILES = 64 * 64;  // tiles per solve (the tile tree fits one block's LDS)

enum SolveStatus {
  SOLVE_INIT = 0,       // admitted, r = b and rho not yet formed
  SOLVE_RUN = 1,
  SOLVE_CONVERGED = 2,
  SOLVE_MAXITER = 3,
  SOLVE_BREAKDOWN = 4
};

enum ServePhase { PH_INIT = 0, PH_SPMV_DOT = 1, PH_AXPY_DOT = 2, PH_UPDATE_P = 3 };

// Work list of one phase: item i is tile item_tile[i] of solve item_slot[i].
struct ServeLaunch {
  SolveDev* solves;
  const int32_t* item_slot;
  const int32_t* item_tile;
  int64_t n_items;
  int64_t items_per_wave;
  int32_t phase;
  int32_t grid;
  const int32_t* fin_slots;  // the solves of this phase, one block each in the scalar update
  int32_t n_fin;
};

}  // namespace dfx
