// Device helpers shared by the op-list kernel and the batched CG kernels:
// the fixed reduction trees that make every sum independent of launch shape.
#pragma once
#include <hip/hip_runtime.h>

#include "vm.h"

namespace dfx {

template <typename T> __device__ __forceinline__ T shfl_xor(T v, int m);
template <> __device__ __forceinline__ double shfl_xor<double>(double v, int m) { return __shfl_xor(v, m, WAVE); }
template <> __device__ __forceinline__ float shfl_xor<float>(float v, int m) { return __shfl_xor(v, m, WAVE); }

// Fixed xor butterfly: every lane ends with the same value (IEEE addition
// is commutative, so lane l and lane l^m compute the identical sum).
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int m = WAVE / 2; m >= 1; m >>= 1) v = v + shfl_xor(v, m);
  return v;
}

// Pairwise power-of-two tree over a[0..L) in LDS: level h adds a[i+h] into
// a[i] for i a multiple of 2h with i+h < L.  Result in a[0].
template <typename T> __device__ void lds_tree(T* a, int L) {
  for (int h = 1; h < L; h <<= 1) {
    for (int i = threadIdx.x * 2 * h; i < L; i += BLOCK * 2 * h)
      if (i + h < L) a[i] = a[i] + a[i + h];
    __syncthreads();
  }
}


// The pairwise power-of-two tree over a[0..L) (as lds_tree) computed by one
// wave from global memory: aligned blocks of 64 leaves are complete subtrees,
// so each is reduced with lane shuffles and the block sums are reduced the
// same way.  L <= 64*64.  Every lane returns the total.
__device__ __forceinline__ double wave_tree(const double* a, int L) {
  const int lane = threadIdx.x & (WAVE - 1);
  double blk = 0.0;
  const int nb = (L + WAVE - 1) / WAVE;
  for (int c = 0; c < nb; ++c) {
    const int Lb = min(WAVE, L - c * WAVE);
    double v = lane < Lb ? __builtin_nontemporal_load(a + c * WAVE + lane) : 0.0;
    for (int h = 1; h < Lb; h <<= 1) {
      const double o = __shfl_down(v, h, WAVE);
      if ((lane & (2 * h - 1)) == 0 && lane + h < Lb) v = v + o;
    }
    const double s = __shfl(v, 0, WAVE);
    if (lane == c) blk = s;
  }
  double v = blk;
  for (int h = 1; h < nb; h <<= 1) {
    const double o = __shfl_down(v, h, WAVE);
    if ((lane & (2 * h - 1)) == 0 && lane + h < nb) v = v + o;
  }
  return nb > 0 ? __shfl(v, 0, WAVE) : 0.0;
}

}  // namespace dfx
