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


// Row i of y = A x for a CSR matrix: summed sequentially in CSR order
// (s = a0*x0, then s = s + ak*xk), nonzeros fetched eight at a time so that
// several gathers are in flight.  Row pointers are clamped to [0, nnz] and
// column indices to [0, nx): a malformed matrix yields wrong values, never an
// access outside the arrays.
template <typename T>
__device__ __forceinline__ T csr_row(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                     const T* __restrict__ val, const T* __restrict__ x, int64_t i, int32_t nnz,
                                     uint32_t nx) {
  const int32_t rb = min(max(rowptr[i], 0), nnz);
  const int32_t re = min(max(rowptr[i + 1], rb), nnz);
  T s = (T)0;
  for (int32_t k = rb; k < re; k += 8) {
    int32_t c[8];
    T a[8], xv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int32_t idx = k + j < re ? k + j : rb;
      c[j] = colidx[idx];
      a[j] = val[idx];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) xv[j] = x[(uint32_t)c[j] < nx ? c[j] : 0];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (k + j < re) {
        const T t = a[j] * xv[j];
        s = (k + j == rb) ? t : s + t;
      }
  }
  return s;
}

// N rows per lane at once (row i[m] when ok[m]), each summed exactly as
// csr_row sums it; the rows' loads are issued together, so their memory
// latencies overlap.  Entries past a row's end read index 0, which exists
// whenever any row of the call has an entry.
template <typename T, int N>
__device__ __forceinline__ void csr_rows(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                         const T* __restrict__ val, const T* __restrict__ x, const int64_t (&i)[N],
                                         const bool (&ok)[N], int32_t nnz, uint32_t nx, T (&y)[N]) {
  int32_t rb[N], len[N], lmax = 0;
#pragma unroll
  for (int m = 0; m < N; ++m) {
    const int32_t b0 = ok[m] ? rowptr[i[m]] : 0, e0 = ok[m] ? rowptr[i[m] + 1] : 0;
    rb[m] = min(max(b0, 0), nnz);
    len[m] = min(max(e0, rb[m]), nnz) - rb[m];
    lmax = max(lmax, len[m]);
    y[m] = (T)0;
  }
  for (int32_t k = 0; k < lmax; k += 8) {
    int32_t c[N][8];
    T a[N][8], xv[N][8];
#pragma unroll
    for (int m = 0; m < N; ++m)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int32_t idx = k + j < len[m] ? rb[m] + k + j : 0;
        c[m][j] = colidx[idx];
        a[m][j] = val[idx];
      }
#pragma unroll
    for (int m = 0; m < N; ++m)
#pragma unroll
      for (int j = 0; j < 8; ++j) xv[m][j] = x[(uint32_t)c[m][j] < nx ? c[m][j] : 0];
#pragma unroll
    for (int m = 0; m < N; ++m)
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (k + j < len[m]) {
          const T t = a[m][j] * xv[m][j];
          y[m] = (k + j == 0) ? t : y[m] + t;
        }
  }
}

// Move per-lane row results to the canonical owners: y[m] of lane l holds the
// element 64m + l of a run of V*64 elements; lane l receives elements V*l + v
// (v < V) in out[v].
template <typename T, int V>
__device__ __forceinline__ void rows_to_owners(const T (&y)[V], T (&out)[4]) {
  const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int e = V * lane + v;
    const int src = e & (WAVE - 1), sel = e / WAVE;
    T r = (T)0;
#pragma unroll
    for (int m = 0; m < V; ++m) {
      const T t = __shfl(y[m], src, WAVE);
      r = sel == m ? t : r;
    }
    out[v] = r;
  }
}

}  // namespace dfx
