// Device helpers shared by the op-list kernel and the batched CG kernels:
// the fixed reduction trees that make every sum independent of launch shape.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

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

// Row g0 + lane of a 64-row group (0 past n), with the group's contiguous
// CSR range staged in this wave's LDS slice (scol, sval: SP_CAP entries) by
// coalesced 16-byte nontemporal loads, so every line of col and val is
// fetched once and does not displace x in L2; each lane then walks its row
// from LDS.  A range longer than SP_CAP is read directly (csr_row).  Either
// way the row is summed sequentially in CSR order.  Every lane of the wave
// calls it.
constexpr int SP_CAP = 512;

template <typename T>
__device__ __forceinline__ T csr_group(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                       const T* __restrict__ val, const T* __restrict__ x, int64_t g0, int64_t n,
                                       int32_t nnz, uint32_t nx, int32_t* __restrict__ scol, T* __restrict__ sval) {
  typedef int32_t i4 __attribute__((ext_vector_type(4)));
  typedef T vv __attribute__((ext_vector_type(16 / sizeof(T))));
  constexpr int VE = 16 / sizeof(T);   // values per 16-byte load
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t i = g0 + lane;
  // the group's range from the lanes' own row pointers (first row, last valid row)
  const int last = (int)(min(g0 + WAVE, n) - g0) - 1;
  const int32_t rb_raw = i < n ? rowptr[i] : 0;
  const int32_t re_raw = i < n ? rowptr[i + 1] : 0;
  const int32_t nb = min(max(__builtin_amdgcn_readfirstlane(rb_raw), 0), nnz);
  const int32_t ne = min(max(__builtin_amdgcn_readlane(re_raw, last), nb), nnz);
  const int32_t a0 = nb & ~3;
  const int32_t cnt = ne - a0;
  if (cnt > SP_CAP) return i < n ? csr_row<T>(rowptr, colidx, val, x, i, nnz, nx) : (T)0;
  // stage [a0, ne) of col and val: every chunk's load is in flight before
  // the first LDS store (cnt <= SP_CAP here)
  constexpr int CC = SP_CAP / (4 * WAVE), VC = SP_CAP / (VE * WAVE);
  i4 cb[CC];
  vv vb[VC];
#pragma unroll
  for (int u = 0; u < CC; ++u) {
    const int j = (u * WAVE + lane) * 4;
    if (j < cnt) {
      if (a0 + j + 3 < nnz) cb[u] = __builtin_nontemporal_load((const i4*)(colidx + a0 + j));
      else
        for (int t = 0; t < 4; ++t) cb[u][t] = a0 + j + t < nnz ? colidx[a0 + j + t] : 0;
    }
  }
#pragma unroll
  for (int u = 0; u < VC; ++u) {
    const int j = (u * WAVE + lane) * VE;
    if (j < cnt) {
      if (a0 + j + VE - 1 < nnz) vb[u] = __builtin_nontemporal_load((const vv*)(val + a0 + j));
      else
        for (int t = 0; t < VE; ++t) vb[u][t] = a0 + j + t < nnz ? val[a0 + j + t] : (T)0;
    }
  }
#pragma unroll
  for (int u = 0; u < CC; ++u) {
    const int j = (u * WAVE + lane) * 4;
    if (j < cnt) *(i4*)(scol + j) = cb[u];
  }
#pragma unroll
  for (int u = 0; u < VC; ++u) {
    const int j = (u * WAVE + lane) * VE;
    if (j < cnt) *(vv*)(sval + j) = vb[u];
  }
  __builtin_amdgcn_wave_barrier();
  T sm = (T)0;
  if (i < n) {
    // clamped into the staged window: a malformed rowptr reads wrong values, never outside it
    const int32_t rb = min(max(rb_raw, nb), ne);
    const int32_t re = min(max(re_raw, rb), ne);
    const int32_t b = rb - a0, e = re - a0;
    for (int32_t k = b; k < e; k += 8) {
      int32_t c[8];
      T av[8], xv[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int32_t kk = k + t < e ? k + t : b;
        c[t] = scol[kk];
        av[t] = sval[kk];
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) xv[t] = x[(uint32_t)c[t] < nx ? c[t] : 0];
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (k + t < e) {
          const T tv = av[t] * xv[t];
          sm = (k + t == b) ? tv : sm + tv;
        }
    }
  }
  // every lane's reads of this group are done before the next group is staged
  __builtin_amdgcn_wave_barrier();
  return sm;
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
