// HIP executor for gfx950: the op-list kernel that runs one fused pass.
//
// A pass is a fused group of tasks over one iteration space (section 4.2's
// fused task; its body is the tasks' bodies composed in program order).  Each
// lane holds VM_E element slots; for every step the kernel loads the input
// streams into virtual registers, interprets the op list over the slots with
// wave-uniform register indices (scalar-branch dispatch, indexed VGPR moves),
// writes the output streams and accumulates reductions.  Temporaries of the
// fused group never leave VGPRs.  Reductions follow the canonical tile tree
// described in vm.h, so the result does not depend on which pass, fusion or
// launch shape produced it; the last block to finish combines the tile sums.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "vm.h"

namespace dfx {

template <typename T> __device__ __forceinline__ T d_sqrt(T x);
template <> __device__ __forceinline__ double d_sqrt<double>(double x) { return sqrt(x); }
template <> __device__ __forceinline__ float d_sqrt<float>(float x) { return sqrtf(x); }
template <typename T> __device__ __forceinline__ T d_exp(T x);
template <> __device__ __forceinline__ double d_exp<double>(double x) { return exp(x); }
template <> __device__ __forceinline__ float d_exp<float>(float x) { return expf(x); }
template <typename T> __device__ __forceinline__ T d_log(T x);
template <> __device__ __forceinline__ double d_log<double>(double x) { return log(x); }
template <> __device__ __forceinline__ float d_log<float>(float x) { return logf(x); }
template <typename T> __device__ __forceinline__ T d_erf(T x);
template <> __device__ __forceinline__ double d_erf<double>(double x) { return erf(x); }
template <> __device__ __forceinline__ float d_erf<float>(float x) { return erff(x); }
template <typename T> __device__ __forceinline__ T d_pow(T x, T y);
template <> __device__ __forceinline__ double d_pow<double>(double x, double y) { return pow(x, y); }
template <> __device__ __forceinline__ float d_pow<float>(float x, float y) { return powf(x, y); }

template <typename T> __device__ __forceinline__ T d_max(T x, T y) { return (x > y || x != x) ? x : y; }
template <typename T> __device__ __forceinline__ T d_min(T x, T y) { return (x < y || x != x) ? x : y; }

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

template <typename T>
__device__ T row_spmv(const VmParams& P, int64_t i) {
  const int32_t b = P.rowptr[i], e = P.rowptr[i + 1];
  const T* val = (const T*)P.val;
  const T* x = (const T*)P.x;
  T s = (T)0;
  if (b < e) {
    s = val[b] * x[P.colidx[b]];
    for (int32_t k = b + 1; k < e; ++k) {
      const T t = val[k] * x[P.colidx[k]];
      s = s + t;
    }
  }
  return s;
}

// Register file: one array of VM_NREG per element slot, indexed only by
// wave-uniform values, so the compiler keeps each in VGPRs and reaches it with
// indexed moves.
template <typename T> struct Regs {
  T z0, z1, z2, z3;         // previous instruction's result (forwarded operand)
  T acc0, acc1, acc2, acc3; // this lane's reduction accumulators
};
#define DFX_RF T (&r0)[NR], T (&r1)[NR], T (&r2)[NR], T (&r3)[NR]

// One step: U rows of the tile, V columns per lane.  FAST: every slot of
// every lane is in range and every stream has unit column stride, so each
// stream is NINB vector loads issued back to back; otherwise per-element
// masked loads.  NINB is the stream bucket: slots n_in..NINB-1 read a
// harmless broadcast address.
template <typename T, bool HEAVY, int NINB, int NR>
__device__ __forceinline__ void vm_step(const VmParams& P, DFX_RF, Regs<T>& G, int64_t row0, int64_t c0,
                                         unsigned vmask, const bool FAST) {
  constexpr int V = Lanes<T>::V, U = Lanes<T>::U, TW = Lanes<T>::TW;
  typedef T vecA __attribute__((ext_vector_type(V), aligned(sizeof(T))));

  // ---- loads: all issued before the first use --------------------------------
  T L[NINB][VM_E];
#pragma unroll
  for (int a = 0; a < NINB; ++a) {
    const T* b = (const T*)P.in[a].base;
    const int64_t sr = P.in[a].s_row, sc = P.in[a].s_col;
    if (FAST) {
      // sc is 1 for real streams and 0 for padding slots
      const int64_t cc = c0 & (-sc);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const vecA w = *(const vecA*)(b + (row0 + u) * sr + cc);
#pragma unroll
        for (int v = 0; v < V; ++v) L[a][u * V + v] = w[v];
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const bool ok = (vmask >> (u * V + v)) & 1;
          const T w = b[ok ? (row0 + u) * sr + (c0 + v) * sc : 0];
          L[a][u * V + v] = ok ? w : (T)0;
        }
    }
  }
#pragma unroll
  for (int a = 0; a < NINB; ++a) {
    r0[a] = L[a][0]; r1[a] = L[a][1]; r2[a] = L[a][2]; r3[a] = L[a][3];
  }
  if (P.spmv) {
    T e[VM_E];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int64_t i = (row0 + u) * TW + c0 + v;
        e[u * V + v] = ((vmask >> (u * V + v)) & 1) ? row_spmv<T>(P, i) : (T)0;
      }
    r0[NR - 1] = e[0]; r1[NR - 1] = e[1]; r2[NR - 1] = e[2]; r3[NR - 1] = e[3];
  }

  // ---- op list ----------------------------------------------------------------
  for (int pc = 0; pc < P.n_code; ++pc) {
    const VmInstr I = P.code[pc];
    const int d = I.dst, ia = I.a, ib = I.b;
    T x0, x1, x2, x3, y0, y1, y2, y3;
    if (I.flags & VF_A_ACC) { x0 = G.z0; x1 = G.z1; x2 = G.z2; x3 = G.z3; }
    else { x0 = r0[ia]; x1 = r1[ia]; x2 = r2[ia]; x3 = r3[ia]; }
    if (I.flags & VF_B_ACC) { y0 = G.z0; y1 = G.z1; y2 = G.z2; y3 = G.z3; }
    else { y0 = r0[ib]; y1 = r1[ib]; y2 = r2[ib]; y3 = r3[ib]; }
    const T k = (T)P.imm[I.imm];
    T z0, z1, z2, z3;
#define BIN(EXPR) { z0 = EXPR(x0, y0); z1 = EXPR(x1, y1); z2 = EXPR(x2, y2); z3 = EXPR(x3, y3); } break;
#define UN(EXPR) { z0 = EXPR(x0); z1 = EXPR(x1); z2 = EXPR(x2); z3 = EXPR(x3); } break;
#define F_ADD(a, b) ((a) + (b))
#define F_SUB(a, b) ((a) - (b))
#define F_MUL(a, b) ((a) * (b))
#define F_DIV(a, b) ((a) / (b))
#define F_ADDI(a) ((a) + k)
#define F_SUBI(a) ((a) - k)
#define F_RSUBI(a) (k - (a))
#define F_MULI(a) ((a) * k)
#define F_DIVI(a) ((a) / k)
#define F_RDIVI(a) (k / (a))
#define F_NEG(a) (-(a))
#define F_ABS(a) ((a) < (T)0 ? -(a) : (a) == (T)0 ? (T)0 : (a))
#define F_SQ(a) ((a) * (a))
#define F_MOV(a) (a)
    switch (I.op) {
      case VO_MOV: UN(F_MOV)
      case VO_NEG: UN(F_NEG)
      case VO_ABS: UN(F_ABS)
      case VO_SQUARE: UN(F_SQ)
      case VO_ADD: BIN(F_ADD)
      case VO_SUB: BIN(F_SUB)
      case VO_MUL: BIN(F_MUL)
      case VO_DIV: BIN(F_DIV)
      case VO_MAX: BIN(d_max<T>)
      case VO_MIN: BIN(d_min<T>)
      case VO_ADDI: UN(F_ADDI)
      case VO_SUBI: UN(F_SUBI)
      case VO_RSUBI: UN(F_RSUBI)
      case VO_MULI: UN(F_MULI)
      case VO_DIVI: UN(F_DIVI)
      case VO_RDIVI: UN(F_RDIVI)
      case VO_FILL: { z0 = k; z1 = k; z2 = k; z3 = k; } break;
      case VO_RED:
      case VO_REDPROD: {
        // sequential over the slots in canonical order, valid slots only
        T s;
        switch (I.slot) {
          case 0: s = G.acc0; break;
          case 1: s = G.acc1; break;
          case 2: s = G.acc2; break;
          default: s = G.acc3; break;
        }
        if (I.op == VO_REDPROD) {
          const T p0 = x0 * y0, p1 = x1 * y1, p2 = x2 * y2, p3 = x3 * y3;
          {
            if (vmask & 1) s = s + p0;
            if (vmask & 2) s = s + p1;
            if (vmask & 4) s = s + p2;
            if (vmask & 8) s = s + p3;
          }
        } else {
          {
            if (vmask & 1) s = s + x0;
            if (vmask & 2) s = s + x1;
            if (vmask & 4) s = s + x2;
            if (vmask & 8) s = s + x3;
          }
        }
        switch (I.slot) {
          case 0: G.acc0 = s; break;
          case 1: G.acc1 = s; break;
          case 2: G.acc2 = s; break;
          default: G.acc3 = s; break;
        }
        z0 = x0; z1 = x1; z2 = x2; z3 = x3;
      } break;
      default:
        if constexpr (HEAVY) {
          switch (I.op) {
            case VO_SQRT: UN(d_sqrt<T>)
            case VO_EXP: UN(d_exp<T>)
            case VO_LOG: UN(d_log<T>)
            case VO_ERF: UN(d_erf<T>)
            case VO_POW: BIN(d_pow<T>)
            default: { z0 = x0; z1 = x1; z2 = x2; z3 = x3; } break;
          }
        } else {
          z0 = x0; z1 = x1; z2 = x2; z3 = x3;
        }
        break;
    }
#undef BIN
#undef UN
    G.z0 = z0; G.z1 = z1; G.z2 = z2; G.z3 = z3;
    if (I.flags & VF_WB) { r0[d] = z0; r1[d] = z1; r2[d] = z2; r3[d] = z3; }
  }

  // ---- stores -----------------------------------------------------------------
#pragma unroll
  for (int s = 0; s < VM_MAXOUT; ++s) {
    if (s < P.n_out) {
      const int o = P.out_reg[s];
      T e[VM_E];
      e[0] = r0[o]; e[1] = r1[o]; e[2] = r2[o]; e[3] = r3[o];
      T* b = (T*)P.out[s].base;
      const int64_t sr = P.out[s].s_row, sc = P.out[s].s_col;
      if (FAST) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          vecA w;
#pragma unroll
          for (int v = 0; v < V; ++v) w[v] = e[u * V + v];
          *(vecA*)(b + (row0 + u) * sr + c0) = w;
        }
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int v = 0; v < V; ++v)
            if ((vmask >> (u * V + v)) & 1) b[(row0 + u) * sr + (c0 + v) * sc] = e[u * V + v];
      }
    }
  }
}

template <typename T, bool HEAVY, int NINB, int NR>
__global__ __launch_bounds__(BLOCK) void vm_kernel(const VmParams P) {
  constexpr int V = Lanes<T>::V, U = Lanes<T>::U, TW = Lanes<T>::TW;
  static_assert(U * V == VM_E, "element slots");
  // the planner never pairs a register file smaller than the stream bucket
  if constexpr (NINB > NR) { return; } else {

  T r0[NR], r1[NR], r2[NR], r3[NR];
  Regs<T> G;
#pragma unroll
  for (int k = 0; k < VM_MAXBC; ++k) {
    if (k < P.n_bc) {
      const T v = *(const T*)P.bc[k];
      const int r = P.bc_reg[k];
      r0[r] = v; r1[r] = v; r2[r] = v; r3[r] = v;
    }
  }
  G.z0 = G.z1 = G.z2 = G.z3 = (T)0;

  const int lane = threadIdx.x & (WAVE - 1);
  const int wib = threadIdx.x / WAVE;
  // XCD-aware numbering: consecutive blocks land on different XCDs, so give
  // each XCD a contiguous range of logical blocks (and therefore of tiles).
  int lb = blockIdx.x;
  if ((P.grid & 7) == 0) lb = (blockIdx.x & 7) * (P.grid >> 3) + (blockIdx.x >> 3);
  const int64_t gw = (int64_t)lb * (BLOCK / WAVE) + wib;
  const int64_t t_begin = gw * P.tiles_per_wave;
  const int64_t t_end = min(t_begin + P.tiles_per_wave, P.n_tiles);

  for (int64_t t = t_begin; t < t_end; ++t) {
    const int64_t tr = t / P.strips;
    const int64_t ts = t - tr * P.strips;
    const int64_t cbase = ts * TW;
    const int64_t c0 = cbase + (int64_t)lane * V;
    G.acc0 = G.acc1 = G.acc2 = G.acc3 = (T)0;
    for (int r = 0; r < RED_TH; r += U) {
      const int64_t row0 = tr * RED_TH + r;
      if (row0 >= P.rows) break;
      const bool interior = P.is1d ? ((row0 + U) * TW <= P.n1d)
                                   : (row0 + U <= P.rows && cbase + TW <= P.cols);
      const bool fast = P.unit_cols && interior;
      unsigned vmask = (1u << VM_E) - 1;
      if (!fast) {
        vmask = 0;
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const int64_t row = row0 + u, col = c0 + v;
            const bool ok = P.is1d ? (row * TW + col < P.n1d) : (row < P.rows && col < P.cols);
            vmask |= (ok ? 1u : 0u) << (u * V + v);
          }
      }
      vm_step<T, HEAVY, NINB, NR>(P, r0, r1, r2, r3, G, row0, c0, vmask, fast);
    }
    // ---- tile partial sums ------------------------------------------------------
    if (P.n_red > 0) {
      T a0 = wave_sum(G.acc0);
      if (lane == 0) ((T*)P.red_partials[0])[t] = a0;
      if (P.n_red > 1) { T a1 = wave_sum(G.acc1); if (lane == 0) ((T*)P.red_partials[1])[t] = a1; }
      if (P.n_red > 2) { T a2 = wave_sum(G.acc2); if (lane == 0) ((T*)P.red_partials[2])[t] = a2; }
      if (P.n_red > 3) { T a3 = wave_sum(G.acc3); if (lane == 0) ((T*)P.red_partials[3])[t] = a3; }
    }
  }

  if (P.n_red == 0) return;
  // ---- last block combines the tile sums --------------------------------------
  __shared__ T sh[FINAL_CHUNK];
  __shared__ T sh2[FINAL_CHUNK];
  __shared__ unsigned int ticket;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) ticket = atomicAdd(P.counter, 1u);
  __syncthreads();
  if (ticket != gridDim.x - 1) return;
  __threadfence();
  for (int k = 0; k < P.n_red; ++k) {
    const T* part = (const T*)P.red_partials[k];
    const int64_t n = P.n_tiles;
    const int nch = (int)((n + FINAL_CHUNK - 1) / FINAL_CHUNK);
    for (int c = 0; c < nch; ++c) {
      const int64_t base = (int64_t)c * FINAL_CHUNK;
      const int L = (int)min((int64_t)FINAL_CHUNK, n - base);
      for (int i = threadIdx.x; i < L; i += BLOCK) sh[i] = __builtin_nontemporal_load(part + base + i);
      __syncthreads();
      lds_tree(sh, L);
      if (threadIdx.x == 0) sh2[c] = sh[0];
      __syncthreads();
    }
    lds_tree(sh2, nch);
    if (threadIdx.x == 0) {
      const T total = nch > 0 ? sh2[0] : (T)0;
      T* res = (T*)P.red_result[k];
      *res = P.red_init[k] ? total : *res + total;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __threadfence();
    atomicExch(P.counter, 0u);
  }
  }
}

#define DFX_INST(T, H, NR) \
  template __global__ void vm_kernel<T, H, 2, NR>(const VmParams); \
  template __global__ void vm_kernel<T, H, 4, NR>(const VmParams); \
  template __global__ void vm_kernel<T, H, 6, NR>(const VmParams); \
  template __global__ void vm_kernel<T, H, 10, NR>(const VmParams);
DFX_INST(double, true, VM_NREG)
DFX_INST(double, false, VM_NREG_LIGHT)
DFX_INST(float, true, VM_NREG)
DFX_INST(float, false, VM_NREG_LIGHT)

template <typename T, bool H, int NR>
static void launch_t(const VmParams& P, int ninb, dim3 grid, hipStream_t st) {
  switch (ninb) {
    case 2: hipLaunchKernelGGL((vm_kernel<T, H, 2, NR>), grid, dim3(BLOCK), 0, st, P); break;
    case 4: hipLaunchKernelGGL((vm_kernel<T, H, 4, NR>), grid, dim3(BLOCK), 0, st, P); break;
    case 6: hipLaunchKernelGGL((vm_kernel<T, H, 6, NR>), grid, dim3(BLOCK), 0, st, P); break;
    default: hipLaunchKernelGGL((vm_kernel<T, H, 10, NR>), grid, dim3(BLOCK), 0, st, P); break;
  }
}

int stream_bucket(int n_in) { return n_in <= 2 ? 2 : n_in <= 4 ? 4 : n_in <= 6 ? 6 : 10; }

// Host-side launch; returns the hipError_t of the launch.
int launch_vm(const VmParams& P, int is_f64, int heavy, hipStream_t stream) {
  const dim3 grid(P.grid);
  const int nb = stream_bucket(P.n_in);
  if (is_f64) {
    if (heavy) launch_t<double, true, VM_NREG>(P, nb, grid, stream);
    else launch_t<double, false, VM_NREG_LIGHT>(P, nb, grid, stream);
  } else {
    if (heavy) launch_t<float, true, VM_NREG>(P, nb, grid, stream);
    else launch_t<float, false, VM_NREG_LIGHT>(P, nb, grid, stream);
  }
  return (int)hipGetLastError();
}

}  // namespace dfx
