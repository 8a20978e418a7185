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
// launch shape produced it; each block reduces its aligned run of tile sums
// in LDS and a one-block kernel launched after the pass combines the block sums.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dev_common.h"
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

// Register file: one array of NR registers per element slot, indexed only by
// wave-uniform values, so the compiler keeps each array in VGPRs and reaches
// it with indexed moves.  Slots 2 and 3 exist only when E == 4.
template <typename T> struct Regs {
  T z0, z1, z2, z3;         // previous instruction's result (forwarded operand)
  T acc0, acc1, acc2, acc3; // this lane's reduction accumulators
};

template <typename T, int HV, bool SPMV> struct Shape {
  static constexpr bool HEAVY = HV > 0;
  static constexpr int V = Lanes<T>::V;
  static constexpr int TW = Lanes<T>::TW;
  // FP64 arithmetic-only passes take two rows per step; passes with
  // transcendental ops or an SpMV prologue take one, to keep the register
  // footprint (and occupancy) in check.  Rows are visited in order either
  // way, so the canonical reduction order does not depend on U.
  static constexpr int U = (sizeof(T) == 8 && !HEAVY && !SPMV) ? 2 : 1;
  static constexpr int E = U * V;
  static constexpr int NR = HEAVY ? VM_NREG : VM_NREG_LIGHT;
};

#define DFX_RF T (&r0)[NR], T (&r1)[NR], T (&r2)[NR], T (&r3)[NR]

enum StepMode { MODE_FAST = 0, MODE_CLAMP = 1, MODE_SLOW = 2 };

// y = A x for the V*64 elements of a step starting at element `base`.  The
// row of element base + 64m + l is computed by lane l (consecutive rows on
// consecutive lanes, so each load instruction touches few cache lines), then
// handed to its owner in the canonical layout by shuffles.
template <typename T, int V>
__device__ __forceinline__ void spmv_rows(const VmParams& P, int64_t base, T (&out)[4]) {
  const int lane = threadIdx.x & (WAVE - 1);
  T y[V];
#pragma unroll
  for (int m = 0; m < V; ++m) {
    const int64_t i = base + m * WAVE + lane;
    y[m] = i < P.n1d ? csr_row<T>(P.rowptr, P.colidx, (const T*)P.val, (const T*)P.x, i, P.nnz, (uint32_t)P.nx)
                     : (T)0;
  }
  rows_to_owners<T, V>(y, out);
}

// One step: U rows of the tile, V columns per lane.
//   MODE_FAST : every slot of every lane valid, unit column strides: vector
//               loads of all streams issued back to back.
//   MODE_CLAMP: validity is whole V-vectors (unit strides, widths multiple
//               of V): the same vector loads with invalid lanes pointed at
//               the stream's first element and zeroed.
//   MODE_SLOW : per-element masked accesses, one stream at a time.
// Slots n_in..NINB-1 of the bucket read a 4 KB zero page in the vector modes.
template <typename T, int HV, bool SPMV, int NINB>
__device__ __forceinline__ void vm_step(const VmParams& P, T (&r0)[Shape<T, HV, SPMV>::NR],
                                         T (&r1)[Shape<T, HV, SPMV>::NR], T (&r2)[Shape<T, HV, SPMV>::NR],
                                         T (&r3)[Shape<T, HV, SPMV>::NR], Regs<T>& G, int64_t row0,
                                         int64_t c0, unsigned vmask, const int mode) {
  typedef Shape<T, HV, SPMV> S;
  constexpr bool HEAVY = S::HEAVY;
  constexpr int V = S::V, U = S::U, TW = S::TW, E = S::E, NR = S::NR;
  static_assert(E == 2 || E == 4, "element slots");
  typedef T vecA __attribute__((ext_vector_type(V), aligned(sizeof(T))));

  // ---- loads: every load of the step in flight before the first wait --------
  if (mode != MODE_SLOW) {
    T L[NINB][E];
    bool okv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) okv[u] = ((vmask >> (u * V)) & ((1u << V) - 1)) != 0;
#pragma unroll
    for (int a = 0; a < NINB; ++a) {
      const T* b = (const T*)P.in[a].base;
      // column stride is 1 for real streams and 0 for padding slots
      const int64_t cc = c0 & (-P.in[a].s_col);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const T* p = b + (row0 + u) * P.in[a].s_row + cc;
        if (mode == MODE_CLAMP) p = okv[u] ? p : b;
        const vecA w = *(const vecA*)p;
#pragma unroll
        for (int v = 0; v < V; ++v) L[a][u * V + v] = w[v];
      }
    }
    if (mode == MODE_CLAMP) {
#pragma unroll
      for (int a = 0; a < NINB; ++a)
#pragma unroll
        for (int e = 0; e < E; ++e) L[a][e] = ((vmask >> e) & 1) ? L[a][e] : (T)0;
    }
#pragma unroll
    for (int a = 0; a < NINB; ++a) {
      r0[a] = L[a][0]; r1[a] = L[a][1];
      if constexpr (E == 4) { r2[a] = L[a][2]; r3[a] = L[a][3]; }
    }
  } else {
    for (int a = 0; a < P.n_in; ++a) {
      const T* b = (const T*)P.in[a].base;
      const int64_t sr = P.in[a].s_row, sc = P.in[a].s_col;
      T w[4];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int u = e / V, v = e % V;
        const bool ok = (vmask >> e) & 1;
        const T q = b[ok ? (row0 + u) * sr + (c0 + v) * sc : 0];
        w[e] = ok ? q : (T)0;
      }
      r0[a] = w[0]; r1[a] = w[1];
      if constexpr (E == 4) { r2[a] = w[2]; r3[a] = w[3]; }
    }
  }
  if constexpr (SPMV) {
    static_assert(U == 1, "SpMV steps take one row of the tiling");
    T y[4];
    spmv_rows<T, V>(P, row0 * TW, y);
    r0[NR - 1] = y[0]; r1[NR - 1] = y[1];
    if constexpr (E == 4) { r2[NR - 1] = y[2]; r3[NR - 1] = y[3]; }
  }

  // ---- op list ----------------------------------------------------------------
  for (int pc = 0; pc < P.n_code; ++pc) {
    const VmInstr I = P.code[pc];   // one scalar load; fields by shifts
    const unsigned w0 = __builtin_amdgcn_readfirstlane(I.w0), w1 = __builtin_amdgcn_readfirstlane(I.w1);
    const unsigned op = w0 & 0xff, flags = w1 & 0xff, slot = (w1 >> 8) & 0xff, immi = w1 >> 16;
    const int d = (w0 >> 8) & 0xff, ia = (w0 >> 16) & 0xff, ib = w0 >> 24;
    T x0, x1, x2 = 0, x3 = 0, y0, y1, y2 = 0, y3 = 0;
    if (flags & VF_A_ACC) {
      x0 = G.z0; x1 = G.z1;
      if constexpr (E == 4) { x2 = G.z2; x3 = G.z3; }
    } else {
      x0 = r0[ia]; x1 = r1[ia];
      if constexpr (E == 4) { x2 = r2[ia]; x3 = r3[ia]; }
    }
    if (flags & VF_B_ACC) {
      y0 = G.z0; y1 = G.z1;
      if constexpr (E == 4) { y2 = G.z2; y3 = G.z3; }
    } else {
      y0 = r0[ib]; y1 = r1[ib];
      if constexpr (E == 4) { y2 = r2[ib]; y3 = r3[ib]; }
    }
    const T k = (T)P.imm[immi];
    T z0, z1, z2 = 0, z3 = 0;
#define BIN(EXPR) { z0 = EXPR(x0, y0); z1 = EXPR(x1, y1); if constexpr (E == 4) { z2 = EXPR(x2, y2); z3 = EXPR(x3, y3); } } break;
#define UN(EXPR) { z0 = EXPR(x0); z1 = EXPR(x1); if constexpr (E == 4) { z2 = EXPR(x2); z3 = EXPR(x3); } } break;
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
#define F_FILL(a) (k)
    switch (op) {
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
      case VO_FILL: UN(F_FILL)
      case VO_RED:
      case VO_REDPROD: {
        // sequential over the slots in canonical order, valid slots only
        T s;
        switch (slot) {
          case 0: s = G.acc0; break;
          case 1: s = G.acc1; break;
          case 2: s = G.acc2; break;
          default: s = G.acc3; break;
        }
        T p0 = x0, p1 = x1, p2 = x2, p3 = x3;
        if (op == VO_REDPROD) {
          p0 = x0 * y0; p1 = x1 * y1;
          if constexpr (E == 4) { p2 = x2 * y2; p3 = x3 * y3; }
        }
        if (vmask & 1) s = s + p0;
        if (vmask & 2) s = s + p1;
        if constexpr (E == 4) {
          if (vmask & 4) s = s + p2;
          if (vmask & 8) s = s + p3;
        }
        switch (slot) {
          case 0: G.acc0 = s; break;
          case 1: G.acc1 = s; break;
          case 2: G.acc2 = s; break;
          default: G.acc3 = s; break;
        }
        z0 = x0; z1 = x1; z2 = x2; z3 = x3;
      } break;
      default:
        if constexpr (HEAVY) {
          switch (op) {
            case VO_SQRT: UN(d_sqrt<T>)
            case VO_EXP: UN(d_exp<T>)
            case VO_LOG: UN(d_log<T>)
            case VO_ERF: UN(d_erf<T>)
            case VO_POW:
              if constexpr (HV >= 2) {
                z0 = d_pow<T>(x0, y0); z1 = d_pow<T>(x1, y1);
                if constexpr (E == 4) { z2 = d_pow<T>(x2, y2); z3 = d_pow<T>(x3, y3); }
              } else {
                z0 = x0; z1 = x1; z2 = x2; z3 = x3;
              }
              break;
            default: { z0 = x0; z1 = x1; z2 = x2; z3 = x3; } break;
          }
        } else {
          z0 = x0; z1 = x1; z2 = x2; z3 = x3;
        }
        break;
    }
#undef BIN
#undef UN
    G.z0 = z0; G.z1 = z1;
    if constexpr (E == 4) { G.z2 = z2; G.z3 = z3; }
    if (flags & VF_WB) {
      r0[d] = z0; r1[d] = z1;
      if constexpr (E == 4) { r2[d] = z2; r3[d] = z3; }
    }
  }

  // ---- stores -----------------------------------------------------------------
  if (mode != MODE_SLOW) {
#pragma unroll
    for (int s = 0; s < VM_MAXOUT; ++s) {
      if (s < P.n_out) {
        const int o = P.out_reg[s];
        T e[4];
        e[0] = r0[o]; e[1] = r1[o];
        if constexpr (E == 4) { e[2] = r2[o]; e[3] = r3[o]; }
        T* b = (T*)P.out[s].base;
        const int64_t sr = P.out[s].s_row;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          vecA w;
#pragma unroll
          for (int v = 0; v < V; ++v) w[v] = e[u * V + v];
          if (mode == MODE_FAST || ((vmask >> (u * V)) & 1)) *(vecA*)(b + (row0 + u) * sr + c0) = w;
        }
      }
    }
  } else {
    for (int s = 0; s < P.n_out; ++s) {
      const int o = P.out_reg[s];
      T e[4];
      e[0] = r0[o]; e[1] = r1[o];
      if constexpr (E == 4) { e[2] = r2[o]; e[3] = r3[o]; }
      T* b = (T*)P.out[s].base;
      const int64_t sr = P.out[s].s_row, sc = P.out[s].s_col;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int u = q / V, v = q % V;
        if ((vmask >> q) & 1) b[(row0 + u) * sr + (c0 + v) * sc] = e[q];
      }
    }
  }
}

template <typename T> __device__ __forceinline__ T block_tree(const T* a, int cnt, int lane);

template <typename T, int HV, bool SPMV, int NINB>
__global__ __launch_bounds__(BLOCK) void vm_kernel(const VmParams P) {
  typedef Shape<T, HV, SPMV> S;
  constexpr int V = S::V, U = S::U, TW = S::TW, E = S::E, NR = S::NR;
  __shared__ T tsum[VM_MAXRED][4 * VM_MAXTPW];  // this block's tile sums

  T r0[NR], r1[NR], r2[NR], r3[NR];
  Regs<T> G;
#pragma unroll
  for (int k = 0; k < VM_MAXBC; ++k) {
    if (k < P.n_bc) {
      const T v = *(const T*)P.bc[k];
      const int r = P.bc_reg[k];
      r0[r] = v; r1[r] = v;
      if constexpr (E == 4) { r2[r] = v; r3[r] = v; }
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
      vm_step<T, HV, SPMV, NINB>(P, r0, r1, r2, r3, G, row0, c0, vmask, mode);
    }
    // ---- tile sums into the block's LDS row ---------------------------------------
    if (P.n_red > 0) {
      const int j = wib * (int)P.tiles_per_wave + (int)(t - t_begin);
      T a0 = wave_sum(G.acc0);
      if (lane == 0) tsum[0][j] = a0;
      if (P.n_red > 1) { T a1 = wave_sum(G.acc1); if (lane == 0) tsum[1][j] = a1; }
      if (P.n_red > 2) { T a2 = wave_sum(G.acc2); if (lane == 0) tsum[2][j] = a2; }
      if (P.n_red > 3) { T a3 = wave_sum(G.acc3); if (lane == 0) tsum[3][j] = a3; }
    }
  }

  if (P.n_red == 0) return;
  // ---- block subtree: the 4 * tiles_per_wave tiles from lb * 4 * tiles_per_wave
  // form one aligned subtree of the tile tree; wave k reduces reduction k.
  __syncthreads();
  if (wib >= P.n_red) return;
  const int64_t blk0 = (int64_t)lb * 4 * P.tiles_per_wave;
  if (blk0 >= P.n_tiles) return;
  const int cnt = (int)min((int64_t)4 * P.tiles_per_wave, P.n_tiles - blk0);
  const T v = block_tree(tsum[wib], cnt, lane);
  if (lane == 0) ((T*)P.red_partials[wib])[lb] = v;
}

// Pairwise tree over a[0..cnt) (cnt <= 4 * WAVE) by one wave: lane l first
// combines the aligned group a[4l..4l+4) -- a complete subtree when full --
// then the group sums are combined across lanes level by level.  Every level
// adds the right neighbour into the left one only when it exists, as in
// lds_tree.  The result is valid in lane 0.
template <typename T> __device__ __forceinline__ T block_tree(const T* a, int cnt, int lane) {
  const int j = 4 * lane;
  T v = (T)0;
  if (j < cnt) {
    const int c = min(4, cnt - j);
    const T v01 = c > 1 ? a[j] + a[j + 1] : a[j];
    v = c == 4 ? v01 + (a[j + 2] + a[j + 3]) : c == 3 ? v01 + a[j + 2] : v01;
  }
  const int L = (cnt + 3) / 4;
  for (int h = 1; h < L; h <<= 1) {
    const T o = __shfl_down(v, h, WAVE);
    if ((lane & (2 * h - 1)) == 0 && lane + h < L) v = v + o;
  }
  return v;
}

// Block sums -> 0-d results: chunks of FINAL_CHUNK block sums (complete
// subtrees except the last) are reduced level by level in LDS, then the chunk
// sums the same way.  All reductions of the pass advance together.
template <typename T> __global__ __launch_bounds__(FINAL_BLOCK) void vm_final(const VmFinal F) {
  __shared__ T sh[VM_MAXRED][FINAL_CHUNK];
  __shared__ T cs[VM_MAXRED][FINAL_CHUNK];
  const int tid = threadIdx.x;
  const int nch = (F.nblocks + FINAL_CHUNK - 1) / FINAL_CHUNK;
  for (int c = 0; c < nch; ++c) {
    const int L = min(FINAL_CHUNK, F.nblocks - c * FINAL_CHUNK);
    for (int k = 0; k < F.n_red; ++k)
      sh[k][tid] = tid < L ? __builtin_nontemporal_load((const T*)F.partials[k] + (int64_t)c * FINAL_CHUNK + tid) : (T)0;
    __syncthreads();
    for (int h = 1; h < L; h <<= 1) {
      const int i = tid * 2 * h;
      if (i + h < L)
        for (int k = 0; k < F.n_red; ++k) sh[k][i] = sh[k][i] + sh[k][i + h];
      __syncthreads();
    }
    if (tid < F.n_red) cs[tid][c] = sh[tid][0];
    __syncthreads();
  }
  for (int h = 1; h < nch; h <<= 1) {
    const int i = tid * 2 * h;
    if (i + h < nch)
      for (int k = 0; k < F.n_red; ++k) cs[k][i] = cs[k][i] + cs[k][i + h];
    __syncthreads();
  }
  if (tid < F.n_red) {
    const T total = nch > 0 ? cs[tid][0] : (T)0;
    T* res = (T*)F.result[tid];
    *res = F.init[tid] ? total : *res + total;
  }
}

#define DFX_INST(T, H, SP) \
  template __global__ void vm_kernel<T, H, SP, 2>(const VmParams); \
  template __global__ void vm_kernel<T, H, SP, 4>(const VmParams); \
  template __global__ void vm_kernel<T, H, SP, 6>(const VmParams);
DFX_INST(double, 0, false)
DFX_INST(double, 0, true)
DFX_INST(double, 1, false)
DFX_INST(double, 1, true)
DFX_INST(float, 0, false)
DFX_INST(float, 0, true)
DFX_INST(float, 1, false)
DFX_INST(float, 1, true)
// the widest stream bucket and pow exist only in the most general tier
template __global__ void vm_kernel<double, 2, false, 10>(const VmParams);
template __global__ void vm_kernel<double, 2, true, 10>(const VmParams);
template __global__ void vm_kernel<float, 2, false, 10>(const VmParams);
template __global__ void vm_kernel<float, 2, true, 10>(const VmParams);

template <typename T, int H, bool SP>
static void launch_t(const VmParams& P, int ninb, dim3 grid, hipStream_t st) {
  if constexpr (H == 2) {
    hipLaunchKernelGGL((vm_kernel<T, 2, SP, 10>), grid, dim3(BLOCK), 0, st, P);
  } else {
    switch (ninb) {
      case 2: hipLaunchKernelGGL((vm_kernel<T, H, SP, 2>), grid, dim3(BLOCK), 0, st, P); break;
      case 4: hipLaunchKernelGGL((vm_kernel<T, H, SP, 4>), grid, dim3(BLOCK), 0, st, P); break;
      default: hipLaunchKernelGGL((vm_kernel<T, H, SP, 6>), grid, dim3(BLOCK), 0, st, P); break;
    }
  }
}

template __global__ void vm_final<double>(const VmFinal);
template __global__ void vm_final<float>(const VmFinal);

int launch_vm_final(const VmFinal& F, int is_f64, hipStream_t stream) {
  if (is_f64) hipLaunchKernelGGL(vm_final<double>, dim3(1), dim3(FINAL_BLOCK), 0, stream, F);
  else hipLaunchKernelGGL(vm_final<float>, dim3(1), dim3(FINAL_BLOCK), 0, stream, F);
  return (int)hipGetLastError();
}

int stream_bucket(int n_in, int tier) { return tier == 2 ? 10 : n_in <= 2 ? 2 : n_in <= 4 ? 4 : 6; }

// Host-side launch; returns the hipError_t of the launch.  `tier`: 0 arithmetic
// only (8 registers), 1 with sqrt/exp/log/erf, 2 with pow (16 registers); tiers
// 0 and 1 take at most 6 streams, tier 2 up to 10.
int launch_vm(const VmParams& P, int is_f64, int tier, hipStream_t stream) {
  const dim3 grid(P.grid);
  const int nb = stream_bucket(P.n_in, tier);
  if (P.n_in > nb) return (int)hipErrorInvalidValue;
  const bool sp = P.spmv != 0;
#define DFX_L(T, H) { if (sp) launch_t<T, H, true>(P, nb, grid, stream); else launch_t<T, H, false>(P, nb, grid, stream); }
  if (is_f64) {
    if (tier == 0) DFX_L(double, 0) else if (tier == 1) DFX_L(double, 1) else DFX_L(double, 2)
  } else {
    if (tier == 0) DFX_L(float, 0) else if (tier == 1) DFX_L(float, 1) else DFX_L(float, 2)
  }
#undef DFX_L
  return (int)hipGetLastError();
}

}  // namespace dfx
