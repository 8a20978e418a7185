// HIP executor for gfx950: the op-list kernel that runs one fused pass.
//
// A pass is a fused group of tasks over one iteration space (section 4.2's
// fused task; its body is the tasks' bodies composed in program order).  Each
// lane holds E element slots; for every step the kernel loads the input
// streams into virtual registers, interprets the op list over the slots with
// wave-uniform register indices (scalar-branch dispatch, indexed VGPR moves),
// writes the output streams and accumulates reductions.  Temporaries of the
// fused group never leave VGPRs.  Reductions follow the canonical tile tree
// described in vm.h, so the result does not depend on which pass, fusion or
// launch shape produced it; each block reduces its aligned run of tile sums
// in LDS and a one-block kernel launched after the pass combines the block
// sums.  The kernel templates are instantiated per tier in their own sources.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <math.h>
#endif
#include <stdint.h>

#include "dev_common.h"
#include "dmath.h"
#include "vm.h"

namespace dfx {

template <typename T> __device__ __forceinline__ T d_sqrt(T x);
template <> __device__ __forceinline__ double d_sqrt<double>(double x) { return sqrt(x); }
template <> __device__ __forceinline__ float d_sqrt<float>(float x) { return sqrtf(x); }
template <typename T> __device__ __forceinline__ T d_exp(T x);
template <> __device__ __forceinline__ double d_exp<double>(double x) { double v[1] = {x}; dm_exp(v); return v[0]; }
template <> __device__ __forceinline__ float d_exp<float>(float x) { return expf(x); }
template <typename T> __device__ __forceinline__ T d_log(T x);
template <> __device__ __forceinline__ double d_log<double>(double x) { double v[1] = {x}; dm_log(v); return v[0]; }
template <> __device__ __forceinline__ float d_log<float>(float x) { return logf(x); }
template <typename T> __device__ __forceinline__ T d_erf(T x);
template <> __device__ __forceinline__ double d_erf<double>(double x) { double v[1] = {x}; dm_erf(v); return v[0]; }
template <> __device__ __forceinline__ float d_erf<float>(float x) { return erff(x); }
template <typename T> __device__ __forceinline__ T d_pow(T x, T y);
template <> __device__ __forceinline__ double d_pow<double>(double x, double y) { return pow(x, y); }
template <> __device__ __forceinline__ float d_pow<float>(float x, float y) { return powf(x, y); }

// FP64 transcendental handlers evaluate the E values of a step in
// DFX_MATH_SPLIT groups (fewer live temporaries per group)
#ifndef DFX_MATH_SPLIT
#define DFX_MATH_SPLIT 1
#endif

template <typename T> __device__ __forceinline__ T d_max(T x, T y) { return (x > y || x != x) ? x : y; }
template <typename T> __device__ __forceinline__ T d_min(T x, T y) { return (x < y || x != x) ? x : y; }
template <typename T> __device__ __forceinline__ T d_abs(T x) { return x < (T)0 ? -x : x == (T)0 ? (T)0 : x; }

#ifndef DFX_TRANS8_F64_ROWS
#define DFX_TRANS8_F64_ROWS 2
#endif
#ifndef DFX_TRANS8_F32_ROWS
#define DFX_TRANS8_F32_ROWS 2
#endif
#ifndef DFX_ARITH_F64_GS
#define DFX_ARITH_F64_GS 1
#endif

// ROWS > 0 fixes the rows per step (the one-row arithmetic kernels, which
// fit four waves per SIMD); 0 takes the rule below.
template <typename T, int HV, bool SPMV, int NR_, int ROWS = 0> struct Shape {
  static constexpr bool HEAVY = HV > 0;
  static constexpr int V = Lanes<T>::V;
  static constexpr int TW = Lanes<T>::TW;
  static constexpr int NR = NR_;
  // Rows per step: two where the register file of NR registers x E elements
  // stays within 64 VGPRs, else one; SpMV steps take one row.  Rows are
  // visited in order either way, so the canonical reduction order does not
  // depend on U.
  static constexpr int FIT = 256 / (NR * V * (int)sizeof(T));
  static constexpr int U = SPMV ? 1
                         : ROWS > 0 ? ROWS
                         : (HEAVY && NR == VM_NREG_LIGHT && sizeof(T) == 8) ? DFX_TRANS8_F64_ROWS
                         : (HEAVY && NR == VM_NREG_LIGHT) ? DFX_TRANS8_F32_ROWS
                         : (FIT >= 2 ? 2 : 1);
  static constexpr int E = U * V;
  // The register file is split into NG arrays of NR vectors of GS elements.
  // An array of at most 128 bytes (32 VGPRs) is the largest that indexed VGPR
  // moves reach without falling back to scratch; fetching an operand for
  // every slot takes NG indexed blocks.  Transcendental and FP32 kernels use
  // the widest groups (fewest blocks per interpreted op); the FP64
  // arithmetic kernels keep one array per slot, which measured faster for
  // their stream-bound passes.
  static constexpr int GS_MAX = 128 / NR / (int)sizeof(T) < E ? 128 / NR / (int)sizeof(T) : E;
  static constexpr int GS = (!HEAVY && sizeof(T) == 8) ? DFX_ARITH_F64_GS : GS_MAX;
  static constexpr int NG = E / GS;
  static_assert(GS >= 1 && GS <= GS_MAX && NG * GS == E && NG <= 4, "register file split");
};

// GS elements of one register group (a scalar when GS == 1).  The groups are
// separate arrays (R0..R3) so each stays its own allocation; FOR_G
// expands a statement for each group with `g` and `Rg` bound at compile time.
#define FOR_G(...)                          \
  {                                         \
    {                                       \
      constexpr int g = 0;                  \
      auto& Rg = R0;                        \
      (void)g; (void)Rg;                    \
      __VA_ARGS__                           \
    }                                       \
    if constexpr (NG > 1) {                 \
      constexpr int g = 1;                  \
      auto& Rg = R1;                        \
      (void)g; (void)Rg;                    \
      __VA_ARGS__                           \
    }                                       \
    if constexpr (NG > 2) {                 \
      constexpr int g = 2;                  \
      auto& Rg = R2;                        \
      (void)g; (void)Rg;                    \
      __VA_ARGS__                           \
    }                                       \
    if constexpr (NG > 3) {                 \
      constexpr int g = 3;                  \
      auto& Rg = R3;                        \
      (void)g; (void)Rg;                    \
      __VA_ARGS__                           \
    }                                       \
  }
template <typename T, int GS> struct GVec { typedef T type __attribute__((ext_vector_type(GS))); };
template <typename T> struct GVec<T, 1> { typedef T type; };

template <typename T, int GS> __device__ __forceinline__ T gget(const typename GVec<T, GS>::type& v, int c) {
  if constexpr (GS == 1) return v;
  else return v[c];
}
template <typename T, int GS> __device__ __forceinline__ void gset(typename GVec<T, GS>::type& v, int c, T x) {
  if constexpr (GS == 1) v = x;
  else v[c] = x;
}

template <typename T, int NG, int GS> struct VmState {
  typedef typename GVec<T, GS>::type gvec;
  gvec z[NG];               // previous instruction's result (forwarded operand)
  T acc0, acc1, acc2, acc3; // this lane's reduction accumulators
  // A tile shared by a block's waves (compiled passes, red_split): reduction
  // slot 0 writes its summands to dsum[(drow + u) * TW + lane * V + v] (drow:
  // the step's first row within the tile) instead of accumulating them.
  // Set by compiled kernels only (the interpreter never reads them).
  T* dsum;
  int drow;
};

// One instruction of the op list over every element slot of a step, for
// compiled passes: their generated program calls it once per instruction
// with the fields as constants, so the op switch folds away and every
// register index is a constant (the register file becomes plain VGPRs).
// The interpreter executes the same body (vm_instr.inc) with the fields it
// decodes at run time, so both forms round alike.
template <typename T, int HV, int NR, int NG, int GS, int E>
__device__ __forceinline__ void vm_instr(typename GVec<T, GS>::type (&R0)[NR], typename GVec<T, GS>::type (&R1)[NR],
                                         typename GVec<T, GS>::type (&R2)[NR], typename GVec<T, GS>::type (&R3)[NR],
                                         VmState<T, NG, GS>& G, const unsigned vmask, const unsigned op,
                                         const unsigned flags, const unsigned slot, const unsigned post,
                                         const unsigned d, const unsigned ia, const unsigned ib, const unsigned ic,
                                         const T k) {
  constexpr bool HEAVY = HV > 0;
  constexpr bool DEFER_OK = true;
  constexpr int V = Lanes<T>::V, TW = Lanes<T>::TW;
  typedef typename GVec<T, GS>::type gvec;
#include "vm_instr.inc"
}

// The op list a kernel executes.  VmInterp interprets the pass's code
// (P.code, P.out_reg, P.bc_reg, P.st_on/st_dr/st_dc).  A compiled pass's
// program type, generated by the host for that one pass, has COMPILED true,
// its output and broadcast register maps and its stencil staging map as
// constants, its waves-per-SIMD target (WAVES), whether a transcendental
// pass software-pipelines its loads (HEAVY_PF) and a run() that calls
// vm_instr for each instruction in order.
struct VmInterp {
  static constexpr bool COMPILED = false;
  static constexpr int N_IN = 0, N_OUT = 0;   // (compiled passes: the pass's stream counts)
  static constexpr bool RELOAD = false;       // (compiled passes: parameters reloaded per step)
  static constexpr int WAVES = 1;
  static constexpr bool HEAVY_PF = false;   // transcendental passes prefetch the next step
  static constexpr int out_reg[VM_MAXOUT] = {};
  static constexpr int bc_reg[VM_MAXBC] = {};
  static constexpr int st_on[VM_MAXIN] = {}, st_dr[VM_MAXIN] = {}, st_dc[VM_MAXIN] = {};
  // (compiled passes) input a's vectors start realign[a] elements past an
  // aligned address once the strips are shifted for the outputs; REALIGN:
  // some do
  static constexpr bool REALIGN = false;
  static constexpr int realign[VM_MAXIN] = {};
  template <typename T, int HV, int NR, int NG, int GS, int E>
  static __device__ __forceinline__ void run(typename GVec<T, GS>::type (&)[NR], typename GVec<T, GS>::type (&)[NR],
                                             typename GVec<T, GS>::type (&)[NR], typename GVec<T, GS>::type (&)[NR],
                                             VmState<T, NG, GS>&, unsigned) {}
};

enum StepMode { MODE_FAST = 0, MODE_CLAMP = 1, MODE_SLOW = 2 };

// y = A x for the V*64 elements of a step starting at element `base`.  The
// row of element base + 64m + l is computed by lane l (consecutive rows on
// consecutive lanes), then handed to its owner in the canonical layout by
// shuffles.  With sp_stage each 64-row group goes through csr_group (its CSR
// range staged in LDS); without, each lane reads its row directly (csr_row).
// Either way a row is summed sequentially in CSR order, so the result does
// not depend on the path.
template <typename T, int V>
__device__ __forceinline__ void spmv_rows(const VmParams& P, int64_t base, T (&out)[4], int32_t* __restrict__ scol,
                                          T* __restrict__ sval) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int32_t* __restrict__ rowptr = P.rowptr;
  const int32_t* __restrict__ colidx = P.colidx;
  const T* __restrict__ val = (const T*)P.val;
  const T* __restrict__ x = (const T*)P.x;
  const int32_t nnz = P.nnz;
  const uint32_t nx = (uint32_t)P.nx;
  T y[V];
#pragma unroll
  for (int m = 0; m < V; ++m) {
    const int64_t g0 = base + m * WAVE;   // first row of the group
    const int64_t i = g0 + lane;
    if (g0 >= P.n1d) { y[m] = (T)0; continue; }
    if (!P.sp_stage) {
      y[m] = i < P.n1d ? csr_row<T>(rowptr, colidx, val, x, i, nnz, nx) : (T)0;
      continue;
    }
    y[m] = csr_group<T>(rowptr, colidx, val, x, g0, P.n1d, nnz, nx, scol, sval);
  }
  rows_to_owners<T, V>(y, out);
}

// The parameter block a compiled pass's step reads.  The straight-line op
// list keeps its constants in scalar registers; stream descriptors and
// bounds held live across the tile loop as well would be spilled to vector
// lanes and read back by VALU instructions at every step.  Offsetting the
// block's address by a zero the compiler cannot see through makes each step
// load what it uses again, with scalar loads from the kernel-argument
// segment.
template <class PG> __device__ __forceinline__ const VmParams& step_params(const VmParams& P) {
  if constexpr (PG::COMPILED && PG::RELOAD) {
    typedef const __attribute__((address_space(4))) char* KB;
    int64_t off = 0;
    asm volatile("" : "+s"(off));
    return *(const VmParams*)((KB)&P + off);
  } else {
    return P;
  }
}

// Address of element (row, cbase) of a stream; a lane adds its 32-bit byte
// offset, so that a compiled pass's fast-mode access is one instruction with
// a scalar base and a vector offset (no per-lane 64-bit address arithmetic).
template <typename T>
__device__ __forceinline__ const char* row_base(const VmStream& s, int64_t row, int64_t cbase) {
  return (const char*)s.base + (row * s.s_row + cbase) * (int64_t)sizeof(T);
}

// Lane l's V elements of a row whose vectors start d (0 < d < V) elements
// past an aligned address: the lane loads the aligned vector that holds its
// first element (rb: the address of the step's first column minus d, plus
// the lane's offset loff) and takes the rest from the next lane's through a
// wave shift (DPP wave_shl: lane l reads lane l + 1); the last lane loads
// the aligned vector after the strip itself.  Aligned loads instead of
// vectors that straddle two 16-byte words.
template <typename T> __device__ __forceinline__ T lane_next(const T x) {
  if constexpr (sizeof(T) == 8) {
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, 0x130, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), 0x130, 0xf, 0xf, false);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x130, 0xf, 0xf, false));
  }
}
// The loads (issued for every realigned row of a step before any is
// combined, so that they are all in flight together) ...
template <typename T, int V, typename VA>
__device__ __forceinline__ void realign_load(const char* rb, const uint32_t loff, VA& w, VA& nx) {
  w = *(const VA*)(rb + loff);
  nx = VA{};
  if ((threadIdx.x & (WAVE - 1)) == WAVE - 1) nx = *(const VA*)(rb + loff + V * sizeof(T));
}
// ... and the lane's elements from them.
template <typename T, int V, typename VA>
__device__ __forceinline__ T realign_elem(const VA& w, const VA& nx, const int d, const int v) {
  if (v < V - d) return w[v + d];
  const T t = lane_next(w[v - (V - d)]);
  return (threadIdx.x & (WAVE - 1)) == WAVE - 1 ? nx[v - (V - d)] : t;
}

// Input and output streams of a pass (compile-time for compiled passes).
template <class PG> __device__ __forceinline__ int n_in_of(const VmParams& P) {
  return PG::COMPILED ? PG::N_IN : P.n_in;
}
template <class PG> __device__ __forceinline__ int n_out_of(const VmParams& P) {
  return PG::COMPILED ? PG::N_OUT : P.n_out;
}

// Vector-mode loads of one step (MODE_FAST or MODE_CLAMP) into L: every
// stream's loads issued back to back before the first wait.  Padding slots
// of the stream bucket are not loaded: their registers are free registers of
// the pass, written before they are read.
template <typename T, int V, int U, int E, int NINB, class PG = VmInterp>
__device__ __forceinline__ void vm_load(const VmParams& P, T (&L)[NINB][E], int64_t row0, int64_t c0, unsigned vmask,
                                        const int mode, const int64_t cbase) {
  typedef T vecA __attribute__((ext_vector_type(V), aligned(sizeof(T))));
  const VmParams& Q = step_params<PG>(P);
  if constexpr (PG::COMPILED) {
    if (mode == MODE_FAST) {
      // (cbase: the step's first column, c0 - lane * V)
      const uint32_t loff = (uint32_t)((threadIdx.x & (WAVE - 1)) * V * sizeof(T));
      vecA RW[PG::REALIGN ? NINB : 1][U], RN[PG::REALIGN ? NINB : 1][U];   // realigned rows
#pragma unroll
      for (int a = 0; a < NINB; ++a) {
        if (a >= n_in_of<PG>(P)) break;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (PG::realign[a] > 0) {
            realign_load<T, V>(row_base<T>(Q.in[a], row0 + u, cbase - PG::realign[a]), loff, RW[a][u], RN[a][u]);
            continue;
          }
          const vecA w = *(const vecA*)(row_base<T>(Q.in[a], row0 + u, cbase) + loff);
#pragma unroll
          for (int v = 0; v < V; ++v) L[a][u * V + v] = w[v];
        }
      }
      if constexpr (PG::REALIGN) {
#pragma unroll
        for (int a = 0; a < NINB; ++a) {
          if (a >= n_in_of<PG>(P)) break;
          if (PG::realign[a] > 0)
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
              for (int v = 0; v < V; ++v) L[a][u * V + v] = realign_elem<T, V>(RW[a][u], RN[a][u], PG::realign[a], v);
        }
      }
      return;
    }
  }
  bool okv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) okv[u] = ((vmask >> (u * V)) & ((1u << V) - 1)) != 0;
#pragma unroll
  for (int a = 0; a < NINB; ++a) {
    if (a >= n_in_of<PG>(P)) break;
    const T* b = (const T*)Q.in[a].base;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T* p = b + (row0 + u) * Q.in[a].s_row + c0;
      if (mode == MODE_CLAMP) p = okv[u] ? p : b;
      const vecA w = *(const vecA*)p;
#pragma unroll
      for (int v = 0; v < V; ++v) L[a][u * V + v] = w[v];
    }
  }
  if (mode == MODE_CLAMP) {
#pragma unroll
    for (int a = 0; a < NINB; ++a) {
      if (PG::COMPILED && a >= n_in_of<PG>(P)) break;
#pragma unroll
      for (int e = 0; e < E; ++e) L[a][e] = ((vmask >> e) & 1) ? L[a][e] : (T)0;
    }
  }
}

// One step: U rows of the tile, V columns per lane.
//   MODE_FAST : every slot of every lane valid, unit column strides: vector
//               loads of all streams issued back to back.
//   MODE_CLAMP: validity is whole V-vectors (unit strides, widths multiple
//               of V): the same vector loads with invalid lanes pointed at
//               the stream's first element and zeroed.
//   MODE_SLOW : per-element masked accesses, one stream at a time.
// Slots n_in..NINB-1 of the bucket read a 4 KB zero page in the vector modes.
// With SPLIT the caller has instead issued the step's loads into L (see
// vm_load), and with `pf_next` (software-pipelined kernels) the loads of the next
// step (row next_row0, known to be MODE_FAST) are issued into L as soon as
// this step's values are in registers, so they are in flight during the op
// list and the stores.
// SPMV_RT (with SPMV): the SpMV prologue runs only for passes that have one
// (P.spmv), so one instantiation serves SpMV and elementwise passes alike
// (the batched executor's).
// STG: the step's staged streams (P.st_on) come from the wave's LDS slice
// `stl` at chunk row q (vm_stencil_tile), the others from global memory;
// MODE_FAST only.
template <typename T, int HV, bool SPMV, int NR, int NINB, bool SPLIT, int ROWS, bool SPMV_RT = false,
          bool STG = false, class PG = VmInterp>
__device__ __forceinline__ void vm_step(
    const VmParams& P,
    typename GVec<T, Shape<T, HV, SPMV, NR, ROWS>::GS>::type (&R0)[NR],
    typename GVec<T, Shape<T, HV, SPMV, NR, ROWS>::GS>::type (&R1)[NR],
    typename GVec<T, Shape<T, HV, SPMV, NR, ROWS>::GS>::type (&R2)[NR],
    typename GVec<T, Shape<T, HV, SPMV, NR, ROWS>::GS>::type (&R3)[NR],
    VmState<T, Shape<T, HV, SPMV, NR, ROWS>::NG, Shape<T, HV, SPMV, NR, ROWS>::GS>& G,
    T (&L)[NINB][Shape<T, HV, SPMV, NR, ROWS>::E], int64_t row0, int64_t c0, unsigned vmask, const int mode,
    const bool pf_next, const int64_t next_row0, int32_t* scol, T* sval, const T* stl, int q, const int64_t cbase) {
  typedef Shape<T, HV, SPMV, NR, ROWS> S;
  constexpr bool HEAVY = S::HEAVY;
  constexpr int V = S::V, U = S::U, TW = S::TW, E = S::E, GS = S::GS, NG = S::NG;
  static_assert(NINB <= NR, "stream bucket exceeds the register file");
  typedef typename GVec<T, GS>::type gvec;
  typedef T vecA __attribute__((ext_vector_type(V), aligned(sizeof(T))));
  const VmParams& Q = step_params<PG>(P);   // the stream descriptors
  // element e of a register lives in group e / GS, component e % GS
#define RSET(a, e, x) { const int g_ = (e) / GS; \
    if (g_ == 0) gset<T, GS>(R0[a], (e) % GS, x); else if (g_ == 1) gset<T, GS>(R1[a], (e) % GS, x); \
    else if (g_ == 2) gset<T, GS>(R2[a], (e) % GS, x); else gset<T, GS>(R3[a], (e) % GS, x); }

  // ---- loads ------------------------------------------------------------------
  if constexpr (STG) {
    constexpr int PITCH = TW + 16 / (int)sizeof(T);
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int a = 0; a < NINB; ++a) {
      if (a >= n_in_of<PG>(P)) break;
      if (PG::COMPILED ? PG::st_on[a] != 0 : P.st_on[a] != 0) {
        const int dr = PG::COMPILED ? PG::st_dr[a] : P.st_dr[a], dc = PG::COMPILED ? PG::st_dc[a] : P.st_dc[a];
        const T* src = stl + (q + dr) * PITCH + lane * V + dc;
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int v = 0; v < V; ++v) RSET(a, u * V + v, src[u * PITCH + v]);
      } else {
        const T* b = (const T*)Q.in[a].base;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const vecA w = *(const vecA*)(b + (row0 + u) * Q.in[a].s_row + c0);
#pragma unroll
          for (int v = 0; v < V; ++v) RSET(a, u * V + v, w[v]);
        }
      }
    }
  } else if (mode != MODE_SLOW && SPLIT) {
    // issued by the caller (or prefetched by the previous step) into L
#pragma unroll
    for (int a = 0; a < NINB; ++a) {
      if (a >= n_in_of<PG>(P)) break;
#pragma unroll
      for (int e = 0; e < E; ++e) RSET(a, e, L[a][e]);
    }
    if (pf_next) vm_load<T, V, U, E, NINB, PG>(P, L, next_row0, c0, (1u << E) - 1, MODE_FAST, cbase);
  } else if (PG::COMPILED && mode == MODE_FAST) {
    // a compiled pass's own streams, each row at its scalar base plus the
    // lane's offset (cbase: the step's first column)
    const uint32_t loff = (uint32_t)((threadIdx.x & (WAVE - 1)) * V * sizeof(T));
    vecA RW[PG::REALIGN ? NINB : 1][U], RN[PG::REALIGN ? NINB : 1][U];   // realigned rows
#pragma unroll
    for (int a = 0; a < NINB; ++a) {
      if (a >= n_in_of<PG>(P)) break;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (PG::realign[a] > 0) {
          realign_load<T, V>(row_base<T>(Q.in[a], row0 + u, cbase - PG::realign[a]), loff, RW[a][u], RN[a][u]);
          continue;
        }
        const vecA w = *(const vecA*)(row_base<T>(Q.in[a], row0 + u, cbase) + loff);
#pragma unroll
        for (int v = 0; v < V; ++v) RSET(a, u * V + v, w[v]);
      }
    }
    if constexpr (PG::REALIGN) {
#pragma unroll
      for (int a = 0; a < NINB; ++a) {
        if (a >= n_in_of<PG>(P)) break;
        if (PG::realign[a] > 0)
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int v = 0; v < V; ++v) RSET(a, u * V + v, (realign_elem<T, V>(RW[a][u], RN[a][u], PG::realign[a], v)));
      }
    }
  } else if (mode != MODE_SLOW) {
    // every stream of the bucket, padding slots from a zero page, in flight
    // before the first wait (a compiled pass loads its own streams only)
    T Ls[NINB][E];
    bool okv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) okv[u] = ((vmask >> (u * V)) & ((1u << V) - 1)) != 0;
#pragma unroll
    for (int a = 0; a < NINB; ++a) {
      if (PG::COMPILED && a >= n_in_of<PG>(P)) break;
      const T* b = (const T*)Q.in[a].base;
      // column stride is 1 for real streams and 0 for padding slots
      const int64_t cc = c0 & (-Q.in[a].s_col);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const T* p = b + (row0 + u) * Q.in[a].s_row + cc;
        if (mode == MODE_CLAMP) p = okv[u] ? p : b;
        const vecA w = *(const vecA*)p;
#pragma unroll
        for (int v = 0; v < V; ++v) Ls[a][u * V + v] = w[v];
      }
    }
    if (mode == MODE_CLAMP) {
#pragma unroll
      for (int a = 0; a < NINB; ++a) {
        if (PG::COMPILED && a >= n_in_of<PG>(P)) break;
#pragma unroll
        for (int e = 0; e < E; ++e) Ls[a][e] = ((vmask >> e) & 1) ? Ls[a][e] : (T)0;
      }
    }
#pragma unroll
    for (int a = 0; a < NINB; ++a) {
      if (PG::COMPILED && a >= n_in_of<PG>(P)) break;
#pragma unroll
      for (int e = 0; e < E; ++e) RSET(a, e, Ls[a][e]);
    }
  } else {
    // per-element masked loads, one stream at a time (a compiled pass
    // unrolls the streams, so its register indices stay constants)
#define DFX_SLOW_LOAD(a)                                                 \
  {                                                                      \
    const T* b = (const T*)Q.in[a].base;                                 \
    const int64_t sr = Q.in[a].s_row, sc = Q.in[a].s_col;                \
    gvec w[NG];                                                          \
    _Pragma("unroll") for (int e = 0; e < E; ++e) {                      \
      const int u = e / V, v = e % V;                                    \
      const bool ok = (vmask >> e) & 1;                                  \
      const T q = b[ok ? (row0 + u) * sr + (c0 + v) * sc : 0];           \
      gset<T, GS>(w[e / GS], e % GS, ok ? q : (T)0);                     \
    }                                                                    \
    FOR_G(Rg[a] = w[g];)                                                 \
  }
    if constexpr (PG::COMPILED) {
      // unrolled over the streams (constant register indices); the row and
      // column pass through an empty asm so that the per-element addresses
      // of this rare path are formed here, not kept live across the tile's
      // row loop by strength reduction
      int64_t row0x = row0, c0x = c0;
      asm volatile("" : "+s"(row0x), "+v"(c0x));
      {
        const int64_t row0 = row0x, c0 = c0x;
#pragma unroll
        for (int a = 0; a < NINB; ++a) {
          if (a >= n_in_of<PG>(P)) break;
          DFX_SLOW_LOAD(a)
        }
      }
    } else {
      for (int a = 0; a < n_in_of<PG>(P); ++a) DFX_SLOW_LOAD(a)
    }
#undef DFX_SLOW_LOAD
  }
  if constexpr (SPMV) {
    static_assert(U == 1, "SpMV steps take one row of the tiling");
    if (!SPMV_RT || P.spmv) {
      T y[4];
      if (!SPMV_RT && P.sp_coop) {
        // rows computed by the whole block before the tile (vm_kernel)
        extern __shared__ __attribute__((aligned(16))) char vm_dyn_lds[];
        const T* yt = (const T*)vm_dyn_lds;
        const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
        for (int v = 0; v < V; ++v) y[v] = yt[row0 * TW + V * lane + v];
      } else {
        spmv_rows<T, V>(P, row0 * TW, y, scol, sval);
      }
#pragma unroll
      for (int e = 0; e < E; ++e) RSET(NR - 1, e, y[e]);
    }
  }

  // ---- op list: the next instruction's load overlaps the current op --------
  if constexpr (PG::COMPILED) {
    PG::template run<T, HV, NR, NG, GS, E>(R0, R1, R2, R3, G, vmask);
  } else {
  constexpr bool DEFER_OK = false;
  VmInstr nx = P.code[0];
  for (int pc = 0; pc < P.n_code; ++pc) {
    const unsigned w0 = __builtin_amdgcn_readfirstlane(nx.w0), w1 = __builtin_amdgcn_readfirstlane(nx.w1);
    const unsigned w2 = __builtin_amdgcn_readfirstlane(nx.w2), w3 = __builtin_amdgcn_readfirstlane(nx.w3);
    nx = P.code[pc + 1];
    const unsigned flags = (w0 >> 8) & 0xff, slot = (w0 >> 16) & 0xff, post = w0 >> 24;
    const unsigned d = w1 & 0xff, ia = (w1 >> 8) & 0xff, ib = (w1 >> 16) & 0xff, ic = w1 >> 24;
    const unsigned op = w0 & 0xff;
    T k;
    if constexpr (sizeof(T) == 8) k = __builtin_bit_cast(double, ((uint64_t)w3 << 32) | w2);
    else k = __builtin_bit_cast(float, w2);
#include "vm_instr.inc"
  }
  }

  // ---- stores -----------------------------------------------------------------
  if (mode != MODE_SLOW) {
#pragma unroll
    for (int s = 0; s < VM_MAXOUT; ++s) {
      if (s < n_out_of<PG>(P)) {
        const int o = PG::COMPILED ? PG::out_reg[s] : P.out_reg[s];
        gvec ev[NG];
        FOR_G(ev[g] = Rg[o];)
        T* b = (T*)Q.out[s].base;
        const int64_t sr = Q.out[s].s_row;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          vecA w;
#pragma unroll
          for (int v = 0; v < V; ++v) w[v] = gget<T, GS>(ev[(u * V + v) / GS], (u * V + v) % GS);
          if (PG::COMPILED && mode == MODE_FAST)
            *(vecA*)(row_base<T>(Q.out[s], row0 + u, cbase) + (uint32_t)((threadIdx.x & (WAVE - 1)) * V * sizeof(T))) =
                w;
          else if (mode == MODE_FAST) *(vecA*)(b + (row0 + u) * sr + c0) = w;
          else if ((vmask >> (u * V)) & 1) *(vecA*)(b + (row0 + u) * sr + c0) = w;
        }
      }
    }
  } else {
#define DFX_SLOW_STORE(s, o)                                                                   \
  {                                                                                            \
    gvec ev[NG];                                                                               \
    FOR_G(ev[g] = Rg[o];)                                                                      \
    T* b = (T*)Q.out[s].base;                                                                  \
    const int64_t sr = Q.out[s].s_row, sc = Q.out[s].s_col;                                    \
    _Pragma("unroll") for (int q = 0; q < E; ++q) {                                            \
      const int u = q / V, v = q % V;                                                          \
      if ((vmask >> q) & 1) b[(row0 + u) * sr + (c0 + v) * sc] = gget<T, GS>(ev[q / GS], q % GS); \
    }                                                                                          \
  }
    if constexpr (PG::COMPILED) {
      // as the slow loads: unrolled, addresses formed here
      int64_t row0x = row0, c0x = c0;
      asm volatile("" : "+s"(row0x), "+v"(c0x));
      {
        const int64_t row0 = row0x, c0 = c0x;
#pragma unroll
        for (int s = 0; s < VM_MAXOUT; ++s) {
          if (s >= n_out_of<PG>(P)) break;
          DFX_SLOW_STORE(s, PG::out_reg[s])
        }
      }
    } else {
      for (int s = 0; s < n_out_of<PG>(P); ++s) {
        const int o = P.out_reg[s];
        DFX_SLOW_STORE(s, o)
      }
    }
#undef DFX_SLOW_STORE
  }
#undef RSET
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

// The block-sum reduction: one block of NW waves reduces F.nblocks block
// sums per reduction (at most MAXCH chunks of FINAL_CHUNK) into the 0-d
// results.  The tree is the canonical one: chunks of FINAL_CHUNK block sums
// are complete subtrees (the last one ragged), then the chunk sums form the
// same tree.  Within a chunk, wave q of a group of four reduces the aligned
// quarter [256q, 256q + 256) with block_tree, and the quarter sums combine
// as the chunk tree's two top levels; each round reduces NW / 4 chunks.  The
// chunk sums take block_tree again (by quarters when there are more than
// 256).  Every addition pairs the operands of the level-by-level pairwise
// tree, so any NW gives the same bits.  The block-sum kernel runs it with
// 16 waves; a compiled one-block pass runs it with its 4 before its own work.
template <typename T, int NW, int MAXCH> __device__ __forceinline__ void fin_sums(const VmFinal& F) {
  static_assert(FINAL_CHUNK == 16 * WAVE && NW % 4 == 0, "four waves of 256 sums per chunk");
  static_assert(MAXCH <= 4 * WAVE || NW >= 4 * VM_MAXRED, "chunk sums by quarters need four waves per reduction");
  constexpr int CPR = NW / 4;   // chunks per round
  __shared__ T fcs[VM_MAXRED][MAXCH];
  __shared__ T fws[VM_MAXRED][NW];
  const int lane = threadIdx.x & (WAVE - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  if (F.tile) {
    // one tile's summands: wave 0 adds them lane by lane over the tile's
    // rows, then columns (valid elements only), then across lanes, as the
    // wave that owns a tile accumulates them
    constexpr int V = Lanes<T>::V, TW = Lanes<T>::TW;
    if (w != 0) return;
    const T* ds = (const T*)F.partials[0];
    const int64_t c0 = -(int64_t)F.col_shift + (int64_t)lane * V;
    T acc = (T)0;
    for (int r = 0; r < RED_TH; ++r) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int64_t col = c0 + v;
        const bool ok = F.is1d ? (r * TW + col < F.n1d) : (r < F.rows && col >= 0 && col < F.cols);
        if (ok) acc = acc + ds[r * TW + lane * V + v];
      }
    }
    const T total = wave_sum(acc);
    if (lane == 0) {
      T* res = (T*)F.result[0];
      *res = F.init[0] ? total : *(volatile T*)res + total;
    }
    return;
  }
  const int q = w % 4;
  const int nch = (F.nblocks + FINAL_CHUNK - 1) / FINAL_CHUNK;
  // the top two levels over four quarter sums of a run of L values
  auto top = [](const T* s4, const int L) {
    T a = s4[0], b = s4[2];
    if (4 * WAVE < L) a = a + s4[1];
    if (12 * WAVE < L) b = b + s4[3];
    if (8 * WAVE < L) a = a + b;
    return a;
  };
  for (int c0 = 0; c0 < nch; c0 += CPR) {
    const int c = c0 + w / 4;
    const int L = c < nch ? min(FINAL_CHUNK, F.nblocks - c * FINAL_CHUNK) : 0;
    const int cnt = min(max(L - q * 4 * WAVE, 0), 4 * WAVE);
#pragma unroll
    for (int k = 0; k < VM_MAXRED; ++k) {
      if (k < F.n_red) {
        const T* a = (const T*)F.partials[k] + (int64_t)c * FINAL_CHUNK + q * 4 * WAVE;
        const T v = cnt > 0 ? block_tree(a, cnt, lane) : (T)0;
        if (lane == 0) fws[k][w] = v;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < F.n_red * CPR) {
      const int k = threadIdx.x / CPR, j = threadIdx.x % CPR;
      if (c0 + j < nch) fcs[k][c0 + j] = top(&fws[k][4 * j], min(FINAL_CHUNK, F.nblocks - (c0 + j) * FINAL_CHUNK));
    }
    __syncthreads();
  }
  T total = (T)0;
  int kr = -1;   // the reduction whose total this wave's lane 0 holds
  if (nch <= 4 * WAVE) {
    if (w < F.n_red) {
      total = nch > 0 ? block_tree(fcs[w], nch, lane) : (T)0;
      kr = w;
    }
  } else if constexpr (MAXCH > 4 * WAVE) {
    const int k = w / 4;
    if (k < F.n_red) {
      const int cnt = min(max(nch - q * 4 * WAVE, 0), 4 * WAVE);
      const T v = cnt > 0 ? block_tree(fcs[k] + q * 4 * WAVE, cnt, lane) : (T)0;
      if (lane == 0) fws[k][q] = v;
    }
    __syncthreads();
    if (w < F.n_red) {
      total = top(fws[w], nch);
      kr = w;
    }
  }
  if (kr >= 0 && lane == 0) {
    // (a vector load: the scalar cache must not keep the old value, which a
    // pass may read again after this store)
    T* res = (T*)F.result[kr];
    *res = F.init[kr] ? total : *(volatile T*)res + total;
  }
}

// Stencil staging: an interior tile of a pass whose input streams include
// shifted views of one store (the stencil of section 2: five offset views of
// one grid).  The tile's rows are processed in chunks of ST_RCH; for each
// chunk the wave loads the window's ST_RCH + 2 rows (TW + 2 columns) once,
// with 16-byte loads all in flight together, into its LDS slice, and every
// staged stream of every step then reads its shifted values from LDS
// instead of fetching them again from L2.  Other streams load as usual.
// The op list runs unchanged on the same values, so the bits are the same.
constexpr int st_pitch(int tw, int es) { return tw + 16 / es; }

template <typename T, int HV, bool SPMV, int NR, int NINB, int ROWS, class PG>
__device__ __forceinline__ void vm_stencil_tile(
    const VmParams& P, typename GVec<T, Shape<T, HV, SPMV, NR, ROWS>::GS>::type (&R0)[NR],
    typename GVec<T, Shape<T, HV, SPMV, NR, ROWS>::GS>::type (&R1)[NR],
    typename GVec<T, Shape<T, HV, SPMV, NR, ROWS>::GS>::type (&R2)[NR],
    typename GVec<T, Shape<T, HV, SPMV, NR, ROWS>::GS>::type (&R3)[NR],
    VmState<T, Shape<T, HV, SPMV, NR, ROWS>::NG, Shape<T, HV, SPMV, NR, ROWS>::GS>& G,
    T (&L)[NINB][Shape<T, HV, SPMV, NR, ROWS>::E], int64_t tr, int64_t cbase, int64_t c0, int wib) {
  typedef Shape<T, HV, SPMV, NR, ROWS> S;
  constexpr int V = S::V, U = S::U, TW = S::TW, E = S::E;
  constexpr int PITCH = st_pitch(TW, (int)sizeof(T));
  constexpr int SR = ST_RCH + 2;   // staged rows per chunk
  static_assert(2 * SR <= 63, "outstanding staged loads fit the wait counter");
  static_assert(ST_RCH % U == 0 && RED_TH % ST_RCH == 0, "stencil chunking");
  extern __shared__ __attribute__((aligned(16))) char vm_dyn_lds[];
  T* sl = (T*)vm_dyn_lds + (size_t)wib * ST_NBUF * SR * PITCH;
  const int lane = threadIdx.x & (WAVE - 1);
  const T* gb = (const T*)P.st_base;
  // stage chunk c (rows [tr * RED_TH + c * ST_RCH, + SR)) into buffer c % ST_NBUF
  auto stage = [&](int c) {
    const int64_t rb = tr * RED_TH + (int64_t)c * ST_RCH;
    T* buf = sl + (size_t)(c % ST_NBUF) * SR * PITCH;
#pragma unroll
    for (int k = 0; k < SR; ++k) {
      const T* rowp = gb + (rb + k) * P.st_srow + cbase;
      __builtin_amdgcn_global_load_lds((const void*)(rowp + lane * V),
                                       (__attribute__((address_space(3))) void*)(buf + k * PITCH), 16, 0, 0);
      if (lane < 4)
        __builtin_amdgcn_global_load_lds((const void*)((const char*)(rowp + TW) + lane * 4),
                                         (__attribute__((address_space(3))) void*)(buf + k * PITCH + TW), 4, 0, 0);
    }
  };
  constexpr int NCH = RED_TH / ST_RCH;
  // direct global-to-LDS loads: each lane's 16 bytes of a row land at lane *
  // 16 of the row's LDS line, the 16 halo bytes past the row by lanes 0..3;
  // a chunk's rows are all in flight at once, holding no registers.  With
  // two buffers the next chunk is staged while the current one is computed.
  __builtin_amdgcn_s_waitcnt(0);   // earlier LDS reads of this slice are complete
  stage(0);
  for (int c = 0; c < NCH; ++c) {
    if constexpr (ST_NBUF > 1) {
      if (c + 1 < NCH) {
        // the buffer chunk c + 1 overwrites was last read two chunks ago:
        // wait for LDS reads only (lgkmcnt 0), then issue its loads
        __builtin_amdgcn_s_waitcnt(0xC07F);
        stage(c + 1);
        // chunk c's loads are complete when at most chunk c + 1's 2 * SR
        // loads (and nothing older) are outstanding: vmcnt(2 * SR)
        __builtin_amdgcn_s_waitcnt(((2 * SR) & 0xF) | (((2 * SR) >> 4) << 14) | 0x70 | 0xF00);
      } else {
        __builtin_amdgcn_s_waitcnt(0);
      }
    } else {
      __builtin_amdgcn_s_waitcnt(0);
    }
    const T* cur = sl + (size_t)(c % ST_NBUF) * SR * PITCH;
    for (int q = 0; q < ST_RCH; q += U)
      vm_step<T, HV, SPMV, NR, NINB, false, ROWS, false, true, PG>(P, R0, R1, R2, R3, G, L,
                                                               tr * RED_TH + (int64_t)c * ST_RCH + q, c0,
                                                               (1u << E) - 1, MODE_FAST, false, 0, nullptr, nullptr,
                                                               cur, q, cbase);
    if constexpr (ST_NBUF == 1)
      if (c + 1 < NCH) {
        __builtin_amdgcn_s_waitcnt(0);
        stage(c + 1);
      }
  }
}

// SpMV passes keep four waves per SIMD (one tile per wave fills the chip
// only if all of them are resident)
#ifndef DFX_SPMV_WAVES
#define DFX_SPMV_WAVES 4
#endif
// STEN: the stencil-staging variant of the arithmetic kernel (a separate
// instantiation, so the other kernels keep their registers).
// A compiled pass states its own waves-per-SIMD target (PG::WAVES).
template <typename T, int HV, bool SPMV, int NR, int NINB, int ROWS, bool STEN = false, class PG = VmInterp>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(PG::COMPILED ? PG::WAVES : SPMV && HV == 0 ? DFX_SPMV_WAVES : 1)))
void vm_kernel(const VmParams P) {
  typedef Shape<T, HV, SPMV, NR, ROWS> S;
  constexpr int V = S::V, U = S::U, TW = S::TW, E = S::E, GS = S::GS, NG = S::NG;
  typedef typename GVec<T, GS>::type gvec;
  __shared__ T tsum[VM_MAXRED][4 * VM_MAXTPW];  // this block's tile sums
  // SpMV kernels: per wave, the staged CSR range of one 64-row group
  __shared__ int32_t sp_col[SPMV ? BLOCK / WAVE : 1][SPMV ? SP_CAP : 1];
  __shared__ T sp_val[SPMV ? BLOCK / WAVE : 1][SPMV ? SP_CAP : 1];

  // a compiled one-block pass first reduces an earlier pass's block sums
  // (P.fin), in place of the block-sum kernel's launch
  if constexpr (PG::COMPILED) {
    if (P.fin.n_red > 0) {
      fin_sums<T, BLOCK / WAVE, FIN_MAX_CHUNKS>(P.fin);
      __syncthreads();
    }
  }

  // One-tile SpMV passes (sp_coop, one block): the block's four waves first
  // compute the tile's rows, four 64-row groups per lane at once, into
  // dynamic LDS; the wave that owns the tile then reads them there.  Each
  // row is summed in CSR order as always, so the bits do not change.
  if constexpr (SPMV) {
    if (P.sp_coop) {
      extern __shared__ __attribute__((aligned(16))) char vm_dyn_lds[];
      T* yt = (T*)vm_dyn_lds;
      const int lane_ = threadIdx.x & (WAVE - 1);
      const int w_ = threadIdx.x / WAVE;
      constexpr int GPW = TW * RED_TH / WAVE / (BLOCK / WAVE);   // 64-row groups per wave
      const uint32_t nx = (uint32_t)P.nx;
#ifndef DFX_COOP_ROWS
#define DFX_COOP_ROWS 2
#endif
      constexpr int CR = DFX_COOP_ROWS;   // rows walked at once per lane
      for (int k0 = 0; k0 < GPW; k0 += CR) {
        int64_t ii[CR];
        bool ok[CR];
        T yy[CR];
#pragma unroll
        for (int m = 0; m < CR; ++m) {
          ii[m] = (int64_t)(w_ * GPW + k0 + m) * WAVE + lane_;
          ok[m] = ii[m] < P.n1d;
        }
        csr_rows<T, CR>(P.rowptr, P.colidx, (const T*)P.val, (const T*)P.x, ii, ok, P.nnz, nx, yy);
#pragma unroll
        for (int m = 0; m < CR; ++m)
          if (ok[m]) yt[ii[m]] = yy[m];
      }
      __syncthreads();
    }
  }

  gvec R0[NR], R1[NR], R2[NR], R3[NR];  // groups beyond NG are unused (and dropped)
  VmState<T, NG, GS> G;
#pragma unroll
  for (int k = 0; k < VM_MAXBC; ++k) {
    if (k < P.n_bc) {
      const gvec v = (gvec)(*(const T*)P.bc[k]);
      const int r = PG::COMPILED ? PG::bc_reg[k] : P.bc_reg[k];
      FOR_G(Rg[r] = v;)
    }
  }
#pragma unroll
  for (int g = 0; g < NG; ++g) G.z[g] = (gvec)(T)0;

  const int lane = threadIdx.x & (WAVE - 1);
  // wave-uniform by construction; readfirstlane lets the compiler keep the
  // tile and row bookkeeping (and the step-mode branches) in scalar registers
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  // XCD-aware numbering: consecutive blocks land on different XCDs, so give
  // each XCD a contiguous range of logical blocks (and therefore of tiles).
  int lb = blockIdx.x;
  // (SpMV passes keep hardware order: the gathered vector is shared by
  // neighbouring row blocks on every XCD through the MALL, which measured
  // slightly faster than XCD-contiguous ranges)
#ifndef DFX_SPMV_XCD_REMAP
#define DFX_SPMV_XCD_REMAP 0
#endif
  if ((P.grid & 7) == 0 && (!SPMV || DFX_SPMV_XCD_REMAP)) lb = (blockIdx.x & 7) * (P.grid >> 3) + (blockIdx.x >> 3);
  const int64_t gw = (int64_t)lb * (BLOCK / WAVE) + wib;
  // rows [r_lo, r_hi) of each tile: all of them, or the wave's share of a
  // tile under row_split (passes without reductions)
  // (red_split, compiled passes with one reduction: block lb owns tile lb
  // and its four waves take a quarter of the rows each)
  const int split = P.row_split > 1 ? P.row_split : 1;
  const bool rsplit = PG::COMPILED && P.red_split != 0;
  const int rsb = rsplit ? P.red_split : 1;   // blocks per tile
  const int64_t t_begin = rsplit ? (int64_t)(lb / rsb) : split > 1 ? gw / split : gw * P.tiles_per_wave;
  const int64_t t_end = min(t_begin + ((split > 1 || rsplit) ? 1 : P.tiles_per_wave), P.n_tiles);
  const int r_lo = rsplit ? ((lb % rsb) * 4 + wib) * (RED_TH / (4 * rsb))
                          : split > 1 ? (int)(gw % split) * (RED_TH / split) : 0;
  const int r_hi = r_lo + (rsplit ? RED_TH / (4 * rsb) : RED_TH / split);

  // Arithmetic passes are stream-bound: their loads are software-pipelined
  // one step ahead inside a tile (up to four streams: the wider bucket would
  // lose a wave of occupancy to the prefetch registers).  Transcendental
  // passes are not (DFX_HEAVY_PF=1 pipelines them too: 2 % faster for
  // Black-Scholes FP64 with the load buffer, but the buffer costs a wave).
#ifndef DFX_PREFETCH_MAX_STREAMS
#define DFX_PREFETCH_MAX_STREAMS 4
#endif
#ifndef DFX_HEAVY_PF
#define DFX_HEAVY_PF 0
#endif
  constexpr bool PF = !SPMV && NINB <= DFX_PREFETCH_MAX_STREAMS && (!S::HEAVY || DFX_HEAVY_PF || PG::HEAVY_PF);
  // FP32 transcendental kernels load through vm_load (padding slots
  // skipped).  The FP64 ones load straight into the register file: without
  // the separate load buffer they fit three waves per SIMD instead of two
  // (1.05 against 1.26 ms for Black-Scholes FP64 over 2^26 options).
#ifndef DFX_HEAVY_SPLIT
#define DFX_HEAVY_SPLIT (sizeof(T) == 4)
#endif
  constexpr bool SPLIT = PF || (S::HEAVY && !SPMV && DFX_HEAVY_SPLIT);
  T L[NINB][E];
  for (int64_t t = t_begin; t < t_end; ++t) {
    const int64_t tr = t / P.strips;
    const int64_t ts = t - tr * P.strips;
    const int64_t cbase = ts * TW - P.col_shift;
    const int64_t c0 = cbase + (int64_t)lane * V;
    G.acc0 = G.acc1 = G.acc2 = G.acc3 = (T)0;
    if constexpr (PG::COMPILED) {
      extern __shared__ __attribute__((aligned(16))) char vm_dyn_lds[];
      G.dsum = !rsplit ? nullptr : rsb > 1 ? (T*)P.red_partials[0] : (T*)vm_dyn_lds;
    }
    bool have = false;  // L already holds this step's values (prefetched)
    bool staged = false;
    if constexpr (STEN && !SPMV && HV == 0) {
      // stencil passes: a whole interior tile whose staged window lies in
      // the store goes through LDS (vm_stencil_tile)
      staged = split == 1 && P.st_n > 0 && P.unit_cols && (tr + 1) * RED_TH <= P.rows && cbase + TW <= P.cols &&
               ((tr + 1) * RED_TH + 1) * P.st_srow + cbase + TW + 16 / (int)sizeof(T) <= P.st_lim;
      if (staged) vm_stencil_tile<T, HV, SPMV, NR, NINB, ROWS, PG>(P, R0, R1, R2, R3, G, L, tr, cbase, c0, wib);
    }
    for (int r = r_lo; r < (staged ? r_lo : r_hi); r += U) {
      // the step's bounds (a compiled pass reads them again at every step;
      // the interpreter's are the kernel argument's, kept live)
      const VmParams* CP = nullptr;
      if constexpr (PG::COMPILED && PG::RELOAD) CP = &step_params<PG>(P);
#define DFX_C(f) (PG::COMPILED && PG::RELOAD ? CP->f : P.f)
      const int64_t row0 = tr * RED_TH + r;
      if (row0 >= DFX_C(rows)) break;
      // (realigned inputs read up to V elements either side of the strip)
      const bool interior = DFX_C(is1d) ? ((row0 + U) * TW <= DFX_C(n1d))
                                        : (row0 + U <= DFX_C(rows) && cbase >= (PG::REALIGN ? V : 0) &&
                                           cbase + TW + (PG::REALIGN ? V : 0) <= DFX_C(cols));
      int mode = MODE_FAST;
      unsigned vmask = (1u << E) - 1;
      if (!(DFX_C(unit_cols) && interior)) {
        mode = DFX_C(vec_cols) ? MODE_CLAMP : MODE_SLOW;
        vmask = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int64_t row = row0 + e / V, col = c0 + e % V;
          const bool ok = DFX_C(is1d) ? (row * TW + col < DFX_C(n1d))
                                      : (row < DFX_C(rows) && col >= 0 && col < DFX_C(cols));
          vmask |= (ok ? 1u : 0u) << e;
        }
      }
      bool next_fast = false;
      if constexpr (SPLIT)
        if (mode != MODE_SLOW && !(have && mode == MODE_FAST))
          vm_load<T, V, U, E, NINB, PG>(P, L, row0, c0, vmask, mode, cbase);
      if constexpr (PF) {
        const int64_t nr = row0 + U;
        next_fast = r + U < r_hi && DFX_C(unit_cols) &&
                    (DFX_C(is1d) ? ((nr + U) * TW <= DFX_C(n1d))
                                 : (nr + U <= DFX_C(rows) && cbase >= (PG::REALIGN ? V : 0) &&
                                    cbase + TW + (PG::REALIGN ? V : 0) <= DFX_C(cols)));
      }
      if constexpr (PG::COMPILED) G.drow = r;
      vm_step<T, HV, SPMV, NR, NINB, SPLIT, ROWS, false, false, PG>(P, R0, R1, R2, R3, G, L, row0, c0, vmask, mode,
                                                                    next_fast, row0 + U, sp_col[SPMV ? wib : 0],
                                                                    sp_val[SPMV ? wib : 0], nullptr, 0, cbase);
#undef DFX_C
      have = next_fast;
    }
    // ---- tile sums into the block's LDS row ---------------------------------------
    if (P.n_red > 0 && !rsplit) {
      const int j = wib * (int)P.tiles_per_wave + (int)(t - t_begin);
      T a0 = wave_sum(G.acc0);
      if (lane == 0) tsum[0][j] = a0;
      if (P.n_red > 1) { T a1 = wave_sum(G.acc1); if (lane == 0) tsum[1][j] = a1; }
      if (P.n_red > 2) { T a2 = wave_sum(G.acc2); if (lane == 0) tsum[2][j] = a2; }
      if (P.n_red > 3) { T a3 = wave_sum(G.acc3); if (lane == 0) tsum[3][j] = a3; }
    }
  }

  if (P.n_red == 0) return;
  if constexpr (PG::COMPILED) {
    if (rsplit) {
      // several blocks: the summands are in the workspace, for the
      // block-sum reduction (VmFinal.tile)
      if (rsb > 1) return;
      // the block's one tile: wave 0 adds the summands lane by lane over the
      // tile's rows, then columns (valid elements only), the order in which
      // one wave would have accumulated them; the tile sum is the block sum
      __syncthreads();
      if (wib != 0 || t_begin >= P.n_tiles) return;
      extern __shared__ __attribute__((aligned(16))) char vm_dyn_lds[];
      const T* ds = (const T*)vm_dyn_lds;
      const int64_t tr = t_begin / P.strips;
      const int64_t c0 = (t_begin - tr * P.strips) * TW - P.col_shift + (int64_t)lane * V;
      T acc = (T)0;
      for (int r = 0; r < RED_TH; ++r) {
        const int64_t row = tr * RED_TH + r;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const int64_t col = c0 + v;
          const bool ok = P.is1d ? (row * TW + col < P.n1d) : (row < P.rows && col >= 0 && col < P.cols);
          if (ok) acc = acc + ds[r * TW + lane * V + v];
        }
      }
      const T v = wave_sum(acc);
      if (lane == 0) {
        if (P.red_direct) {
          T* res = (T*)P.red_result[0];
          *res = P.red_init[0] ? v : *res + v;
        } else {
          ((T*)P.red_partials[0])[lb] = v;
        }
      }
      return;
    }
  }
  // ---- block subtree: the 4 * tiles_per_wave tiles from lb * 4 * tiles_per_wave
  // form one aligned subtree of the tile tree; wave k reduces reduction k.
  __syncthreads();
  if (wib >= P.n_red) return;
  const int64_t blk0 = (int64_t)lb * 4 * P.tiles_per_wave;
  if (blk0 >= P.n_tiles) return;
  const int cnt = (int)min((int64_t)4 * P.tiles_per_wave, P.n_tiles - blk0);
  const T v = block_tree(tsum[wib], cnt, lane);
  if (lane == 0) {
    if (P.red_direct) {
      T* res = (T*)P.red_result[wib];
      *res = P.red_init[wib] ? v : *res + v;
    } else {
      ((T*)P.red_partials[wib])[lb] = v;
    }
  }
}

#ifndef __HIPCC_RTC__
// Launch one pass on a tier's kernels: element type, SpMV prologue and
// stream bucket select the instantiation.
template <int HV, int NR, int NB0, int NB1, int NB2, int ROWS = 0>
int launch_tier(const VmParams& P, int is_f64, int nb, hipStream_t st) {
  const dim3 g(P.grid), b(BLOCK);
  const bool sp = P.spmv != 0;
  const bool sten = HV == 0 && ROWS == 0 && !sp && P.st_n > 0 && nb != NB0;
  const size_t dyn = vm_dyn_lds_bytes(P, sten);
#define DFX_L(T, SP)                                                                                \
  {                                                                                                 \
    if (nb == NB0) hipLaunchKernelGGL((vm_kernel<T, HV, SP, NR, NB0, ROWS>), g, b, dyn, st, P);     \
    else if (nb == NB1) hipLaunchKernelGGL((vm_kernel<T, HV, SP, NR, NB1, ROWS>), g, b, dyn, st, P); \
    else hipLaunchKernelGGL((vm_kernel<T, HV, SP, NR, NB2, ROWS>), g, b, dyn, st, P);               \
  }
  if constexpr (ROWS > 0) {
    if (sp) return (int)hipErrorInvalidValue;   // SpMV steps take one row in every variant
    if (is_f64) DFX_L(double, false) else DFX_L(float, false)
  } else if (sten) {
    // stencil staging (three or more staged streams: the wider buckets)
    if (is_f64) {
      if (nb == NB1) hipLaunchKernelGGL((vm_kernel<double, HV, false, NR, NB1, 0, true>), g, b, dyn, st, P);
      else hipLaunchKernelGGL((vm_kernel<double, HV, false, NR, NB2, 0, true>), g, b, dyn, st, P);
    } else {
      if (nb == NB1) hipLaunchKernelGGL((vm_kernel<float, HV, false, NR, NB1, 0, true>), g, b, dyn, st, P);
      else hipLaunchKernelGGL((vm_kernel<float, HV, false, NR, NB2, 0, true>), g, b, dyn, st, P);
    }
  } else {
    if (is_f64) {
      if (sp) DFX_L(double, true) else DFX_L(double, false)
    } else {
      if (sp) DFX_L(float, true) else DFX_L(float, false)
    }
  }
#undef DFX_L
  return (int)hipGetLastError();
}

// Waves of one non-SpMV kernel of a tier that one compute unit holds at once
// (its occupancy), from the runtime's occupancy calculator.
template <int HV, int NR, int NB0, int NB1, int NB2, int ROWS = 0>
int tier_waves_per_cu(int is_f64, int nb) {
  int blocks = 0;
  const void* f = nullptr;
  if (is_f64)
    f = nb == NB0 ? (const void*)&vm_kernel<double, HV, false, NR, NB0, ROWS>
      : nb == NB1 ? (const void*)&vm_kernel<double, HV, false, NR, NB1, ROWS>
                  : (const void*)&vm_kernel<double, HV, false, NR, NB2, ROWS>;
  else
    f = nb == NB0 ? (const void*)&vm_kernel<float, HV, false, NR, NB0, ROWS>
      : nb == NB1 ? (const void*)&vm_kernel<float, HV, false, NR, NB1, ROWS>
                  : (const void*)&vm_kernel<float, HV, false, NR, NB2, ROWS>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, BLOCK, 0) != hipSuccess) return 0;
  return blocks * (BLOCK / WAVE);
}

#endif  // __HIPCC_RTC__

}  // namespace dfx
