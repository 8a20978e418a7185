// Kernel-side description of one fused pass, shared by the host planner and
// the HIP executor.  Plain data only: it is passed by value as the kernel
// argument block.
#pragma once
#include <stdint.h>
#ifndef __HIPCC_RTC__
#include <stddef.h>
#endif

namespace dfx {

constexpr int VM_NREG = 16;      // virtual registers per element slot, large register file
constexpr int VM_NREG_LIGHT = 8; // small register file
constexpr int VM_MAXIN = 10;    // input streams
constexpr int VM_MAXOUT = 6;    // output streams
constexpr int VM_MAXBC = 8;     // broadcast 0-d inputs
constexpr int VM_MAXRED = 4;    // reductions per pass
constexpr int VM_MAXCODE = 112; // instructions per pass
// The SpMV row result lands in the last register of the file (NR - 1).

// Canonical reduction tiling.  The iteration space is a set of rows of at
// most TW elements (a 2-D space's rows, or a 1-D space cut into rows of TW);
// a tile is RED_TH consecutive rows of one TW-wide column strip.  Lane l of
// the wave that owns a tile holds columns [l*V, l*V+V) of the strip and
// accumulates its elements sequentially, rows ascending then columns; the 64
// lane sums are combined by an xor butterfly (32, 16, 8, 4, 2, 1), and the
// tile sums by a pairwise power-of-two tree over the tile index.  V = 16
// bytes / element size.  Nothing here depends on the launch configuration.
//
// Evaluation of the tile tree: a wave owns a power-of-two run of at most
// VM_MAXTPW tiles starting at a multiple of the run length, so the 4 runs of
// a block form one aligned subtree, which the block reduces in LDS; a
// one-block kernel launched after the pass reduces the block sums (subtrees
// of equal size) with the same tree.  Kernel boundaries order the two, so no
// device-scope fence is needed inside the pass.
constexpr int RED_TH = 32;
constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int VM_MAXTPW = 64;      // tiles per wave (power of two)
constexpr int FINAL_CHUNK = 1024;  // tree level width processed in LDS (power of two)
constexpr int FINAL_BLOCK = 1024;  // threads of the block-sum kernel (= FINAL_CHUNK)
#ifndef DFX_ST_RCH
#define DFX_ST_RCH 8
#endif
#ifndef DFX_ST_NBUF
#define DFX_ST_NBUF 1
#endif
constexpr int ST_RCH = DFX_ST_RCH;   // output rows per stencil staging chunk (ST_RCH + 2 rows staged)
constexpr int ST_NBUF = DFX_ST_NBUF; // staging buffers per wave (2: the next chunk loads during this one)

template <typename T> struct Lanes;
template <> struct Lanes<double> { static constexpr int V = 2, TW = WAVE * 2; };
template <> struct Lanes<float> { static constexpr int V = 4, TW = WAVE * 4; };

enum VmOp : uint8_t {
  VO_MOV = 0, VO_NEG, VO_ABS, VO_SQUARE, VO_ADD, VO_SUB, VO_MUL, VO_DIV, VO_MAX, VO_MIN,
  VO_RSUB, VO_RDIV,   // b - a, b / a: the accumulator as the right operand
  VO_ADDI, VO_SUBI, VO_RSUBI, VO_MULI, VO_DIVI, VO_RDIVI, VO_FILL,
  VO_RED, VO_REDPROD,
  // ops below need the transcendental kernel variant
  VO_SQRT, VO_EXP, VO_LOG, VO_ERF, VO_POW,
  VO_COUNT
};
constexpr int VO_FIRST_HEAVY = VO_SQRT;

// The interpreter is an accumulator machine: the previous instruction's
// result stays in the accumulator, which each instruction updates in place.
enum VmFlag : uint8_t {
  VF_A_ACC = 1,   // operand a is the previous instruction's result (the accumulator)
  VF_B_ACC = 2,   // operand b is the previous instruction's result
  VF_WB = 4,      // write the result to register dst
  VF_B_REG = 8,   // operand b is register b (binary ops)
  VF_A_REG = 16,  // operand a is register a: loaded into the accumulator first
  VF_C_REG = 32   // the post op's operand b is register c
};

// One instruction, four 32-bit words fetched with one scalar load:
//   w0 = op | flags << 8 | slot << 16 | post << 24
//   w1 = dst | a << 8 | b << 16 | c << 24  (register indices, extracted by bit-field)
//   w2, w3 = the immediate in the pass's element type (FP32: w2 only)
// slot is the reduction slot of RED/REDPROD.  post (0 = none, else a VmOp + 1)
// is a second op applied to the accumulator after the first, with operand b
// from register c when it is binary (a two-op superinstruction).
struct VmInstr {
  uint32_t w0, w1, w2, w3;
};
inline VmInstr vm_instr(unsigned op, unsigned dst, unsigned a, unsigned b, unsigned flags, unsigned slot,
                        double imm, bool f64, unsigned post = 0, unsigned c = 0) {
  VmInstr I{op | flags << 8 | slot << 16 | post << 24, dst | a << 8 | b << 16 | c << 24, 0, 0};
  if (f64) {
    uint64_t u;
    __builtin_memcpy(&u, &imm, 8);
    I.w2 = (uint32_t)u;
    I.w3 = (uint32_t)(u >> 32);
  } else {
    const float f = (float)imm;
    __builtin_memcpy(&I.w2, &f, 4);
  }
  return I;
}

// Kernel tiers: register file size and op set.  Tiers 0-2 take up to 6 input
// streams; tier 3 takes up to VM_MAXIN.
enum VmTier {
  TIER_ARITH = 0,   // arithmetic ops, 8 registers
  TIER_TRANS8 = 1,  // plus sqrt/exp/log/erf, 8 registers
  TIER_TRANS16 = 2, // plus sqrt/exp/log/erf, 16 registers
  TIER_POW = 3      // every op, 16 registers, up to VM_MAXIN streams
};

struct VmStream {
  const void* base;     // address of the element at row 0, column 0
  int64_t s_row, s_col; // element strides
};

// The block-sum kernel: reduces `nblocks` block sums per reduction and stores
// (init) or accumulates into the 0-d result.
struct VmFinal {
  int32_t n_red, nblocks;
  const void* partials[VM_MAXRED];
  void* result[VM_MAXRED];
  int32_t init[VM_MAXRED];
  // tile: 1 when partials[0] holds the summands of a one-tile pass's single
  // reduction (red_split over several blocks) at their places in the tile,
  // to be added in the canonical order (valid elements of the tile's space:
  // is1d, n1d, rows, cols, col_shift as in VmParams)
  int32_t tile, is1d, col_shift;
  int64_t n1d, rows, cols;
};

// Block sums a one-block compiled pass reduces before its own work (an
// earlier pass's VmFinal), at most FIN_MAX_CHUNKS chunks of FINAL_CHUNK.
constexpr int FIN_MAX_CHUNKS = 64;

struct VmParams {
  int32_t n_code, n_in, n_out, n_bc, n_red;
  int32_t is1d;         // 1: space of n1d elements cut into rows of TW
  int32_t spmv;         // 1: row result of y = A x lands in VM_SPMV_REG first
  int32_t grid;         // blocks launched
  int32_t unit_cols;    // every stream has column stride 1 (padding slots 0)
  int32_t vec_cols;     // unit_cols and the row width is a multiple of V
  int64_t rows, cols;   // 2-D space; for 1-D: rows = ceil(n1d / TW), cols = TW
  int64_t n1d;
  int64_t n_tiles, strips;  // tiles, tiles per tile-row
  int64_t tiles_per_wave;  // power of two, at most VM_MAXTPW
  // row_split (a power of two dividing RED_TH, a multiple of the rows per
  // step; passes without reductions, one tile per wave): waves per tile,
  // wave k of a tile taking rows [k, k + 1) * RED_TH / row_split.  No
  // reduction order is involved, so the split changes no bit.
  int32_t row_split;
  // red_split (compiled passes with one reduction): B = red_split blocks
  // per tile, whose 4B waves take RED_TH / 4B of its rows each and stage the
  // reduction's summands (the values one wave would accumulate) at their
  // places in the tile: with B = 1 in dynamic LDS, wave 0 then adding them
  // in the canonical order, so the tile sum has the bits of one wave's; with
  // B > 1 (a one-tile pass) in the block-sum workspace, added in the same
  // order by the block-sum reduction (VmFinal.tile)
  int32_t red_split;
  // col_shift (2-D passes without reductions, 0 <= col_shift < V): strips
  // start col_shift columns early (strip s covers columns [s * TW -
  // col_shift, (s + 1) * TW - col_shift)), so that the output streams' 16-byte
  // vectors are aligned; columns outside [0, cols) are masked.
  int32_t col_shift;
  VmStream in[VM_MAXIN];
  VmStream out[VM_MAXOUT];
  int32_t out_reg[VM_MAXOUT];
  int32_t bc_reg[VM_MAXBC];
  const void* bc[VM_MAXBC];
  void* red_partials[VM_MAXRED];   // one subtree sum per block
  // red_direct: the pass's tiles form one block's subtree (one block
  // reduces), so that block's sum is the whole tree's: the block writes the
  // 0-d result itself (red_result[k] = red_init[k] ? sum : red_result[k] +
  // sum, the block-sum kernel's arithmetic for one block sum) and no
  // block-sum kernel follows
  int32_t red_direct;
  int32_t red_init[VM_MAXRED];
  void* red_result[VM_MAXRED];
  const int32_t* rowptr;           // SpMV operands (n1d + 1 row pointers)
  const int32_t* colidx;
  const void* val;
  const void* x;
  int32_t nnz;                     // length of colidx and val
  int64_t nx;                      // length of x
  int32_t sp_stage;                // stage each 64-row group's CSR range in LDS
  int32_t sp_coop;                 // one-tile pass: the block's four waves compute its rows into LDS first
  // Stencil staging (arithmetic 2-D passes): input streams that are shifted
  // views of one store.  Element (row, col) of staged stream a is element
  // (row + st_dr[a], col + st_dc[a]) of the window at st_base (row stride
  // st_srow, st_lim elements readable from st_base).
  int32_t st_n;                    // staged streams (0: none)
  int8_t st_on[VM_MAXIN], st_dr[VM_MAXIN], st_dc[VM_MAXIN];
  const void* st_base;
  int64_t st_srow, st_lim;
  // (compiled one-block passes) an earlier pass's block sums to reduce into
  // its 0-d results first, with the block-sum kernel's tree (fin.n_red 0:
  // none); the host attaches it in place of that kernel's launch
  VmFinal fin;
  VmInstr code[VM_MAXCODE + 1];    // one spare entry: the kernel prefetches code[pc + 1]
};

// Dynamic LDS bytes of a pass's launch: a one-tile SpMV pass stages the
// tile's rows, a red_split pass its reduction's summands (either way RED_TH
// rows of 16 bytes per lane, FP64 and FP32 alike); a
// stencil-staged pass gives each wave ST_NBUF buffers of ST_RCH + 2 rows of
// TW elements plus 16 bytes of halo.
inline size_t vm_dyn_lds_bytes(const VmParams& P, bool sten) {
  return (P.spmv && P.sp_coop) || P.red_split ? (size_t)RED_TH * WAVE * 16
         : sten              ? (size_t)(BLOCK / WAVE) * ST_NBUF * (ST_RCH + 2) * (WAVE * 16 + 16)
                             : 0;
}

// Allocation-free execution (dfx_flush_noalloc): the block sums of a pass's
// reductions go to a fixed device array of NOALLOC_BLOCKS sums per reduction
// slot instead of the plan's workspace.
constexpr int NOALLOC_BLOCKS = 16384;
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)NOALLOC_BLOCKS * VM_MAXRED * 8;

}  // namespace dfx
