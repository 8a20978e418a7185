// Compiled passes: a memoised pass's op list turned into a kernel of its own.
//
// The interpreter (vm_kernel with VmInterp) decodes a pass's instructions at
// run time.  A compiled pass instantiates the same kernel template with a
// program type generated for that pass: every instruction becomes one call
// of vm_instr with its fields as constants, and the output and broadcast
// register maps become constants, so the dispatch, the indexed register
// moves and the unused registers disappear.  Tiling, loads, stores and the
// reduction tree are the kernel template's own, so a compiled pass returns
// the same bits as the interpreted one.  This is the counterpart of the
// paper's JIT code generation of fused tasks (section 6): kernels are built
// at run time with hiprtc for the device's architecture.
//
// Compilation runs on one background thread (or in the caller, when asked
// to); a pass keeps running interpreted until its kernel is ready.  Kernels
// are cached per process by their entry (the instantiation) and source
// text, and optionally on disk.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "vm.h"

namespace dfx {

// What a pass's kernel is instantiated with (the interpreter's choice of
// variant for the same pass, see launch_vm and launch_tier).
struct JitVariant {
  int is_f64 = 1;
  int hv = 0;      // op set: 0 arithmetic, 1 sqrt/exp/log/erf, 2 also pow
  int nr = 8;      // registers
  int nb = 2;      // input-stream bucket
  int rows = 0;    // rows per step (0: the kernel's rule)
  int spmv = 0;
  int sten = 0;    // stencil staging variant
  int waves = 2;   // waves-per-SIMD target given to the compiler
  int heavy_pf = 0; // transcendental pass: load the next step during this one
  int reload = -1;  // parameters reloaded at every step (step_params): 1, 0, -1 the default rule
};

// A pass's program: its instructions and register maps.
struct JitProgram {
  int n_in = 0, n_out = 0;   // input and output streams
  std::vector<VmInstr> code;
  std::vector<int32_t> out_reg, bc_reg;
  std::vector<int32_t> st_on, st_dr, st_dc;   // stencil staging map (empty: none)
  std::vector<int32_t> realign;   // per input: elements past alignment after the strip shift (empty: none)
};

struct JitEntry;

// The kernel variant of a compiled pass of `tier` with `n_in` streams, SpMV
// prologue `spmv`, `st_n` staged streams and the planner's rows per step:
// the interpreter's, except that FP32 transcendental passes take one row
// per step (their straight-line code keeps few registers that way, so more
// waves are resident) and prefetch the next step's loads, and FP64 ones
// take two.  DFX_JIT_ROWS (0, 1 or 2) and DFX_JIT_WAVES override the
// choice for non-SpMV, unstaged passes, DFX_JIT_PF (0 or 1) the prefetch,
// DFX_JIT_RELOAD (0 or 1) whether parameters are reloaded at every step.
JitVariant jit_variant(int is_f64, int tier, int n_in, int spmv, int st_n, int rows);

// Source text of the pass's kernel and the name expression of its entry.
std::string jit_source(const JitVariant& v, const JitProgram& g, std::string* name_expr);

// The process-wide entry for this entry and source: created and compiled (queued
// for the background thread, or compiled now when `sync`) on first
// request; later requests share it.  Never null.
std::shared_ptr<JitEntry> jit_request(const std::string& src, const std::string& name_expr, bool sync);

// The entry's kernel on the current device `device`, loading its code
// object there on first use when `may_load` (module loading is kept out of
// stream capture).  Null while compiling, after a failure, or when not
// loaded and !may_load.
hipFunction_t jit_function(JitEntry& e, int device, bool may_load);

// 1: compiled, 0: pending, -1: failed (log in *log when given).
int jit_state(const JitEntry& e, std::string* log = nullptr);

// Blocks until no compilation is queued or running.
void jit_wait_idle();

struct JitCounters {
  int64_t compiled = 0, failed = 0, disk_hits = 0;
  int32_t pending = 0;
  double seconds = 0.0;   // compile time spent (disk hits excluded)
};
JitCounters jit_counters();

// Directory of the on-disk code-object cache ("" turns it off).
void jit_set_cache_dir(const std::string& dir);

}  // namespace dfx
