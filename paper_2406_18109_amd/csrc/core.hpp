// Host-side data structures of the fused task-stream executor.
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <deque>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/dfx.h"
#include "jit.h"
#include "vm.h"

namespace dfx {

int launch_vm(const VmParams& P, int is_f64, int tier, int rows, hipStream_t stream);
int arith_waves_per_cu(int is_f64, int n_in, int rows);
int launch_vm_final(const VmFinal& F, int is_f64, hipStream_t stream);
int stream_bucket(int n_in, int tier);
int scratch_address(int device, void** out);
struct Ctx;
int batch_record_pass(Ctx& c, const VmParams& P, const VmFinal& F, int dtype, int tier);
void batch_record_drop(Ctx& c);

enum PartKind { PK_NONE = 0, PK_TILING = 1, PK_IMAGE = 2 };

// Store(id, shape) of section 3.1, with split reference counts (section 5.1).
struct StoreRec {
  int64_t id = 0;
  int ndim = 0;
  int64_t shape[DFX_MAX_DIM] = {0, 0, 0, 0};
  int dtype = DFX_F64;
  int64_t elems = 1;
  size_t bytes = 0;
  void* ptr = nullptr;
  bool external = false;
  int app_refs = 1;     // references held by the application
  int pending = 0;      // references held by tasks still in the window
};

struct ProjRec {
  int nin = 0, nout = 0;
  int keep[DFX_MAX_DIM] = {0, 0, 0, 0};  // launch dim feeding store dim k
};

// Partitions are interned: two partitions are equal iff their handles are
// equal, an O(1) test (section 3.1, section 4.2's alias check).
struct PartRec {
  int kind = PK_NONE;
  int ndim = 0;
  int64_t tile[DFX_MAX_DIM] = {0, 0, 0, 0};
  int64_t off[DFX_MAX_DIM] = {0, 0, 0, 0};
  int proj = -1;
  int64_t img_src = -1;
  int img_part = -1;
};

struct ArgRec {
  int64_t store;
  int part;
  int priv;
};

struct TaskRec {
  uint32_t op = 0;
  int ndim = 0;
  int64_t launch[DFX_MAX_DIM] = {1, 1, 1, 1};
  std::vector<ArgRec> args;
  std::vector<double> imm;
  int64_t seq = 0;
};

enum OpKind { K_UNARY, K_BINARY, K_IMM, K_FILL, K_AXPY, K_RED, K_SPMV };

struct OpInfo {
  uint32_t op;
  const char* name;
  OpKind kind;
  int nargs;
  int vm;        // VmOp for elementwise kinds
};

// ---- plans ------------------------------------------------------------------
// A plan is built from a canonical window prefix: stores are referred to by
// their canonical index (order of first appearance in the window).
struct PStream {
  int cstore;
  int64_t off;          // element offset of the stream's (0, 0) element
  int64_t s_row, s_col;
};

struct PassPlan {
  int kind = 0;          // 0 elementwise/reduction, 1 SpMV, 2 single task
  int dtype = DFX_F64;
  int is1d = 1;
  int64_t rows = 1, cols = 1, n1d = 1;
  int64_t n_tiles = 0, strips = 1, tiles_per_wave = 1;
  int grid = 1;
  int nreg = 0;          // registers the allocation uses
  int tier = 0;          // kernel tier: 0 arithmetic, 1 transcendental, 2 with pow
  int unit_cols = 1;
  std::vector<PStream> ins;
  std::vector<PStream> outs;
  std::vector<int32_t> out_reg;
  std::vector<int> bc_cstore;
  std::vector<int32_t> bc_reg;
  std::vector<int> red_cstore;
  std::vector<int> red_init;
  int spmv_rowptr = -1, spmv_col = -1, spmv_val = -1, spmv_x = -1;
  // stencil staging: input streams that are shifted views of store st_cs
  int st_cs = -1;
  int64_t st_off0 = 0, st_srow = 0;   // window origin (element offset) and row stride
  std::vector<int8_t> st_on, st_dr, st_dc;
  // realigned inputs of the compiled kernel (run_pass): the strip shift
  // that aligns the outputs and, per input, its elements past alignment
  int realign_shift = 0;
  std::vector<int8_t> realign;
  std::vector<VmInstr> code;
  std::vector<double> imm;
  int64_t alg_bytes = 0;
  // per-plan device workspace: one reduction subtree sum per block
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // launch-shape tuner: tiles-per-wave candidates timed on the plan's first
  // executions (empty once the choice is fixed, or when tuning is off)
  std::vector<int64_t> tune_cand;   // candidate 0 is the default shape
  std::vector<float> tune_ms;       // fastest timing per candidate
  int tune_step = 0;          // execution count while tuning (0: the untimed warm-up)
  int tune_pending = -1;      // candidate whose events are in flight
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // compiled kernel of this pass (jit = 1 or 2): requested at the first
  // execution, shared by every plan with the same program and variant
  std::shared_ptr<JitEntry> jit;
  bool jit_checked = false;   // whether the pass runs compiled is decided
};

struct Plan {
  int prefix = 0;
  std::vector<int> temps;   // canonical indices of eliminated stores
  std::vector<PassPlan> passes;
  int64_t alg_bytes = 0;
};

struct Graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t launches = 0;
  int64_t alg_bytes = 0;
  int64_t compiled = 0;   // launches of compiled kernels in the graph
};

struct Ctx {
  dfx_config cfg{};
  hipStream_t stream = nullptr;
  bool analysis_only = false;
  bool over_limit = false;  // the last lowering failed on a kernel capacity limit
  std::string err;

  int64_t next_store = 1;
  std::unordered_map<int64_t, StoreRec> stores;
  std::vector<ProjRec> projs;
  std::unordered_map<std::string, int> proj_index;
  std::vector<PartRec> parts;
  std::unordered_map<std::string, int> part_index;

  std::deque<TaskRec> window;
  int window_cur = 1;       // tasks that fill the window (grows under auto_window)
  int64_t next_seq = 0;

  std::unordered_map<std::string, std::unique_ptr<Plan>> memo;
  std::vector<dfx_group_info> groups;

  bool capturing = false;
  int64_t capture_launches = 0, capture_bytes = 0, capture_compiled = 0;
  // Block sums of the last reducing pass not yet reduced (run_pass): the
  // next compiled one-block pass reduces them in its prologue instead of a
  // block-sum kernel launch; launched at the latest when the window ends.
  bool fin_pending = false;
  VmFinal fin{};
  int fin_f64 = 0;
  std::vector<int64_t> fin_stores;   // its 0-d result stores
  std::vector<std::unique_ptr<Graph>> graphs;

  dfx_stats stats{};
  void* server = nullptr;   // continuous-batching CG server, if started
  void* batch_rec = nullptr;  // recording into a batch (batch.cpp): passes are kept, not launched
  // allocation-free flush: the device's scratch array, the mode flag, and the
  // device frees deferred while the mode is on
  void* scratch = nullptr;
  bool no_alloc = false;
  std::vector<std::pair<void*, size_t>> deferred_free;
  // resident waves of the arithmetic kernels: [f64][stream bucket 2/4/6][rows 1]
  int n_cu = 0;
  int waves_cu[2][3][2] = {};
};

}  // namespace dfx
