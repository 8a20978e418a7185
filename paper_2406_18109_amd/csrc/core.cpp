// Host core of the fused task-stream executor: the IR tables of section 3,
// the task window and fusion analysis of section 4.2, temporary elimination
// and memoisation (sections 5.1 and 5.2), lowering of a fused group to op
// lists, and dispatch to the HIP kernels.
#include "core.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>

namespace dfx {

// ---------------------------------------------------------------------------
// Operation table: one entry per op (the per-op "generator" of section 6,
// here a descriptor the lowering reads).
static const OpInfo kOps[] = {
    {DFX_OP_NEG, "neg", K_UNARY, 2, VO_NEG},
    {DFX_OP_ABS, "abs", K_UNARY, 2, VO_ABS},
    {DFX_OP_SQRT, "sqrt", K_UNARY, 2, VO_SQRT},
    {DFX_OP_EXP, "exp", K_UNARY, 2, VO_EXP},
    {DFX_OP_LOG, "log", K_UNARY, 2, VO_LOG},
    {DFX_OP_ERF, "erf", K_UNARY, 2, VO_ERF},
    {DFX_OP_SQUARE, "square", K_UNARY, 2, VO_SQUARE},
    {DFX_OP_COPY, "copy", K_UNARY, 2, VO_MOV},
    {DFX_OP_ADD, "add", K_BINARY, 3, VO_ADD},
    {DFX_OP_SUB, "sub", K_BINARY, 3, VO_SUB},
    {DFX_OP_MUL, "mul", K_BINARY, 3, VO_MUL},
    {DFX_OP_DIV, "div", K_BINARY, 3, VO_DIV},
    {DFX_OP_POW, "pow", K_BINARY, 3, VO_POW},
    {DFX_OP_MAX, "max", K_BINARY, 3, VO_MAX},
    {DFX_OP_MIN, "min", K_BINARY, 3, VO_MIN},
    {DFX_OP_ADD_IMM, "add_imm", K_IMM, 2, VO_ADDI},
    {DFX_OP_SUB_IMM, "sub_imm", K_IMM, 2, VO_SUBI},
    {DFX_OP_RSUB_IMM, "rsub_imm", K_IMM, 2, VO_RSUBI},
    {DFX_OP_MUL_IMM, "mul_imm", K_IMM, 2, VO_MULI},
    {DFX_OP_DIV_IMM, "div_imm", K_IMM, 2, VO_DIVI},
    {DFX_OP_RDIV_IMM, "rdiv_imm", K_IMM, 2, VO_RDIVI},
    {DFX_OP_FILL, "fill", K_FILL, 1, VO_FILL},
    {DFX_OP_AXPY, "axpy", K_AXPY, 3, VO_ADD},
    {DFX_OP_SUM, "sum", K_RED, 2, VO_RED},
    {DFX_OP_SUMSQ, "sumsq", K_RED, 2, VO_REDPROD},
    {DFX_OP_DOT, "dot", K_RED, 3, VO_REDPROD},
    {DFX_OP_SPMV_CSR, "spmv_csr", K_SPMV, 5, 0},
};

static const OpInfo* op_info(uint32_t op) {
  for (const auto& o : kOps)
    if (o.op == op) return &o;
  return nullptr;
}

static bool is_float(int dt) { return dt == DFX_F32 || dt == DFX_F64; }
static size_t dtype_size(int dt) { return (dt == DFX_F32 || dt == DFX_I32) ? 4 : 8; }
static bool reads(int pr) { return pr == DFX_R || pr == DFX_RW; }
static bool writes(int pr) { return pr == DFX_W || pr == DFX_RW; }
static bool reduces(int pr) { return pr == DFX_RD; }
static bool heavy_op(int vm) { return vm >= VO_FIRST_HEAVY; }
static bool pow_op(int vm) { return vm == VO_POW; }

static int fail(Ctx& c, int code, const std::string& msg) {
  c.err = msg;
  return code;
}

// A fused group that one kernel cannot hold (streams, ops, reduction slots,
// live values): the dispatcher answers it with a shorter prefix.
static int fail_limit(Ctx& c, const std::string& msg) {
  c.over_limit = true;
  return fail(c, DFX_EUNSUPPORTED, msg);
}

#define HIPCHK(c, expr)                                                             \
  do {                                                                              \
    hipError_t e__ = (expr);                                                        \
    if (e__ != hipSuccess)                                                          \
      return fail((c), DFX_EHIP, std::string(#expr) + ": " + hipGetErrorString(e__)); \
  } while (0)

// ---------------------------------------------------------------------------
// Device memory

static void* dev_alloc(Ctx& c, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (c.cfg.alloc) return c.cfg.alloc(bytes, (void*)c.stream, c.cfg.alloc_user);
  void* p = nullptr;
  if (hipMallocAsync(&p, bytes, c.stream) != hipSuccess) return nullptr;
  return p;
}

// Reduce the block sums that wait for a consumer pass (run_pass) with the
// block-sum kernel.  Called at the end of every flush and before the memory
// that holds the block sums or their results is returned.
static int launch_pending_final(Ctx& c) {
  if (!c.fin_pending) return 0;
  c.fin_pending = false;
  return launch_vm_final(c.fin, c.fin_f64, c.stream);
}

static void dev_free(Ctx& c, void* p, size_t bytes) {
  if (!p) return;
  if (c.fin_pending) {
    // (partials[0] is the start of the pass's workspace)
    bool mine = p == c.fin.partials[0];
    for (int k = 0; k < c.fin.n_red; ++k) mine = mine || p == c.fin.result[k];
    if (mine) (void)launch_pending_final(c);   // (a launch error reappears at the next launch)
  }
  if (c.no_alloc) {   // returned at the next call that may free
    c.deferred_free.emplace_back(p, bytes);
    return;
  }
  if (c.cfg.dealloc) {
    c.cfg.dealloc(p, bytes, (void*)c.stream, c.cfg.alloc_user);
    return;
  }
  (void)hipFreeAsync(p, c.stream);
}

static void drain_deferred_frees(Ctx& c) {
  if (c.no_alloc) return;
  std::vector<std::pair<void*, size_t>> v;
  v.swap(c.deferred_free);
  for (auto& pb : v) dev_free(c, pb.first, pb.second);
}

static int ensure_alloc(Ctx& c, StoreRec& s) {
  if (s.ptr || s.bytes == 0) return DFX_OK;
  if (c.analysis_only) return DFX_OK;
  if (c.no_alloc)
    return fail(c, DFX_ESTATE, "store " + std::to_string(s.id) +
                                   " needs device memory in an allocation-free flush");
  if (c.capturing)
    return fail(c, DFX_ESTATE, "store " + std::to_string(s.id) +
                                   " needs memory while a graph is being recorded");
  s.ptr = dev_alloc(c, s.bytes);
  if (!s.ptr) return fail(c, DFX_ENOMEM, "device allocation of " + std::to_string(s.bytes) + " bytes failed");
  return DFX_OK;
}

static void maybe_free(Ctx& c, int64_t id) {
  auto it = c.stores.find(id);
  if (it == c.stores.end()) return;
  StoreRec& s = it->second;
  if (s.app_refs > 0 || s.pending > 0) return;
  if (s.ptr && !s.external) dev_free(c, s.ptr, s.bytes);
  c.stores.erase(it);
}

// ---------------------------------------------------------------------------
// Interning of projections and partitions (structural equality = handle equality)

// Interning keys list the fields explicitly (struct padding is not part of
// a partition's structure).
static void put_i64(std::string& k, int64_t v) { k.append((const char*)&v, 8); }

static std::string proj_key(const ProjRec& r) {
  std::string k;
  put_i64(k, r.nin);
  put_i64(k, r.nout);
  for (int i = 0; i < r.nout; ++i) put_i64(k, r.keep[i]);
  return k;
}

static std::string part_key(const PartRec& r) {
  std::string k;
  put_i64(k, r.kind);
  put_i64(k, r.ndim);
  for (int i = 0; i < r.ndim; ++i) { put_i64(k, r.tile[i]); put_i64(k, r.off[i]); }
  put_i64(k, r.proj);
  put_i64(k, r.img_src);
  put_i64(k, r.img_part);
  return k;
}

static int intern_proj(Ctx& c, const ProjRec& r) {
  std::string k = proj_key(r);
  auto it = c.proj_index.find(k);
  if (it != c.proj_index.end()) return it->second;
  int id = (int)c.projs.size();
  c.projs.push_back(r);
  c.proj_index.emplace(k, id);
  return id;
}

static int intern_part(Ctx& c, const PartRec& r) {
  std::string k = part_key(r);
  auto it = c.part_index.find(k);
  if (it != c.part_index.end()) return it->second;
  int id = (int)c.parts.size();
  c.parts.push_back(r);
  c.part_index.emplace(k, id);
  return id;
}

// ---------------------------------------------------------------------------
// Validation of a submitted task

static bool same_domain(const TaskRec& a, const TaskRec& b) {
  if (a.ndim != b.ndim) return false;
  for (int i = 0; i < a.ndim; ++i)
    if (a.launch[i] != b.launch[i]) return false;
  return true;
}

// Iteration space of a task: launch domain times the element shape of one
// point (index task), or the shape of its array arguments (single task).
struct Space {
  int rank = 1;
  int64_t d[DFX_MAX_DIM] = {1, 1, 1, 1};
};

static bool space_eq(const Space& a, const Space& b) {
  if (a.rank != b.rank) return false;
  for (int i = 0; i < a.rank; ++i)
    if (a.d[i] != b.d[i]) return false;
  return true;
}

struct TaskShape {
  Space space;
  int dtype = DFX_F64;
  int64_t elem[DFX_MAX_DIM] = {1, 1, 1, 1};
};

static int task_shape(Ctx& c, const TaskRec& t, TaskShape& out) {
  const OpInfo* oi = op_info(t.op);
  int dt = -1;
  for (size_t i = 0; i < t.args.size(); ++i) {
    const StoreRec& s = c.stores.at(t.args[i].store);
    if (oi->kind == K_SPMV && (i == 0 || i == 1)) continue;
    if (dt < 0) dt = s.dtype;
  }
  out.dtype = dt < 0 ? DFX_F64 : dt;
  if (oi->kind == K_SPMV) {
    const PartRec& py = c.parts[t.args[4].part];
    const StoreRec& y = c.stores.at(t.args[4].store);
    out.space.rank = 1;
    if (t.ndim == 0) out.space.d[0] = y.shape[0];
    else out.space.d[0] = py.tile[0] * t.launch[0];
    out.elem[0] = t.ndim == 0 ? y.shape[0] : py.tile[0];
    return DFX_OK;
  }
  if (t.ndim == 0) {
    // single task: array arguments through None, all of one shape
    int rank = 0;
    int64_t shp[DFX_MAX_DIM] = {1, 1, 1, 1};
    for (const auto& a : t.args) {
      const StoreRec& s = c.stores.at(a.store);
      if (s.ndim == 0) continue;
      if (rank == 0) {
        rank = s.ndim;
        for (int k = 0; k < rank; ++k) shp[k] = s.shape[k];
      } else {
        if (s.ndim != rank) return fail(c, DFX_EINVAL, "single task arrays differ in rank");
        for (int k = 0; k < rank; ++k)
          if (s.shape[k] != shp[k]) return fail(c, DFX_EINVAL, "single task arrays differ in shape");
      }
    }
    if (rank == 0) {
      out.space.rank = 1;
      out.space.d[0] = 1;
    } else {
      out.space.rank = rank;
      for (int k = 0; k < rank; ++k) out.space.d[k] = shp[k];
    }
    for (int k = 0; k < rank; ++k) out.elem[k] = shp[k];
    return DFX_OK;
  }
  bool have = false;
  for (const auto& a : t.args) {
    const PartRec& p = c.parts[a.part];
    if (p.kind != PK_TILING) continue;
    const ProjRec& pj = c.projs[p.proj];
    if (pj.nout == t.ndim) {
      bool ident = true;
      for (int k = 0; k < pj.nout; ++k) ident = ident && pj.keep[k] == k;
      if (ident) {
        for (int k = 0; k < t.ndim; ++k) out.elem[k] = p.tile[k];
        have = true;
        break;
      }
    }
  }
  if (!have) return fail(c, DFX_EINVAL, "index task needs an argument tiled with the identity projection");
  out.space.rank = t.ndim;
  for (int k = 0; k < t.ndim; ++k) out.space.d[k] = out.elem[k] * t.launch[k];
  return DFX_OK;
}

static int validate(Ctx& c, const TaskRec& t) {
  const OpInfo* oi = op_info(t.op);
  if (!oi) return fail(c, DFX_EINVAL, "unknown op " + std::to_string(t.op));
  if ((int)t.args.size() != oi->nargs)
    return fail(c, DFX_EINVAL, std::string(oi->name) + " takes " + std::to_string(oi->nargs) + " arguments");
  if (t.ndim < 0 || t.ndim > DFX_MAX_DIM) return fail(c, DFX_EINVAL, "launch rank out of range");
  int64_t volume = 1;
  for (int i = 0; i < t.ndim; ++i) {
    if (t.launch[i] < 1) return fail(c, DFX_EINVAL, "launch extents must be >= 1");
    volume *= t.launch[i];
  }
  for (const auto& a : t.args) {
    if (!c.stores.count(a.store)) return fail(c, DFX_ENOTFOUND, "unknown store " + std::to_string(a.store));
    if (a.part < 0 || a.part >= (int)c.parts.size()) return fail(c, DFX_ENOTFOUND, "unknown partition");
    if (a.priv < DFX_R || a.priv > DFX_RD) return fail(c, DFX_EINVAL, "bad privilege");
    if (c.stores.at(a.store).app_refs <= 0)
      return fail(c, DFX_EINVAL, "store " + std::to_string(a.store) + " was released");
  }
  // privileges by role
  auto need = [&](int i, bool in, bool out_, bool red) -> int {
    int pr = t.args[i].priv;
    if (red) return pr == DFX_RD ? DFX_OK : fail(c, DFX_EINVAL, std::string(oi->name) + ": result needs Rd");
    if (in && !out_ && !reads(pr)) return fail(c, DFX_EINVAL, std::string(oi->name) + ": argument " + std::to_string(i) + " needs R");
    if (out_ && !in && !writes(pr)) return fail(c, DFX_EINVAL, std::string(oi->name) + ": argument " + std::to_string(i) + " needs W");
    if (out_ && in && pr != DFX_RW) return fail(c, DFX_EINVAL, std::string(oi->name) + ": argument " + std::to_string(i) + " needs RW");
    return DFX_OK;
  };
  int rc = DFX_OK;
  const int n = (int)t.args.size();
  switch (oi->kind) {
    case K_UNARY: case K_IMM: rc = need(0, true, false, false); if (!rc) rc = need(1, false, true, false); break;
    case K_BINARY: rc = need(0, true, false, false); if (!rc) rc = need(1, true, false, false); if (!rc) rc = need(2, false, true, false); break;
    case K_FILL: rc = need(0, false, true, false); break;
    case K_AXPY: rc = need(0, true, false, false); if (!rc) rc = need(1, true, false, false); if (!rc) rc = need(2, true, true, false); break;
    case K_RED: for (int i = 0; i < n - 1 && !rc; ++i) rc = need(i, true, false, false); if (!rc) rc = need(n - 1, false, false, true); break;
    case K_SPMV: for (int i = 0; i < 4 && !rc; ++i) rc = need(i, true, false, false); if (!rc) rc = need(4, false, true, false); break;
  }
  if (rc) return rc;
  if ((oi->kind == K_IMM || oi->kind == K_FILL) && t.imm.empty())
    return fail(c, DFX_EINVAL, std::string(oi->name) + " needs an immediate");
  // dtypes
  int fdt = -1;
  for (int i = 0; i < n; ++i) {
    const StoreRec& s = c.stores.at(t.args[i].store);
    if (oi->kind == K_SPMV && i < 2) {
      if (s.dtype != DFX_I32) return fail(c, DFX_EINVAL, "spmv_csr: rowptr and col must be I32");
      continue;
    }
    if (!is_float(s.dtype)) return fail(c, DFX_EINVAL, std::string(oi->name) + ": arguments must be F32 or F64");
    if (fdt < 0) fdt = s.dtype;
    else if (s.dtype != fdt) return fail(c, DFX_EINVAL, std::string(oi->name) + ": mixed floating dtypes");
  }
  // partitions: kinds, ranks, bounds, legality
  for (int i = 0; i < n; ++i) {
    const ArgRec& a = t.args[i];
    const StoreRec& s = c.stores.at(a.store);
    const PartRec& p = c.parts[a.part];
    const bool spmv_mat = oi->kind == K_SPMV && i < 3;
    const bool spmv_x = oi->kind == K_SPMV && i == 3;
    if (p.kind == PK_IMAGE) {
      if (!spmv_x) return fail(c, DFX_EINVAL, "Image partitions are only read as the gathered SpMV operand");
      continue;
    }
    if (t.ndim == 0 && p.kind != PK_NONE) return fail(c, DFX_EINVAL, "single tasks take None partitions");
    if (p.kind == PK_NONE) {
      if (t.ndim > 0 && s.ndim == 0 && writes(a.priv))
        return fail(c, DFX_EINVAL, "index tasks reduce into 0-d stores; single tasks write them");
      if (writes(a.priv) && volume > 1)
        return fail(c, DFX_EINVAL, "writing through None from several points interferes");
      if (t.ndim > 0 && s.ndim != 0 && !spmv_mat && !spmv_x)
        return fail(c, DFX_EINVAL, "None partitions of index tasks are for 0-d broadcasts");
      if (reduces(a.priv) && s.ndim != 0) return fail(c, DFX_EINVAL, "reductions produce 0-d stores");
      continue;
    }
    // Tiling
    if (spmv_mat) return fail(c, DFX_EINVAL, "spmv_csr: matrix arrays are read through None");
    if (reduces(a.priv)) return fail(c, DFX_EINVAL, "reductions produce 0-d stores through None");
    if (p.ndim != s.ndim) return fail(c, DFX_EINVAL, "partition rank differs from store rank");
    const ProjRec& pj = c.projs[p.proj];
    if (pj.nin != t.ndim || pj.nout != s.ndim)
      return fail(c, DFX_EINVAL, "projection ranks do not match launch and store");
    for (int k = 0; k < s.ndim; ++k) {
      const int64_t ext = p.tile[k] * t.launch[pj.keep[k]];
      if (p.off[k] < 0 || p.off[k] + ext > s.shape[k])
        return fail(c, DFX_EINVAL, "tiles of store " + std::to_string(s.id) + " leave its bounds");
    }
    if (writes(a.priv)) {
      bool used[DFX_MAX_DIM] = {false, false, false, false};
      for (int k = 0; k < pj.nout; ++k) used[pj.keep[k]] = true;
      for (int d = 0; d < t.ndim; ++d)
        if (!used[d] && t.launch[d] > 1)
          return fail(c, DFX_EINVAL, "writing through an aliased (projected) tiling interferes");
    }
  }
  // a point task may not write a store it also reads through another partition
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (i == j || t.args[i].store != t.args[j].store) continue;
      if (writes(t.args[i].priv) && t.args[i].part != t.args[j].part)
        return fail(c, DFX_EINVAL, "task writes store " + std::to_string(t.args[i].store) +
                                       " and accesses it through another partition");
      if (reduces(t.args[i].priv) && !reduces(t.args[j].priv))
        return fail(c, DFX_EINVAL, "task reduces a store it also reads or writes");
    }
  TaskShape ts;
  rc = task_shape(c, t, ts);
  if (rc) return rc;
  // element shapes of all tiled arguments agree
  if (t.ndim > 0) {
    for (int i = 0; i < n; ++i) {
      const PartRec& p = c.parts[t.args[i].part];
      if (p.kind != PK_TILING) continue;
      const ProjRec& pj = c.projs[p.proj];
      for (int k = 0; k < pj.nout; ++k)
        if (p.tile[k] != ts.elem[pj.keep[k]])
          return fail(c, DFX_EINVAL, "tiles of the arguments do not share one element shape");
    }
  }
  if (oi->kind == K_SPMV) {
    const StoreRec& rp = c.stores.at(t.args[0].store);
    const StoreRec& col = c.stores.at(t.args[1].store);
    const StoreRec& val = c.stores.at(t.args[2].store);
    const StoreRec& y = c.stores.at(t.args[4].store);
    const StoreRec& x = c.stores.at(t.args[3].store);
    if (rp.ndim != 1 || col.ndim != 1 || val.ndim != 1 || x.ndim != 1 || y.ndim != 1)
      return fail(c, DFX_EINVAL, "spmv_csr: all arrays are 1-D");
    if (rp.shape[0] != y.shape[0] + 1) return fail(c, DFX_EINVAL, "spmv_csr: rowptr needs rows+1 entries");
    if (col.shape[0] != val.shape[0]) return fail(c, DFX_EINVAL, "spmv_csr: col and val differ in length");
    if (t.ndim > 1) return fail(c, DFX_EINVAL, "spmv_csr: 1-D launch domain");
    const PartRec& py = c.parts[t.args[4].part];
    if (t.ndim == 1 && py.kind != PK_TILING) return fail(c, DFX_EINVAL, "spmv_csr: y is tiled by rows");
    if (t.ndim == 1 && py.off[0] != 0) return fail(c, DFX_EINVAL, "spmv_csr: y's tiling starts at row 0");
  }
  return DFX_OK;
}

// ---------------------------------------------------------------------------
// Fusion analysis over the window (section 4.2)

// Longest prefix satisfying launch-domain equivalence, true dependence, anti
// dependence and reduction, by a forward pass that records, per store, the
// partitions it has been read and written through and whether it has been
// reduced.  Each new task is checked against the effects of all earlier
// tasks of the prefix; the constraints quantify over pairs, so the set of
// fusible prefixes is closed under taking prefixes and the first violation
// ends the longest one.
struct Effects {
  std::vector<int> read_parts, write_parts;
  bool reduced = false;
};

static int longest_prefix(Ctx& c) {
  const auto& W = c.window;
  if (W.empty()) return 0;
  std::unordered_map<int64_t, Effects> eff;
  int f = 0;
  for (size_t j = 0; j < W.size(); ++j) {
    const TaskRec& t = W[j];
    bool ok = same_domain(t, W[0]);
    for (const auto& a : t.args) {
      if (!ok) break;
      auto it = eff.find(a.store);
      if (it == eff.end()) continue;
      const Effects& e = it->second;
      if (reads(a.priv) || writes(a.priv)) {
        for (int p : e.write_parts) if (p != a.part) ok = false;   // true dependence
        if (e.reduced) ok = false;                                 // reduction
      }
      if (writes(a.priv))
        for (int p : e.read_parts) if (p != a.part) ok = false;    // anti dependence
      if (reduces(a.priv) && (!e.read_parts.empty() || !e.write_parts.empty()))
        ok = false;                                                // reduction
    }
    if (!ok) break;
    for (const auto& a : t.args) {
      Effects& e = eff[a.store];
      if (reads(a.priv) && std::find(e.read_parts.begin(), e.read_parts.end(), a.part) == e.read_parts.end())
        e.read_parts.push_back(a.part);
      if (writes(a.priv) && std::find(e.write_parts.begin(), e.write_parts.end(), a.part) == e.write_parts.end())
        e.write_parts.push_back(a.part);
      if (reduces(a.priv)) e.reduced = true;
    }
    f = (int)j + 1;
  }
  return f;
}

// covers(S, P): the sub-stores of P over the launch domain hold all of S.
static bool covers(Ctx& c, const StoreRec& s, int part, const TaskRec& t) {
  const PartRec& p = c.parts[part];
  if (p.kind == PK_NONE) return true;
  if (p.kind != PK_TILING) return false;
  const ProjRec& pj = c.projs[p.proj];
  for (int k = 0; k < s.ndim; ++k) {
    if (p.off[k] > 0) return false;
    if (p.off[k] + p.tile[k] * t.launch[pj.keep[k]] < s.shape[k]) return false;
  }
  return true;
}

// Temporary stores of the fusion of window[0, f) (section 5.1):
//  (1) every read through P in the prefix follows, in an earlier prefix
//      task, a write through the same P that covers the store;
//  (2) no task after the prefix reads or reduces it;
//  (3) no application reference remains.
static std::set<int64_t> temporaries(Ctx& c, int f) {
  const auto& W = c.window;
  std::map<int64_t, std::vector<int>> covered;  // store -> covering write partitions so far
  std::set<int64_t> bad, seen;
  std::vector<int64_t> order;
  for (int j = 0; j < f; ++j) {
    const TaskRec& t = W[j];
    for (const auto& a : t.args) {
      if (!seen.count(a.store)) { seen.insert(a.store); order.push_back(a.store); }
      if (reads(a.priv)) {
        const auto& cv = covered[a.store];
        if (std::find(cv.begin(), cv.end(), a.part) == cv.end()) bad.insert(a.store);
      }
    }
    for (const auto& a : t.args)
      if (writes(a.priv) && covers(c, c.stores.at(a.store), a.part, t)) covered[a.store].push_back(a.part);
  }
  std::set<int64_t> later;
  for (size_t k = f; k < W.size(); ++k)
    for (const auto& a : W[k].args)
      if (reads(a.priv) || reduces(a.priv)) later.insert(a.store);
  std::set<int64_t> temps;
  for (int64_t s : order) {
    if (bad.count(s) || later.count(s)) continue;
    const StoreRec& r = c.stores.at(s);
    if (r.app_refs > 0 || r.external) continue;
    temps.insert(s);
  }
  return temps;
}

// Canonical form of the window (section 5.2): stores renamed by order of
// first appearance, so isomorphic windows share one key.  The key also holds
// what the plan depends on: ops, launch domains, immediates, partitions,
// privileges, and each store's rank, shape, dtype and live bit.
static void put(std::string& k, const void* p, size_t n) { k.append((const char*)p, n); }

// A partition by its structure (kind, tiles, offsets, projection), so that a
// key means the same in every context; interned handles make this
// equivalent to handle equality inside one context.
static void put_part(std::string& k, const Ctx& c, int part) {
  const PartRec& p = c.parts[part];
  put(k, &p.kind, 4);
  put(k, &p.ndim, 4);
  put(k, p.tile, 8 * p.ndim);
  put(k, p.off, 8 * p.ndim);
  int32_t np = p.proj >= 0 ? 1 : 0;
  put(k, &np, 4);
  if (np) {
    const ProjRec& r = c.projs[p.proj];
    put(k, &r.nin, 4);
    put(k, &r.nout, 4);
    put(k, r.keep, 4 * r.nout);
  }
}

static std::string canonical_key(Ctx& c, std::vector<int64_t>& order) {
  std::unordered_map<int64_t, int> idx;
  order.clear();
  auto cid = [&](int64_t s) {
    auto it = idx.find(s);
    if (it != idx.end()) return it->second;
    int i = (int)order.size();
    idx.emplace(s, i);
    order.push_back(s);
    return i;
  };
  std::string k;
  k.reserve(1024);
  int32_t n = (int32_t)c.window.size();
  put(k, &n, 4);
  for (const auto& t : c.window) {
    put(k, &t.op, 4);
    put(k, &t.ndim, 4);
    put(k, t.launch, 8 * t.ndim);
    int32_t ni = (int32_t)t.imm.size(), na = (int32_t)t.args.size();
    put(k, &ni, 4);
    if (ni) put(k, t.imm.data(), 8 * ni);
    put(k, &na, 4);
    for (const auto& a : t.args) {
      int32_t s = cid(a.store);
      put(k, &s, 4);
      const PartRec& p = c.parts[a.part];
      if (p.kind == PK_IMAGE) {
        int32_t tag = -2 - cid(p.img_src);
        put(k, &tag, 4);
        put_part(k, c, p.img_part);
      } else {
        put_part(k, c, a.part);
      }
      put(k, &a.priv, 4);
    }
  }
  for (int64_t s : order) {
    const StoreRec& r = c.stores.at(s);
    put(k, &r.ndim, 4);
    put(k, r.shape, 8 * r.ndim);
    put(k, &r.dtype, 4);
    int32_t live = (r.app_refs > 0 || r.external) ? 1 : 0;
    put(k, &live, 4);
  }
  return k;
}

// ---------------------------------------------------------------------------
// Lowering a fused group to passes and op lists

struct Box { int64_t lo[2], hi[2]; };

static int64_t union_volume(const std::vector<Box>& bs) {
  if (bs.empty()) return 0;
  std::vector<int64_t> xs, ys;
  for (const auto& b : bs) { xs.push_back(b.lo[0]); xs.push_back(b.hi[0]); ys.push_back(b.lo[1]); ys.push_back(b.hi[1]); }
  std::sort(xs.begin(), xs.end()); xs.erase(std::unique(xs.begin(), xs.end()), xs.end());
  std::sort(ys.begin(), ys.end()); ys.erase(std::unique(ys.begin(), ys.end()), ys.end());
  int64_t v = 0;
  for (size_t i = 0; i + 1 < xs.size(); ++i)
    for (size_t j = 0; j + 1 < ys.size(); ++j) {
      bool in = false;
      for (const auto& b : bs)
        if (b.lo[0] <= xs[i] && xs[i + 1] <= b.hi[0] && b.lo[1] <= ys[j] && ys[j + 1] <= b.hi[1]) { in = true; break; }
      if (in) v += (xs[i + 1] - xs[i]) * (ys[j + 1] - ys[j]);
    }
  return v;
}

struct SVal {
  int kind;           // 0 input stream, 1 broadcast, 2 computed, 3 SpMV row result
  int idx;            // stream / broadcast index, or defining instruction
  int last_use = -1;
  bool stored = false;
  int reg = -1;
  bool wb = false;
};

struct SInstr {
  uint8_t op;
  int a = -1, b = -1, dst = -1;   // value ids
  int imm = 0, slot = 0;
  bool dead = false;
  bool operator==(const SInstr& o) const {
    return op == o.op && a == o.a && b == o.b && dst == o.dst && imm == o.imm && slot == o.slot;
  }
  bool operator!=(const SInstr& o) const { return !(*this == o); }
};

struct Lowering {
  Ctx& c;
  const std::vector<int64_t>& order;  // canonical index -> store id
  std::unordered_map<int64_t, int> cidx;
  std::set<int64_t> temps;
  Lowering(Ctx& c_, const std::vector<int64_t>& o) : c(c_), order(o) {
    for (size_t i = 0; i < o.size(); ++i) cidx[o[i]] = (int)i;
  }
};

// Stream (offset, row stride, column stride) of argument (s, part) in a pass
// over `sp`; 1-D spaces are cut into rows of TW elements.
static PStream make_stream(Ctx& c, const StoreRec& s, int part, const Space& sp, int tw, int cs) {
  PStream ps{cs, 0, 0, 0};
  int64_t st[DFX_MAX_DIM];
  int64_t acc = 1;
  for (int k = s.ndim - 1; k >= 0; --k) { st[k] = acc; acc *= s.shape[k]; }
  const PartRec& p = c.parts[part];
  if (s.ndim == 0) return ps;
  int keep[DFX_MAX_DIM];
  int64_t off[DFX_MAX_DIM] = {0, 0, 0, 0};
  if (p.kind == PK_TILING) {
    const ProjRec& pj = c.projs[p.proj];
    for (int k = 0; k < s.ndim; ++k) { keep[k] = pj.keep[k]; off[k] = p.off[k]; }
  } else {
    for (int k = 0; k < s.ndim; ++k) keep[k] = k + (sp.rank - s.ndim);
  }
  int64_t srow = 0, scol = 0;
  for (int k = 0; k < s.ndim; ++k) {
    ps.off += off[k] * st[k];
    if (sp.rank == 1) { if (keep[k] == 0) scol += st[k]; }
    else {
      if (keep[k] == 0) srow += st[k];
      else if (keep[k] == 1) scol += st[k];
    }
  }
  if (sp.rank == 1) { ps.s_row = scol * tw; ps.s_col = scol; }
  else { ps.s_row = srow; ps.s_col = scol; }
  return ps;
}

static Box stream_box(Ctx& c, const StoreRec& s, int part, const Space& sp) {
  Box b{{0, 0}, {1, 1}};
  const PartRec& p = c.parts[part];
  if (s.ndim == 0) return b;
  for (int k = 0; k < s.ndim && k < 2; ++k) {
    int L;
    int64_t off = 0;
    if (p.kind == PK_TILING) { L = c.projs[p.proj].keep[k]; off = p.off[k]; }
    else L = k + (sp.rank - s.ndim);
    const int kk = s.ndim == 1 ? 1 : k;   // 1-D stores occupy the second box axis
    b.lo[kk] = off;
    b.hi[kk] = off + sp.d[L];
  }
  return b;
}

// DFX_TRACE=1 prints one line per lowered pass to stderr, DFX_TRACE=2 also
// its instructions.
static int trace_level() {
  static const int lvl = [] {
    const char* e = std::getenv("DFX_TRACE");
    return e ? std::atoi(e) : 0;
  }();
  return lvl;
}


// Launch shape of a pass for `tpw` tiles per wave (a power of two, so that
// each block's tiles form an aligned subtree of the reduction tree): four
// waves per block, the grid a multiple of 8 (one share per XCD) when large.
static void set_shape(PassPlan& p, int64_t tpw) {
  p.tiles_per_wave = tpw;
  const int64_t waves = (p.n_tiles + tpw - 1) / tpw;
  int64_t grid = std::max<int64_t>(1, (waves + 3) / 4);
  if (grid > 8) grid = (grid + 7) / 8 * 8;
  p.grid = (int)grid;
}

// Reorder a pass's instructions so that a value is consumed right after it
// is produced whenever a consumer is ready: that consumer takes it from the
// accumulator (no register write-back for a single use, no operand fetch)
// and may merge with it into one dispatch.  Any topological order of the
// value graph computes the same bits (every op rounds on its own; each
// reduction has its own slot), so the choice is free; otherwise the
// original order is kept.
static void schedule_chain(std::vector<SInstr>& code, size_t n_vals) {
  const int n = (int)code.size();
  std::vector<int> prod(n_vals, -1);
  for (int i = 0; i < n; ++i)
    if (code[i].dst >= 0) prod[code[i].dst] = i;
  std::vector<char> done(n, 0);
  auto ready = [&](int i) {
    for (int v : {code[i].a, code[i].b})
      if (v >= 0 && prod[v] >= 0 && !done[prod[v]]) return false;
    return true;
  };
  std::vector<SInstr> out;
  out.reserve(n);
  int prev = -1;
  for (int k = 0; k < n; ++k) {
    int pick = -1;
    if (prev >= 0)
      for (int i = 0; i < n && pick < 0; ++i)
        if (!done[i] && (code[i].a == prev || code[i].b == prev) && ready(i)) pick = i;
    for (int i = 0; i < n && pick < 0; ++i)
      if (!done[i] && ready(i)) pick = i;
    done[pick] = 1;
    out.push_back(code[pick]);
    prev = code[pick].dst;
  }
  code.swap(out);
}

static int lower_pass(Ctx& c, Lowering& L, const std::vector<const TaskRec*>& tasks, const Space& sp,
                      int dtype, int kind, PassPlan& out) {
  const int tw = dtype == DFX_F64 ? Lanes<double>::TW : Lanes<float>::TW;
  const size_t es = dtype_size(dtype);
  out.kind = kind;
  out.dtype = dtype;
  out.is1d = sp.rank == 1;
  if (sp.rank == 1) {
    out.n1d = sp.d[0];
    out.rows = (sp.d[0] + tw - 1) / tw;
    out.cols = tw;
    out.strips = 1;
  } else {
    out.rows = sp.d[0];
    out.cols = sp.d[1];
    out.strips = (sp.d[1] + tw - 1) / tw;
    out.n1d = sp.d[0] * sp.d[1];
  }
  const int64_t tile_rows = (out.rows + RED_TH - 1) / RED_TH;
  out.n_tiles = tile_rows * out.strips;
  if (out.n_tiles > (int64_t)FINAL_CHUNK * FINAL_CHUNK)
    return fail(c, DFX_EUNSUPPORTED, "iteration space too large for the reduction tree");

  std::vector<SVal> vals;
  std::vector<SInstr> code;
  std::map<std::pair<int, int>, int> cur;       // (cstore, part) -> value holding its current contents
  std::map<std::pair<int, int>, int> in_index;  // (cstore, part) -> input stream index
  std::map<int, int> bc_index;                  // cstore -> broadcast index
  std::vector<std::pair<int, int>> written;     // (cstore, part) in first-write order
  std::vector<std::pair<int64_t, int>> in_args; // (store id, part) per input stream

  auto read_val = [&](const ArgRec& a) -> int {
    const int cs = L.cidx.at(a.store);
    auto key = std::make_pair(cs, a.part);
    auto it = cur.find(key);
    if (it != cur.end()) return it->second;
    const StoreRec& s = c.stores.at(a.store);
    if (kind != 2 && s.ndim == 0) {
      auto bi = bc_index.find(cs);
      if (bi != bc_index.end()) return bi->second;
      int k = (int)out.bc_cstore.size();
      out.bc_cstore.push_back(cs);
      vals.push_back({1, k});
      int v = (int)vals.size() - 1;
      bc_index[cs] = v;
      return v;
    }
    int k = (int)out.ins.size();
    out.ins.push_back(make_stream(c, s, a.part, sp, tw, cs));
    in_args.push_back({a.store, a.part});
    vals.push_back({0, k});
    int v = (int)vals.size() - 1;
    in_index[key] = k;
    cur[key] = v;
    return v;
  };
  auto write_val = [&](const ArgRec& a, int v) {
    const int cs = L.cidx.at(a.store);
    auto key = std::make_pair(cs, a.part);
    if (std::find(written.begin(), written.end(), key) == written.end()) written.push_back(key);
    cur[key] = v;
  };
  auto emit = [&](uint8_t op, int a, int b, int imm, int slot, bool has_dst) -> int {
    SInstr I;
    I.op = op; I.a = a; I.b = b; I.imm = imm; I.slot = slot;
    if (has_dst) {
      vals.push_back({2, (int)code.size()});
      I.dst = (int)vals.size() - 1;
    }
    code.push_back(I);
    return I.dst;
  };
  auto add_imm = [&](double v) -> int {
    for (size_t i = 0; i < out.imm.size(); ++i)
      if (std::memcmp(&out.imm[i], &v, 8) == 0) return (int)i;
    out.imm.push_back(v);
    return (int)out.imm.size() - 1;
  };

  for (const TaskRec* t : tasks) {
    const OpInfo* oi = op_info(t->op);
    const auto& A = t->args;
    switch (oi->kind) {
      case K_UNARY: {
        int x = read_val(A[0]);
        int z = oi->vm == VO_MOV ? x : emit((uint8_t)oi->vm, x, x, 0, 0, true);
        write_val(A[1], z);
      } break;
      case K_BINARY: {
        int x = read_val(A[0]), y = read_val(A[1]);
        write_val(A[2], emit((uint8_t)oi->vm, x, y, 0, 0, true));
      } break;
      case K_IMM: {
        int x = read_val(A[0]);
        write_val(A[1], emit((uint8_t)oi->vm, x, x, add_imm(t->imm[0]), 0, true));
      } break;
      case K_FILL: {
        write_val(A[0], emit(VO_FILL, -1, -1, add_imm(t->imm[0]), 0, true));
      } break;
      case K_AXPY: {
        int al = read_val(A[0]), x = read_val(A[1]), y = read_val(A[2]);
        int p = emit(VO_MUL, al, x, 0, 0, true);
        const bool minus = !t->imm.empty() && t->imm[0] < 0;
        write_val(A[2], emit(minus ? VO_SUB : VO_ADD, y, p, 0, 0, true));
      } break;
      case K_RED: {
        const int slot = (int)out.red_cstore.size();
        if (slot >= VM_MAXRED) return fail_limit(c, "too many reductions in one pass");
        const int cs = L.cidx.at(A.back().store);
        out.red_cstore.push_back(cs);
        out.red_init.push_back(!t->imm.empty() && t->imm[0] != 0);
        int x = read_val(A[0]);
        int y = t->op == DFX_OP_DOT ? read_val(A[1]) : x;
        emit((uint8_t)oi->vm, x, y, 0, slot, false);
      } break;
      case K_SPMV: {
        out.spmv_rowptr = L.cidx.at(A[0].store);
        out.spmv_col = L.cidx.at(A[1].store);
        out.spmv_val = L.cidx.at(A[2].store);
        out.spmv_x = L.cidx.at(A[3].store);
        vals.push_back({3, 0});
        write_val(A[4], (int)vals.size() - 1);
      } break;
    }
  }
  // outputs: final value of every written, non-temporary (store, partition)
  std::vector<std::pair<int, int>> outs;  // (value, written index)
  for (size_t i = 0; i < written.size(); ++i) {
    const int64_t sid = L.order[written[i].first];
    if (L.temps.count(sid)) continue;
    outs.push_back({cur[written[i]], (int)i});
    vals[cur[written[i]]].stored = true;
  }
  // dead code: keep instructions whose values reach a store or a reduction
  std::vector<bool> live(vals.size(), false);
  for (auto& o : outs) live[o.first] = true;
  for (int i = (int)code.size() - 1; i >= 0; --i) {
    SInstr& I = code[i];
    bool need = (I.op == VO_RED || I.op == VO_REDPROD) || (I.dst >= 0 && live[I.dst]);
    if (!need) { I.dead = true; continue; }
    if (I.a >= 0) live[I.a] = true;
    if (I.b >= 0) live[I.b] = true;
  }
  std::vector<SInstr> kept;
  for (auto& I : code)
    if (!I.dead) kept.push_back(I);
  code.swap(kept);
  const std::vector<SInstr> program_order = code;
  schedule_chain(code, vals.size());
  // definitions, operand uses, last uses and write-backs of the current order
  const int INF = 1 << 30;
  auto analyse = [&]() {
    for (size_t i = 0; i < code.size(); ++i)
      if (code[i].dst >= 0) vals[code[i].dst].idx = (int)i;
    std::vector<std::vector<int>> uses(vals.size());
    for (size_t i = 0; i < code.size(); ++i) {
      if (code[i].a >= 0) uses[code[i].a].push_back((int)i);
      if (code[i].b >= 0 && code[i].b != code[i].a) uses[code[i].b].push_back((int)i);
    }
    for (size_t v = 0; v < vals.size(); ++v) {
      int lu = -1;
      for (int u : uses[v]) lu = std::max(lu, u);
      if (vals[v].stored) lu = INF;
      vals[v].last_use = lu;
      if (vals[v].kind == 2) {
        const int d = vals[v].idx;
        bool only_next = !vals[v].stored && !uses[v].empty();
        for (int u : uses[v]) only_next = only_next && u == d + 1;
        vals[v].wb = !only_next;
      }
    }
  };
  analyse();
  // unused inputs are still loaded (their stream is bound); unused
  // broadcasts are dropped from the register file but keep their slot
  if (out.ins.size() > (size_t)VM_MAXIN || out.bc_cstore.size() > (size_t)VM_MAXBC ||
      code.size() > (size_t)VM_MAXCODE ||
      outs.size() > (size_t)VM_MAXOUT)
    return fail_limit(c, "fused pass exceeds the kernel's stream/op limits");

  bool heavy = false, has_pow = false;
  for (auto& I : code) { heavy = heavy || heavy_op(I.op); has_pow = has_pow || pow_op(I.op); }
  // register allocation: inputs fixed at 0..n_in-1, SpMV result at NR-1,
  // broadcasts in permanent registers above the stream bucket, computed
  // values by linear scan (an operand's register is free for the
  // instruction's result)
  int tier = 0;
  auto allocate = [&](int NR, int nload) -> bool {
    for (auto& v : vals) v.reg = -1;
    std::vector<int> busy_until(NR, -2);  // last instruction reading the register; INF permanent
    const int nin = (int)out.ins.size();
    if (nin > NR || nload > NR) return false;
    const bool has_spmv = kind == 1;
    for (size_t v = 0; v < vals.size(); ++v) {
      if (vals[v].kind == 0) {
        vals[v].reg = vals[v].idx;
        busy_until[vals[v].idx] = std::max(vals[v].last_use, -1);
      } else if (vals[v].kind == 3) {
        if (NR - 1 < nload) return false;
        vals[v].reg = NR - 1;
        busy_until[NR - 1] = std::max(vals[v].last_use, -1);
      }
    }
    if (has_spmv && busy_until[NR - 1] < -1) busy_until[NR - 1] = -1;
    // the kernel loads every slot of the stream bucket each step, so
    // permanent registers start above the bucket
    for (size_t v = 0; v < vals.size(); ++v) {
      if (vals[v].kind != 1) continue;
      int r = -1;
      for (int q = nload; q < NR - (has_spmv ? 1 : 0); ++q)
        if (busy_until[q] == -2) { r = q; break; }
      if (r < 0) return false;
      vals[v].reg = r;
      busy_until[r] = INF;
    }
    for (size_t i = 0; i < code.size(); ++i) {
      const int d = code[i].dst;
      if (d < 0 || !vals[d].wb) continue;
      int r = -1;
      for (int q = 0; q < NR; ++q)
        if (busy_until[q] != INF && busy_until[q] <= (int)i) { r = q; break; }
      if (r < 0) return false;
      vals[d].reg = r;
      busy_until[r] = vals[d].last_use;
    }
    return true;
  };
  const int nin = (int)out.ins.size();
  // keep the chained order only if it fits the register file the program
  // order fits
  if (!has_pow && nin <= 6 && code != program_order) {
    const int b8 = stream_bucket(nin, heavy ? TIER_TRANS8 : TIER_ARITH);
    if (!allocate(VM_NREG_LIGHT, b8)) {
      const std::vector<SInstr> chained = code;
      code = program_order;
      analyse();
      if (!allocate(VM_NREG_LIGHT, b8)) {
        code = chained;
        analyse();
      }
    }
  }
  bool ok = false;
  if (!has_pow && nin <= 6) {
    tier = heavy ? TIER_TRANS8 : TIER_ARITH;
    ok = allocate(VM_NREG_LIGHT, stream_bucket(nin, tier));
    if (!ok) { tier = TIER_TRANS16; ok = allocate(VM_NREG, stream_bucket(nin, tier)); }
  }
  if (!ok) { tier = TIER_POW; ok = allocate(VM_NREG, stream_bucket(nin, tier)); }
  if (!ok) return fail_limit(c, "fused pass needs more than 16 live values");
  out.tier = tier;
  out.nreg = 0;
  for (auto& v : vals) out.nreg = std::max(out.nreg, v.reg + 1);
  // emit kernel instructions with operand forwarding
  struct EI {
    unsigned op, flags, d, a, b, slot;
    double imm;
    bool uses_imm;
    unsigned post = 0, c = 0;
  };
  std::vector<EI> em;
  for (size_t i = 0; i < code.size(); ++i) {
    SInstr I = code[i];
    unsigned flags = 0, ra = 0, rb = 0, rd = 0;
    const int prev = i > 0 ? code[i - 1].dst : -1;
    const bool binary = I.op == VO_ADD || I.op == VO_SUB || I.op == VO_MUL || I.op == VO_DIV ||
                        I.op == VO_MAX || I.op == VO_MIN || I.op == VO_REDPROD || I.op == VO_POW;
    // IEEE addition and multiplication are commutative bit for bit: put the
    // forwarded operand first so it stays in the accumulator.  A forwarded
    // right operand of a subtraction or division stays in the accumulator
    // through the reversed op (b - a and b / a are the same IEEE operations).
    if (binary && (I.op == VO_ADD || I.op == VO_MUL || I.op == VO_REDPROD) && I.b == prev && I.a != prev)
      std::swap(I.a, I.b);
    else if ((I.op == VO_SUB || I.op == VO_DIV) && I.b == prev && I.a != prev) {
      I.op = I.op == VO_SUB ? VO_RSUB : VO_RDIV;
      std::swap(I.a, I.b);
    }
    if (I.a >= 0) {
      if (I.a == prev) flags |= VF_A_ACC;
      else { ra = (unsigned)vals[I.a].reg; flags |= VF_A_REG; }
    }
    if ((binary || I.op == VO_RSUB || I.op == VO_RDIV) && I.b >= 0) {
      if (I.b == prev) flags |= VF_B_ACC;
      else { rb = (unsigned)vals[I.b].reg; flags |= VF_B_REG; }
    }
    if (I.dst >= 0 && vals[I.dst].wb) {
      flags |= VF_WB;
      rd = (unsigned)vals[I.dst].reg;
    }
    const bool uses_imm = I.op == VO_ADDI || I.op == VO_SUBI || I.op == VO_RSUBI || I.op == VO_MULI ||
                          I.op == VO_DIVI || I.op == VO_RDIVI || I.op == VO_FILL;
    const double immv = I.imm >= 0 && I.imm < (int)out.imm.size() ? out.imm[I.imm] : 0.0;
    em.push_back(EI{I.op, flags, rd, ra, rb, (unsigned)I.slot, immv, uses_imm});
  }
  // two-op superinstructions: an op whose result only feeds the next op as
  // its operand a carries that op as its post op (operand b of a binary post
  // op from register c), when at most one of the two uses the immediate
  auto post_ok = [](unsigned op) {
    return op == VO_NEG || op == VO_SQUARE || op == VO_ADDI || op == VO_SUBI || op == VO_RSUBI ||
           op == VO_MULI || op == VO_ADD || op == VO_SUB || op == VO_MUL || op == VO_RSUB;
  };
  std::vector<EI> merged;
  for (size_t i = 0; i < em.size(); ++i) {
    if (i + 1 < em.size()) {
      const EI& f = em[i];
      const EI& s2 = em[i + 1];
      const bool first_ok = f.op != VO_RED && f.op != VO_REDPROD && !(f.flags & VF_WB);
      const bool second_ok = post_ok(s2.op) && (s2.flags & VF_A_ACC) && !(s2.flags & (VF_A_REG | VF_B_ACC));
      if (first_ok && second_ok && !(f.uses_imm && s2.uses_imm)) {
        EI m = f;
        m.post = s2.op + 1;
        m.flags = (f.flags & (VF_A_ACC | VF_A_REG | VF_B_ACC | VF_B_REG)) | (s2.flags & VF_WB) |
                  ((s2.flags & VF_B_REG) ? VF_C_REG : 0);
        m.d = s2.d;
        m.c = s2.b;
        if (s2.uses_imm) { m.imm = s2.imm; m.uses_imm = true; }
        merged.push_back(m);
        ++i;
        continue;
      }
    }
    merged.push_back(em[i]);
  }
  for (const EI& e : merged)
    out.code.push_back(vm_instr(e.op, e.d, e.a, e.b, e.flags, e.slot, e.imm, dtype == DFX_F64, e.post, e.c));
  for (auto& o : outs) {
    const auto key = written[o.second];
    const StoreRec& s = c.stores.at(L.order[key.first]);
    out.outs.push_back(make_stream(c, s, key.second, sp, tw, key.first));
    out.out_reg.push_back(vals[o.first].reg);
  }
  for (size_t v = 0; v < vals.size(); ++v)
    if (vals[v].kind == 1) out.bc_reg.push_back(vals[v].reg);
  out.unit_cols = 1;
  for (auto& s : out.ins) out.unit_cols &= s.s_col == 1;
  for (auto& s : out.outs) out.unit_cols &= s.s_col == 1;
  // Stencil staging (arithmetic 2-D passes): three or more input streams
  // that are views of one store with the same row stride, unit column
  // stride and origins within a 3 x 3 window are read through LDS.
  out.st_cs = -1;
  out.st_on.assign(out.ins.size(), 0);
  out.st_dr.assign(out.ins.size(), 0);
  out.st_dc.assign(out.ins.size(), 0);
  if (kind == 0 && sp.rank == 2 && tier == TIER_ARITH) {
    std::map<int, std::vector<int>> by_store;
    for (size_t a = 0; a < out.ins.size(); ++a) by_store[out.ins[a].cstore].push_back((int)a);
    for (auto& kv : by_store) {
      const std::vector<int>& m = kv.second;
      if (m.size() < 3 || m.size() <= (size_t)std::count(out.st_on.begin(), out.st_on.end(), 1)) continue;
      const int64_t srow = out.ins[m[0]].s_row;
      bool ok = srow > 0;
      int64_t r0 = INT64_MAX, c0 = INT64_MAX;
      for (int a : m) {
        const PStream& q = out.ins[a];
        ok = ok && q.s_col == 1 && q.s_row == srow && q.off >= 0;
        if (!ok) break;
        r0 = std::min(r0, q.off / srow);
        c0 = std::min(c0, q.off % srow);
      }
      for (int a : m) {
        if (!ok) break;
        const int64_t dr = out.ins[a].off / srow - r0, dc = out.ins[a].off % srow - c0;
        ok = dr <= 2 && dc <= 2;
      }
      if (!ok) continue;
      out.st_cs = kv.first;
      out.st_off0 = r0 * srow + c0;
      out.st_srow = srow;
      std::fill(out.st_on.begin(), out.st_on.end(), 0);
      for (int a : m) {
        out.st_on[a] = 1;
        out.st_dr[a] = (int8_t)(out.ins[a].off / srow - r0);
        out.st_dc[a] = (int8_t)(out.ins[a].off % srow - c0);
      }
    }
  }
  // launch shape: contiguous tile chunks per wave
  // (a power of two, so that each block's tiles form an aligned subtree of
  // the reduction tree)
  // One tile per wave up to 32768 tiles: waves that each stream a long
  // contiguous run spread the resident waves' accesses over more of HBM and
  // lose bandwidth (measured on a plain copy: 5.5 TB/s with 32-row runs,
  // 5.0 with 64, 4.4 with 256).
  const int64_t target_waves = 32768;
  int64_t tpw = 1;
  while (tpw < VM_MAXTPW && tpw * target_waves < out.n_tiles) tpw *= 2;
  set_shape(out, tpw);
  // the tuner also times 2x and 4x the default (fewer, longer-running
  // waves); small passes keep the default
  out.tune_cand.clear();
  if (c.cfg.tune && c.cfg.memo && !c.analysis_only && kind != 2 && out.n_tiles >= 64)
    for (int64_t t = tpw; t <= VM_MAXTPW && t <= 4 * tpw; t *= 2) out.tune_cand.push_back(t);
  // algorithmic bytes: union footprint of every store read, and of every
  // store written, once per pass
  std::map<int64_t, std::vector<Box>> rd, wr;
  for (auto& ia : in_args) rd[ia.first].push_back(stream_box(c, c.stores.at(ia.first), ia.second, sp));
  for (auto& o : outs) {
    const auto key = written[o.second];
    const int64_t sid = L.order[key.first];
    wr[sid].push_back(stream_box(c, c.stores.at(sid), key.second, sp));
  }
  int64_t bytes = 0;
  for (auto& kv : rd) bytes += union_volume(kv.second) * (int64_t)es;
  for (auto& kv : wr) bytes += union_volume(kv.second) * (int64_t)es;
  bytes += (int64_t)(out.bc_cstore.size() + 2 * out.red_cstore.size()) * (int64_t)es;
  if (kind == 1) {
    const StoreRec& rp = c.stores.at(L.order[out.spmv_rowptr]);
    const StoreRec& col = c.stores.at(L.order[out.spmv_col]);
    const StoreRec& x = c.stores.at(L.order[out.spmv_x]);
    bytes += rp.elems * 4 + col.elems * (4 + (int64_t)es);
    // the gathered vector is read once; it is often also a streamed operand
    if (!rd.count(L.order[out.spmv_x])) bytes += x.elems * (int64_t)es;
  }
  out.alg_bytes = bytes;
  if (trace_level() > 0) {
    std::fprintf(stderr,
                 "dfx: pass kind=%d %s tier=%d regs=%d code=%zu in=%zu out=%zu bc=%zu red=%zu tiles=%lld "
                 "tiles/wave=%lld grid=%d alg_bytes=%lld staged=%d\n",
                 kind, dtype == DFX_F64 ? "f64" : "f32", out.tier, out.nreg, out.code.size(), out.ins.size(),
                 out.outs.size(), out.bc_cstore.size(), out.red_cstore.size(), (long long)out.n_tiles,
                 (long long)out.tiles_per_wave, out.grid, (long long)out.alg_bytes,
                 (int)std::count(out.st_on.begin(), out.st_on.end(), 1));
    if (trace_level() > 1)
      for (auto& K : out.code)
        std::fprintf(stderr, "dfx:   op=%u flags=%u slot=%u post=%u dst=%u a=%u b=%u c=%u imm=%08x%08x\n",
                     K.w0 & 0xff, (K.w0 >> 8) & 0xff, (K.w0 >> 16) & 0xff, K.w0 >> 24, K.w1 & 0xff,
                     (K.w1 >> 8) & 0xff, (K.w1 >> 16) & 0xff, K.w1 >> 24, K.w3, K.w2);
  }
  return DFX_OK;
}

// Split the prefix into passes: maximal runs of tasks sharing one iteration
// space and dtype; an SpMV starts a pass of its own kind.
static int build_plan(Ctx& c, int f, const std::set<int64_t>& temps, const std::vector<int64_t>& order,
                      Plan& plan) {
  plan.prefix = f;
  struct G { std::vector<const TaskRec*> tasks; Space sp; int dtype; int kind; };
  std::vector<G> groups;
  for (int j = 0; j < f; ++j) {
    const TaskRec& t = c.window[j];
    TaskShape ts;
    int rc = task_shape(c, t, ts);
    if (rc) return rc;
    if (ts.space.rank > 2) return fail(c, DFX_EUNSUPPORTED, "iteration spaces of rank > 2 are not executable");
    const bool sp = t.op == DFX_OP_SPMV_CSR;
    const int kind = sp ? 1 : (t.ndim == 0 ? 2 : 0);
    bool fresh = groups.empty() || sp || !space_eq(groups.back().sp, ts.space) ||
                 groups.back().dtype != ts.dtype || (groups.back().kind == 2) != (kind == 2);
    if (!fresh && groups.back().tasks.size() >= 48) fresh = true;
    if (fresh) groups.push_back({{}, ts.space, ts.dtype, kind});
    groups.back().tasks.push_back(&t);
  }
  // a temporary used by two passes must be materialised between them
  std::map<int64_t, std::set<int>> used_in;
  for (size_t g = 0; g < groups.size(); ++g)
    for (auto* t : groups[g].tasks)
      for (auto& a : t->args) used_in[a.store].insert((int)g);
  Lowering L(c, order);
  for (int64_t s : temps)
    if (used_in[s].size() <= 1) L.temps.insert(s);
  for (int64_t s : L.temps) plan.temps.push_back(L.cidx.at(s));
  for (auto& g : groups) {
    PassPlan pp;
    int rc = lower_pass(c, L, g.tasks, g.sp, g.dtype, g.kind, pp);
    if (rc) return rc;
    // a pass that stores nothing (every value it computes is a temporary
    // nobody reads, as the residual of a Jacobi sweep whose program has
    // already dropped it) has no effect and is not launched
    if (pp.outs.empty() && pp.red_cstore.empty()) continue;
    plan.alg_bytes += pp.alg_bytes;
    plan.passes.push_back(std::move(pp));
  }
  return DFX_OK;
}

// ---------------------------------------------------------------------------
// Execution

static void* g_dummy_stream = nullptr;  // zeroed 4 KB read by padding stream slots

// Block sums a pass's workspace holds per reduction: one per block, or one
// per tile when a compiled pass gives every tile its own block (red_split,
// at most RED_SPLIT_MAX_TILES tiles), or, for a one-tile pass with one
// reduction, the tile's summands (red_split over several blocks).
constexpr int64_t RED_SPLIT_MAX_TILES = 2048;
// blocks of a one-tile reducing pass: 16 waves of two rows each (a multiple
// of every kernel's rows per step), or for SpMV passes (one row per step)
// 32 waves of one row; DFX_RED_GLOB=<n> sets the blocks (1, 2, 4 or 8; 0: off)
constexpr int RED_SPLIT_BLOCKS = 4;
static size_t block_sum_slots(const PassPlan& p) {
  int64_t n = std::max<int64_t>(p.grid, p.n_tiles <= RED_SPLIT_MAX_TILES ? p.n_tiles : 0);
  if (p.n_tiles == 1 && p.red_cstore.size() == 1)
    n = std::max<int64_t>(n, (int64_t)RED_TH * (p.dtype == DFX_F64 ? Lanes<double>::TW : Lanes<float>::TW));
  return (size_t)n;
}

static int ensure_workspace(Ctx& c, PassPlan& p) {
  if (c.analysis_only || p.red_cstore.empty() || p.ws) return DFX_OK;
  if (c.capturing) return fail(c, DFX_ESTATE, "a new fused window appeared while a graph is being recorded");
  const size_t es = dtype_size(p.dtype);
  const size_t part = (block_sum_slots(p) * es + 255) / 256 * 256;  // one sum per block
  p.ws_bytes = part * p.red_cstore.size();
  p.ws = dev_alloc(c, p.ws_bytes);
  if (!p.ws) return fail(c, DFX_ENOMEM, "workspace allocation failed");
  return DFX_OK;
}

// Rows per step of an arithmetic pass: one (four waves per SIMD) when the
// default two-row kernel could not hold all of the pass's waves at once but
// the one-row kernel can, so the pass runs in one round instead of leaving a
// partial second one (a 4096-tile pass at three waves per SIMD, for one).
// Passes of many rounds keep two rows per step, which streams better.
// (DFX_ARITH_ROWS=1 or 2 overrides the choice.)
static int pick_rows(Ctx& c, const PassPlan& p) {
  if (p.tier != TIER_ARITH || p.kind != 0) return 0;
  const char* env = std::getenv("DFX_ARITH_ROWS");
  if (env && (env[0] == '1' || env[0] == '2')) return env[0] == '1' ? 1 : 0;
  const int64_t waves = (p.n_tiles + p.tiles_per_wave - 1) / p.tiles_per_wave;
  const int f64 = p.dtype == DFX_F64;
  const int nin = (int)p.ins.size();
  const int bi = stream_bucket(nin, TIER_ARITH) / 2 - 1;
  if (!c.n_cu) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, c.cfg.device) != hipSuccess || v < 1) v = 1;
    c.n_cu = v;
  }
  auto resident = [&](int rows) -> int64_t {
    int& w = c.waves_cu[f64][bi][rows];
    if (!w) w = std::max(1, arith_waves_per_cu(f64, nin, rows));
    return (int64_t)w * c.n_cu;
  };
  return waves > resident(0) && waves <= resident(1) ? 1 : 0;
}

// Device resources a plan holds: reduction workspaces and tuner events.
static void release_plan(Ctx& c, Plan& plan) {
  for (auto& p : plan.passes) {
    if (p.ws) dev_free(c, p.ws, p.ws_bytes);
    p.ws = nullptr;
    if (p.ev0) (void)hipEventDestroy(p.ev0);
    if (p.ev1) (void)hipEventDestroy(p.ev1);
    p.ev0 = p.ev1 = nullptr;
  }
}

// Stencil staging on (default) unless DFX_STENCIL=0.
static bool stencil_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("DFX_STENCIL");
    return !(e && e[0] == '0');
  }();
  return on;
}

// Whether a compiled pass runs each tile on a block of four waves
// (red_split): one reduction, one tile per wave, no staging or row split,
// and either a lone tile or more tiles than one block holds (so that the
// block-sum launch is needed either way) up to RED_SPLIT_MAX_TILES.
// DFX_RED_SPLIT=0 turns it off.
static bool red_split_ok(const PassPlan& p, const VmParams& P) {
  const char* e = std::getenv("DFX_RED_SPLIT");
  if (e && e[0] == '0') return false;
  return P.n_red == 1 && P.st_n == 0 && P.row_split <= 1 && p.tiles_per_wave == 1 && p.kind != 2 &&
         (p.n_tiles == 1 || (p.n_tiles > 4 && p.n_tiles <= RED_SPLIT_MAX_TILES)) && block_sum_slots(p) >= (size_t)p.n_tiles;
}

// A reducing pass whose tiles all belong to block 0 (one block sum) writes
// its 0-d results from that block; not when recorded into a batch (the
// batched executor reduces tile sums itself).  DFX_RED_DIRECT=0 turns it off.
static bool red_direct(const Ctx& c, const PassPlan& p) {
  static const bool on = [] {
    const char* e = std::getenv("DFX_RED_DIRECT");
    return !(e && e[0] == '0');
  }();
  return on && !c.batch_rec && p.n_tiles >= 1 && p.n_tiles <= 4 * p.tiles_per_wave;
}

// Blocks of four waves for `waves` waves (a multiple of 8 beyond 8 blocks,
// for the kernel's XCD-contiguous block numbering).
static int grid_for(int64_t waves) {
  int64_t grid = std::max<int64_t>(1, (waves + 3) / 4);
  if (grid > 8) grid = (grid + 7) / 8 * 8;
  return (int)grid;
}

// Columns by which a 2-D pass without reductions starts its strips early so
// that its 16-byte vectors are aligned (0: none).  A view that starts inside
// a 16-byte word (the interior of a grid, one element in) has every vector
// access straddle two words.  Shifting pays only when every stream, input
// and output, has the same offset (an in-place update of an interior view):
// for the Jacobi sweep's copy from an aligned array into the grid interior,
// moving the misalignment from the stores to the loads made the sweep slower
// (0.471 against 0.457 ms).  Row strides must keep the offset.
// DFX_COL_SHIFT=0 turns it off.
static int col_shift_for(const PassPlan& p, const VmParams& P, size_t es) {
  const char* e = std::getenv("DFX_COL_SHIFT");
  if (e && e[0] == '0') return 0;
  if (p.kind != 0 || p.is1d || P.n_red != 0 || P.st_n != 0 || !p.unit_cols || P.n_out == 0) return 0;
  const int64_t V = 16 / (int64_t)es;
  int64_t mis = -1;
  auto same = [&](const VmStream& st) {
    const uintptr_t a = (uintptr_t)st.base;
    if (a % es != 0 || st.s_row % V != 0 || st.s_col != 1) return false;
    const int64_t m = (int64_t)((a / es) % (uintptr_t)V);
    if (mis >= 0 && m != mis) return false;
    mis = m;
    return true;
  };
  for (int k = 0; k < P.n_out; ++k)
    if (!same(P.out[k])) return 0;
  for (int k = 0; k < P.n_in; ++k)
    if (!same(P.in[k])) return 0;
  return mis > 0 ? (int)mis : 0;
}

// Realigned inputs (compiled passes): a 2-D pass without reductions whose
// outputs share a misalignment m (elements past a 16-byte word, 0 < m < V)
// while some input has another one.  Shifting the strips by m aligns every
// output vector; input a then starts d_a = (m_a - m) mod V elements past a
// word, and the compiled kernel loads it with aligned vectors and a lane
// shift (realigned_row).  The Jacobi sweep's copy from an aligned array into
// the grid interior is the case.  Returns m and fills d (0: not this case).
// DFX_REALIGN=0 turns it off.
static int realign_for(const PassPlan& p, const VmParams& P, size_t es, std::vector<int8_t>& d) {
  d.clear();
  const char* e = std::getenv("DFX_REALIGN");
  if (e && e[0] == '0') return 0;
  if (p.kind != 0 || p.is1d || P.n_red != 0 || P.st_n != 0 || !p.unit_cols || P.n_out == 0) return 0;
  const int64_t V = 16 / (int64_t)es;
  auto mis = [&](const VmStream& st) -> int64_t {
    const uintptr_t a = (uintptr_t)st.base;
    if (a % es != 0 || st.s_row % V != 0 || st.s_col != 1) return -1;
    return (int64_t)((a / es) % (uintptr_t)V);
  };
  int64_t m = -1;
  for (int k = 0; k < P.n_out; ++k) {
    const int64_t mk = mis(P.out[k]);
    if (mk < 0 || (m >= 0 && mk != m)) return 0;
    m = mk;
  }
  if (m <= 0) return 0;
  bool any = false;
  for (int k = 0; k < P.n_in; ++k) {
    const int64_t mk = mis(P.in[k]);
    if (mk < 0) { d.clear(); return 0; }
    const int8_t dk = (int8_t)(((mk - m) % V + V) % V);
    d.push_back(dk);
    any = any || dk != 0;
  }
  if (!any) d.clear();
  return any ? (int)m : 0;
}

// Waves per tile of a pass without reductions (a power of two up to 32).
// With one wave per tile a pass of few tiles leaves most of the chip idle
// and each wave walks its tile's 32 rows in sequence (the 256-tile passes
// of the GMG fine level ran 256 waves); splitting a tile's rows over several
// waves changes no bit when nothing is reduced.  The split aims at about
// 8192 waves per pass, down to one row per wave for SpMV passes (one row
// per step) and two otherwise (two-row steps); transcendental passes aim at
// 32768.  Stencil-staged passes stage whole tiles and keep one wave.
// DFX_ROW_SPLIT=<n> caps it (0 or 1: off), DFX_SPLIT_WAVES=<n> sets the aim.
static int row_split_for(const PassPlan& p, const VmParams& P) {
  int cap = p.kind == 1 ? RED_TH : RED_TH / 2;
  if (const char* e = std::getenv("DFX_ROW_SPLIT")) cap = std::max(1, std::min(cap, std::atoi(e)));
  if (P.n_red != 0 || P.st_n != 0 || P.tiles_per_wave != 1 || p.kind == 2) return 1;
  // waves per pass to aim at: transcendental passes keep the VALU busy and
  // gain from a finer tail (Black-Scholes FP32 over 2^26 options, 8192
  // tiles: 0.383 ms at 8192 waves, 0.372 at 16384, 0.359 at 32768); streaming
  // passes lose from the extra waves (the COPY pass: 0.208 ms at 8192, 0.218
  // at 32768)
  int64_t target = p.tier != TIER_ARITH ? 32768 : 8192;
  if (const char* e = std::getenv("DFX_SPLIT_WAVES")) target = std::max<int64_t>(1, std::atoll(e));
  int s = 1;
  while (2 * s <= cap && P.n_tiles * 2 * s <= target) s *= 2;
  // a lone tile of one row has work for one wave only
  if (P.n_tiles == 1 && p.rows <= 1) s = 1;
  return s;
}

// Passes that run compiled when jit is on (measured on MI355X):
// transcendental passes, where the interpreter's dispatch dominates
// (Black-Scholes FP64 over 2^26 options: 0.79 against 1.05 ms); small
// passes of fewer than 1024 tiles, which are latency-bound (CG 64^2: 0.074
// against 0.100 ms per iteration; the GMG 1023^2 iteration, whose fine-level
// passes have 256 tiles: 0.82 ms with them compiled against 0.97 ms with the
// limit at 256; 4096 gave 0.82 ms as well); stencil-staged passes (the 8192^2 Jacobi
// sweep: 0.46 against 0.51 ms).  Large arithmetic and staged-SpMV passes
// stream at the interpreter's rate or slightly below it compiled (the CG
// 256^3 SpMV + dot: 438 against 390 us) and stay interpreted.
// DFX_JIT_ALL=1 compiles every pass.
static bool jit_wanted(const PassPlan& p, int st_n) {
  const char* all = std::getenv("DFX_JIT_ALL");
  if (all && all[0] == '1') return true;
  int64_t small = 1024;
  if (const char* e = std::getenv("DFX_JIT_SMALL")) small = std::atoll(e);
  return p.tier != TIER_ARITH || p.n_tiles < small || st_n > 0;
}

// The pass's program and kernel variant for compilation (rows: the rows per
// step the interpreter would take).
static std::shared_ptr<JitEntry> request_compiled(PassPlan& p, int st_n, int rows, bool sync) {
  JitProgram g;
  g.n_in = (int)p.ins.size();
  g.n_out = (int)p.outs.size();
  for (int8_t d : p.realign) g.realign.push_back(d);
  g.code = p.code;
  g.out_reg = p.out_reg;
  g.bc_reg = p.bc_reg;
  if (st_n > 0)
    for (size_t a = 0; a < p.ins.size(); ++a) {
      g.st_on.push_back(p.st_on[a]);
      g.st_dr.push_back(p.st_dr[a]);
      g.st_dc.push_back(p.st_dc[a]);
    }
  const JitVariant v = jit_variant(p.dtype == DFX_F64, p.tier, (int)p.ins.size(), p.kind == 1, st_n, rows);
  std::string name;
  const std::string src = jit_source(v, g, &name);
  return jit_request(src, name, sync);
}

// Staged streams of a pass when it runs (stencil staging on and the plan's
// views recorded).
static int staged_streams(const PassPlan& p, size_t n_stores) {
  if (!(p.st_cs >= 0 && (size_t)p.st_cs < n_stores && stencil_enabled() && p.st_on.size() == p.ins.size() &&
        p.st_dr.size() == p.ins.size() && p.st_dc.size() == p.ins.size()))
    return 0;
  int n = 0;
  for (int8_t o : p.st_on) n += o;
  return n;
}

// Does the pass name one of the stores in `ids` (as input, output,
// broadcast, reduction or SpMV operand)?
static bool pass_touches(const PassPlan& p, const std::vector<int64_t>& order, const std::vector<int64_t>& ids) {
  auto hit = [&](int cs) { return cs >= 0 && std::find(ids.begin(), ids.end(), order[cs]) != ids.end(); };
  for (auto& s : p.ins) if (hit(s.cstore)) return true;
  for (auto& s : p.outs) if (hit(s.cstore)) return true;
  for (int cs : p.bc_cstore) if (hit(cs)) return true;
  for (int cs : p.red_cstore) if (hit(cs)) return true;
  if (p.kind == 1)
    for (int cs : {p.spmv_rowptr, p.spmv_col, p.spmv_val, p.spmv_x}) if (hit(cs)) return true;
  return false;
}

static int run_pass(Ctx& c, PassPlan& p, const std::vector<int64_t>& order) {
  auto S = [&](int cs) -> StoreRec& { return c.stores.at(order[cs]); };
  const size_t es = dtype_size(p.dtype);
  int rc;
  for (auto& s : p.ins) if ((rc = ensure_alloc(c, S(s.cstore)))) return rc;
  for (auto& s : p.outs) if ((rc = ensure_alloc(c, S(s.cstore)))) return rc;
  for (int cs : p.bc_cstore) if ((rc = ensure_alloc(c, S(cs)))) return rc;
  for (int cs : p.red_cstore) if ((rc = ensure_alloc(c, S(cs)))) return rc;
  if (p.kind == 1)
    for (int cs : {p.spmv_rowptr, p.spmv_col, p.spmv_val, p.spmv_x})
      if ((rc = ensure_alloc(c, S(cs)))) return rc;
  if (c.no_alloc && !c.analysis_only) {
    if (!p.red_cstore.empty() && p.grid > NOALLOC_BLOCKS)
      return fail(c, DFX_EUNSUPPORTED, "pass of " + std::to_string(p.grid) +
                                           " blocks exceeds the allocation-free scratch (" +
                                           std::to_string(NOALLOC_BLOCKS) + " blocks)");
    if (!c.scratch) return fail(c, DFX_ESTATE, "no scratch memory on this device");
  } else if (!c.no_alloc && !c.batch_rec && (rc = ensure_workspace(c, p))) {
    return rc;
  }
  // the pass, plus the block-sum kernel when it reduces over more than one
  // block (counted once the launch shape is final)
  auto count_launches = [&]() {
    const int n_launch = p.red_cstore.empty() || red_direct(c, p) ? 1 : 2;
    c.stats.launches += n_launch;
    c.stats.alg_bytes += p.alg_bytes;
    if (c.capturing) { c.capture_launches += n_launch; c.capture_bytes += p.alg_bytes; }
  };
  if (c.analysis_only) {
    count_launches();
    return DFX_OK;
  }

  // Launch-shape tuner.  A memoised pass runs once untimed (warm-up), then
  // each candidate twice, interleaved, between two events; a timing is read
  // at the plan's next execution, so tuning adds no synchronisation of its
  // own.  A candidate replaces the default only if its faster run beats the
  // default's by 3 %.  A graph being recorded takes the default shape.
  bool timed = false;
  if (!p.tune_cand.empty() && !c.no_alloc && !c.batch_rec) {
    const int nc = (int)p.tune_cand.size();
    if (p.tune_pending >= 0 && !c.capturing) {
      float ms = 0.f;
      if (hipEventSynchronize(p.ev1) == hipSuccess && hipEventElapsedTime(&ms, p.ev0, p.ev1) == hipSuccess)
        p.tune_ms[p.tune_pending] = std::min(p.tune_ms[p.tune_pending], ms);
      p.tune_pending = -1;
    }
    if (c.capturing) {
      set_shape(p, p.tune_cand[0]);
    } else if (p.tune_step > 2 * nc) {
      int best = 0;
      for (int k = 1; k < nc; ++k)
        if (p.tune_ms[k] < p.tune_ms[best]) best = k;
      if (p.tune_ms[best] > 0.97f * p.tune_ms[0]) best = 0;
      set_shape(p, p.tune_cand[best]);
      if (trace_level() > 0)
        std::fprintf(stderr, "dfx: tuned pass kind=%d tiles=%lld tiles/wave=%lld (%.4f ms, default %.4f ms)\n",
                     p.kind, (long long)p.n_tiles, (long long)p.tiles_per_wave, p.tune_ms[best], p.tune_ms[0]);
      p.tune_cand.clear();
    } else {
      if (!p.ev0 && (hipEventCreate(&p.ev0) != hipSuccess || hipEventCreate(&p.ev1) != hipSuccess))
        return fail(c, DFX_EHIP, "event creation failed");
      if (p.tune_ms.size() != (size_t)nc) p.tune_ms.assign(nc, 3.0e38f);
      const int k = p.tune_step == 0 ? 0 : (p.tune_step - 1) % nc;
      set_shape(p, p.tune_cand[k]);
      if (p.tune_step > 0) {
        p.tune_pending = k;
        timed = true;
      }
      p.tune_step += 1;
    }
  }

  count_launches();
  VmParams P;
  std::memset(&P, 0, sizeof(P));
  P.n_code = (int)p.code.size();
  P.n_in = (int)p.ins.size();
  P.n_out = (int)p.outs.size();
  P.n_bc = (int)p.bc_cstore.size();
  P.n_red = (int)p.red_cstore.size();
  P.is1d = p.is1d;
  P.spmv = p.kind == 1;
  P.grid = p.grid;
  P.unit_cols = p.unit_cols;
  {
    const int64_t V = p.dtype == DFX_F64 ? Lanes<double>::V : Lanes<float>::V;
    P.vec_cols = p.unit_cols && (p.is1d ? (p.n1d % V == 0) : (p.cols % V == 0));
  }
  P.rows = p.rows;
  P.cols = p.cols;
  P.n1d = p.n1d;
  P.n_tiles = p.n_tiles;
  P.strips = p.strips;
  P.tiles_per_wave = p.tiles_per_wave;
  const int nb = stream_bucket(P.n_in, p.tier);
  for (int k = 0; k < VM_MAXIN; ++k) {
    if (k < P.n_in) {
      const PStream& s = p.ins[k];
      P.in[k].base = (const char*)S(s.cstore).ptr + s.off * (int64_t)es;
      P.in[k].s_row = s.s_row;
      P.in[k].s_col = s.s_col;
    } else if (k < nb) {
      P.in[k].base = g_dummy_stream;
      P.in[k].s_row = 0;
      P.in[k].s_col = 0;
    }
  }
  for (int k = 0; k < P.n_out; ++k) {
    const PStream& s = p.outs[k];
    P.out[k].base = (char*)S(s.cstore).ptr + s.off * (int64_t)es;
    P.out[k].s_row = s.s_row;
    P.out[k].s_col = s.s_col;
    P.out_reg[k] = p.out_reg[k];
  }
  for (int k = 0; k < P.n_bc; ++k) {
    P.bc[k] = S(p.bc_cstore[k]).ptr;
    P.bc_reg[k] = p.bc_reg[k];
  }
  const size_t part = (block_sum_slots(p) * es + 255) / 256 * 256;
  VmFinal F;
  std::memset(&F, 0, sizeof(F));
  F.n_red = P.n_red;
  F.nblocks = (int32_t)((p.n_tiles + 4 * p.tiles_per_wave - 1) / (4 * p.tiles_per_wave));
  for (int k = 0; k < P.n_red; ++k) {
    P.red_partials[k] = c.no_alloc ? (char*)c.scratch + (size_t)NOALLOC_BLOCKS * 8 * k : (char*)p.ws + part * k;
    F.partials[k] = P.red_partials[k];
    F.result[k] = S(p.red_cstore[k]).ptr;
    F.init[k] = p.red_init[k];
    P.red_result[k] = F.result[k];
    P.red_init[k] = F.init[k];
  }
  P.red_direct = P.n_red > 0 && red_direct(c, p) ? 1 : 0;
  if (p.kind == 1) {
    P.rowptr = (const int32_t*)S(p.spmv_rowptr).ptr;
    P.colidx = (const int32_t*)S(p.spmv_col).ptr;
    P.val = S(p.spmv_val).ptr;
    P.x = S(p.spmv_x).ptr;
    P.nnz = (int32_t)std::min<int64_t>(S(p.spmv_col).elems, S(p.spmv_val).elems);
    P.nx = S(p.spmv_x).elems;
    // staging pays where many waves run at once (L2 holds x for its
    // neighbours); a small system is latency-bound and walks CSR directly
    // (DFX_SPMV_STAGE=0 or 1 overrides the choice)
    const char* st = std::getenv("DFX_SPMV_STAGE");
    P.sp_stage = st && (st[0] == '0' || st[0] == '1') ? st[0] == '1' : p.n_tiles >= 256;
    // a one-tile pass is one block: its four waves compute the rows together
    // (DFX_SPMV_COOP=0 or 1 overrides)
    const char* co = std::getenv("DFX_SPMV_COOP");
    P.sp_coop = (p.n_tiles == 1 && p.grid == 1) &&
                (co && (co[0] == '0' || co[0] == '1') ? co[0] == '1' : true);
  }
  for (size_t i = 0; i < p.code.size(); ++i) P.code[i] = p.code[i];
  P.st_n = 0;
  if (staged_streams(p, order.size()) > 0) {
    const StoreRec& ss = S(p.st_cs);
    for (size_t a = 0; a < p.ins.size(); ++a) {
      P.st_on[a] = p.st_on[a];
      P.st_dr[a] = p.st_dr[a];
      P.st_dc[a] = p.st_dc[a];
      P.st_n += p.st_on[a];
    }
    P.st_base = (const char*)ss.ptr + p.st_off0 * (int64_t)es;
    P.st_srow = p.st_srow;
    P.st_lim = ss.elems - p.st_off0;
  }
  P.row_split = 1;
  P.col_shift = 0;
  if (c.batch_rec) return batch_record_pass(c, P, F, p.dtype, p.tier);
  const int rows = pick_rows(c, p);
  // compiled kernel, once ready (module loading is kept out of captures);
  // a pass with realigned inputs compiles them in (see realign_for) and runs
  // its kernel only while its streams keep those alignments
  hipFunction_t fn = nullptr;
  std::vector<int8_t> ra;
  const int ra_shift = c.cfg.jit ? realign_for(p, P, es, ra) : 0;
  if (c.cfg.jit) {
    if (!p.jit_checked) {
      p.jit_checked = true;
      p.realign = ra;
      p.realign_shift = ra_shift;
      if (jit_wanted(p, P.st_n) || ra_shift > 0) p.jit = request_compiled(p, P.st_n, rows, c.cfg.jit == 2);
    }
    if (p.jit && ra == p.realign) fn = jit_function(*p.jit, c.cfg.device, !c.capturing);
  }
  // column shift (aligned output vectors), then row split, of passes
  // without reductions; either changes the launch shape only
  const int cs_shift = fn && ra_shift > 0 ? ra_shift : col_shift_for(p, P, es);
  if (const int cs = cs_shift; cs > 0) {
    const int64_t TWp = p.dtype == DFX_F64 ? Lanes<double>::TW : Lanes<float>::TW;
    const int64_t row_tiles = p.n_tiles / std::max<int64_t>(1, p.strips);
    P.col_shift = cs;
    P.vec_cols = 0;
    P.strips = (p.cols + cs + TWp - 1) / TWp;
    P.n_tiles = row_tiles * P.strips;
    P.grid = grid_for((P.n_tiles + p.tiles_per_wave - 1) / p.tiles_per_wave);
  }
  if (const int rs = row_split_for(p, P); rs > 1) {
    P.row_split = rs;
    P.sp_coop = 0;
    P.grid = grid_for(P.n_tiles * rs);
  }
  // a compiled pass of one reduction and few tiles gives each tile a block
  // of four waves (red_split; bit-identical tile sums)
  if (fn && red_split_ok(p, P)) {
    // a one-tile pass spreads its rows over RED_SPLIT_BLOCKS blocks (two
    // rows per wave) and leaves the ordered sum of the summands to the
    // block-sum reduction, which the next compiled one-block pass (the
    // scalar task after a dot product) takes over (DFX_RED_GLOB=0: one block)
    const char* rg = std::getenv("DFX_RED_GLOB");
    int B = P.spmv ? 2 * RED_SPLIT_BLOCKS : RED_SPLIT_BLOCKS;
    if (rg && (rg[0] == '0' || rg[0] == '1' || rg[0] == '2' || rg[0] == '4' || rg[0] == '8') && !rg[1])
      B = rg[0] == '0' ? 1 : std::min(B, rg[0] - '0');
    if (p.n_tiles != 1) B = 1;
    P.red_split = B;
    P.sp_coop = 0;
    P.grid = (int)p.n_tiles * B;
    F.nblocks = (int)p.n_tiles;
    if (B > 1) {
      F.tile = 1;
      F.nblocks = 0;
      F.is1d = P.is1d;
      F.col_shift = P.col_shift;
      F.n1d = P.n1d;
      F.rows = P.rows;
      F.cols = P.cols;
      if (P.red_direct) {
        // the block-sum reduction now follows (count_launches assumed none)
        P.red_direct = 0;
        c.stats.launches += 1;
        if (c.capturing) c.capture_launches += 1;
      }
    }
  }
  // Block sums an earlier pass left waiting: a compiled one-block pass of
  // the same element type reduces them first, in its own launch (the same
  // tree as the block-sum kernel); a pass that reduces (its block sums may
  // share the allocation-free scratch) or names one of their result stores
  // has them reduced by the block-sum kernel before it; any other pass runs
  // with them still waiting (it reads none of their stores).
  // DFX_FIN_ATTACH=0 turns the attachment off.
  int e = 0;
  if (c.fin_pending) {
    const char* fa = std::getenv("DFX_FIN_ATTACH");
    const bool fin_attach = !(fa && fa[0] == '0');
    if (fin_attach && fn && P.grid == 1 && c.fin_f64 == (p.dtype == DFX_F64 ? 1 : 0) &&
        c.fin.nblocks <= FIN_MAX_CHUNKS * FINAL_CHUNK) {
      P.fin = c.fin;
      c.fin_pending = false;
      c.stats.launches -= 1;
      if (c.capturing) c.capture_launches -= 1;
    } else if (P.n_red > 0 || pass_touches(p, order, c.fin_stores)) {
      e = launch_pending_final(c);
    }
  }
  if (timed) (void)hipEventRecord(p.ev0, c.stream);
  if (e != 0) {
  } else if (fn) {
    const JitVariant v = jit_variant(p.dtype == DFX_F64, p.tier, P.n_in, P.spmv, P.st_n, rows);
    void* args[] = {(void*)&P};
    e = (int)hipModuleLaunchKernel(fn, (unsigned)P.grid, 1, 1, BLOCK, 1, 1, (unsigned)vm_dyn_lds_bytes(P, v.sten != 0),
                                   c.stream, args, nullptr);
    c.stats.compiled_launches += 1;
    if (c.capturing) c.capture_compiled += 1;
  } else {
    e = launch_vm(P, p.dtype == DFX_F64, p.tier, rows, c.stream);
  }
  if (e == 0 && F.n_red > 0 && !P.red_direct) {
    // its block sums wait for the next pass (above), or for the window's end
    c.fin_pending = true;
    c.fin = F;
    c.fin_f64 = p.dtype == DFX_F64 ? 1 : 0;
    c.fin_stores.clear();
    for (int cs : p.red_cstore) c.fin_stores.push_back(order[cs]);
  }
  if (timed) (void)hipEventRecord(p.ev1, c.stream);
  if (e != 0) return fail(c, DFX_EHIP, std::string("kernel launch failed: ") + hipGetErrorString((hipError_t)e));
  return DFX_OK;
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// may_grow: called because the window filled up (not from a flush); under
// auto_window a full window whose every task fuses is kept and the window
// size doubled instead
static int dispatch_one(Ctx& c, bool may_grow = false) {
  if (c.window.empty()) return DFX_OK;
  if (!c.deferred_free.empty()) drain_deferred_frees(c);
  std::vector<int64_t> order;
  std::string key = canonical_key(c, order);
  Plan* plan = nullptr;
  std::unique_ptr<Plan> owned;
  bool hit = false;
  if (c.cfg.memo) {
    auto it = c.memo.find(key);
    if (it != c.memo.end()) { plan = it->second.get(); hit = true; }
  }
  const bool grow = may_grow && c.cfg.auto_window > 0 && c.window_cur < c.cfg.auto_window;
  if (!plan) {
    const double t0 = now_s();
    const int f = c.cfg.fuse ? longest_prefix(c) : 1;
    // the decision needs the analysis only: no plan is built for a window
    // that keeps growing (its stores may still be named by the application)
    if (grow && f == (int)c.window.size()) {
      c.stats.analysis_seconds += now_s() - t0;
      c.window_cur = (int)std::min<int64_t>(2 * (int64_t)c.window_cur, c.cfg.auto_window);
      return DFX_OK;
    }
    // A group one kernel cannot hold is cut short: every prefix of a fusible
    // prefix is fusible, so the longest prefix that lowers is dispatched and
    // the rest stays in the window.
    int rc;
    for (int g = f;; --g) {
      std::set<int64_t> temps;
      if (c.cfg.fuse) temps = temporaries(c, g);
      owned.reset(new Plan());
      c.over_limit = false;
      rc = build_plan(c, g, temps, order, *owned);
      if (!(rc == DFX_EUNSUPPORTED && c.over_limit && g > 1)) break;
    }
    if (rc) {
      if (!(c.analysis_only && rc == DFX_EUNSUPPORTED)) return rc;
      owned->passes.clear();
    }
    c.stats.analysis_seconds += now_s() - t0;
    c.stats.memo_misses += 1;
    plan = owned.get();
    if (c.cfg.memo) {
      if (c.memo.size() >= 4096) {
        // a recorded graph keeps using the workspaces of the plans it ran, so
        // they are returned only while no graph exists
        const bool graphs_live = std::any_of(c.graphs.begin(), c.graphs.end(), [](const auto& g) { return (bool)g; });
        if (!c.analysis_only && !graphs_live && !c.capturing)
          for (auto& kv : c.memo) release_plan(c, *kv.second);
        c.memo.clear();
      }
      c.memo.emplace(key, std::move(owned));
    }
  } else {
    c.stats.memo_hits += 1;
  }
  if (grow && hit && plan->prefix == (int)c.window.size()) {
    c.window_cur = (int)std::min<int64_t>(2 * (int64_t)c.window_cur, c.cfg.auto_window);
    return DFX_OK;
  }
  if (c.no_alloc && !c.analysis_only) {
    // nothing of the group is launched unless every pass can run without
    // device memory: its stores allocated, its block sums within the scratch
    for (auto& p : plan->passes) {
      std::vector<int> need;
      for (auto& s : p.ins) need.push_back(s.cstore);
      for (auto& s : p.outs) need.push_back(s.cstore);
      for (int cs : p.bc_cstore) need.push_back(cs);
      for (int cs : p.red_cstore) need.push_back(cs);
      if (p.kind == 1) for (int cs : {p.spmv_rowptr, p.spmv_col, p.spmv_val, p.spmv_x}) need.push_back(cs);
      for (int cs : need) {
        const StoreRec& s = c.stores.at(order[cs]);
        if (!s.ptr && s.bytes != 0)
          return fail(c, DFX_ESTATE, "store " + std::to_string(s.id) +
                                         " needs device memory in an allocation-free flush");
      }
      if (!p.red_cstore.empty() && p.grid > NOALLOC_BLOCKS)
        return fail(c, DFX_EUNSUPPORTED, "pass of " + std::to_string(p.grid) +
                                             " blocks exceeds the allocation-free scratch");
    }
  }
  for (auto& p : plan->passes) {
    int rc = run_pass(c, p, order);
    if (rc) {
      if (owned && !c.analysis_only && !c.capturing) release_plan(c, *owned);
      return rc;
    }
  }
  // an unmemoised plan is used once (its workspace is freed in stream order),
  // unless a graph being recorded refers to it
  if (owned && !c.analysis_only && !c.capturing) release_plan(c, *owned);
  // record the group
  dfx_group_info gi;
  std::memset(&gi, 0, sizeof(gi));
  gi.first_task = c.window.front().seq;
  gi.prefix_len = plan->prefix;
  gi.memo_hit = hit;
  gi.n_passes = (int)plan->passes.size();
  for (int i = 0; i < gi.n_passes && i < 8; ++i) gi.pass_kind[i] = plan->passes[i].kind;
  gi.n_temporaries = (int)std::min<size_t>(plan->temps.size(), DFX_INFO_MAX);
  for (int i = 0; i < gi.n_temporaries; ++i) gi.temporaries[i] = order[plan->temps[i]];
  gi.alg_bytes = plan->alg_bytes;
  if (c.groups.size() < 1000000) c.groups.push_back(gi);
  c.stats.groups_dispatched += 1;
  c.stats.tasks_dispatched += plan->prefix;
  c.stats.temporaries_eliminated += (int64_t)plan->temps.size();
  // retire the prefix: drop the window's references
  std::vector<int64_t> touched;
  for (int j = 0; j < plan->prefix; ++j) {
    const TaskRec& t = c.window.front();
    std::set<int64_t> seen;
    for (auto& a : t.args)
      if (seen.insert(a.store).second) {
        c.stores.at(a.store).pending -= 1;
        touched.push_back(a.store);
      }
    c.window.pop_front();
  }
  for (int64_t s : touched) maybe_free(c, s);
  return DFX_OK;
}

static int flush(Ctx& c) {
  while (!c.window.empty()) {
    int rc = dispatch_one(c);
    if (rc) return rc;
  }
  if (const int e = launch_pending_final(c))
    return fail(c, DFX_EHIP, std::string("kernel launch failed: ") + hipGetErrorString((hipError_t)e));
  return DFX_OK;
}

}  // namespace dfx

// ===========================================================================
// C ABI
using namespace dfx;

namespace {
constexpr char kPlanMagic[8] = {'D', 'F', 'X', 'P', 'L', 'A', 'N', '1'};
const std::string& build_stamp() {
  static const std::string s = std::string(dfx_version()) + " " + __DATE__ + " " + __TIME__;
  return s;
}
uint64_t fnv1a(const char* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) { h ^= (unsigned char)p[i]; h *= 1099511628211ull; }
  return h;
}
struct Wr {
  std::string b;
  template <class T> void v(const T& x) { b.append((const char*)&x, sizeof(T)); }
  template <class T> void vec(const std::vector<T>& x) {
    const uint32_t n = (uint32_t)x.size();
    v(n);
    if (n) b.append((const char*)x.data(), n * sizeof(T));
  }
  void str(const std::string& x) {
    const uint32_t n = (uint32_t)x.size();
    v(n);
    b.append(x);
  }
};
struct Rd {
  const char* p;
  const char* e;
  bool ok = true;
  template <class T> void v(T& x) {
    if (!ok || (size_t)(e - p) < sizeof(T)) { ok = false; x = T(); return; }
    std::memcpy(&x, p, sizeof(T));
    p += sizeof(T);
  }
  template <class T> void vec(std::vector<T>& x) {
    uint32_t n = 0;
    v(n);
    if (!ok || n > (1u << 24) || (size_t)(e - p) < (size_t)n * sizeof(T)) { ok = false; return; }
    x.resize(n);
    if (n) std::memcpy(x.data(), p, n * sizeof(T));
    p += (size_t)n * sizeof(T);
  }
  void str(std::string& x) {
    uint32_t n = 0;
    v(n);
    if (!ok || (size_t)(e - p) < n) { ok = false; return; }
    x.assign(p, n);
    p += n;
  }
};
template <class IO, class P> void pass_fields(IO& io, P& q) {
  io.v(q.kind); io.v(q.dtype); io.v(q.is1d); io.v(q.rows); io.v(q.cols); io.v(q.n1d);
  io.v(q.n_tiles); io.v(q.strips); io.v(q.tiles_per_wave); io.v(q.grid); io.v(q.nreg);
  io.v(q.tier); io.v(q.unit_cols);
  io.vec(q.ins); io.vec(q.outs); io.vec(q.out_reg); io.vec(q.bc_cstore); io.vec(q.bc_reg);
  io.vec(q.red_cstore); io.vec(q.red_init);
  io.v(q.spmv_rowptr); io.v(q.spmv_col); io.v(q.spmv_val); io.v(q.spmv_x);
  io.vec(q.code); io.vec(q.imm); io.v(q.alg_bytes); io.vec(q.tune_cand);
  io.v(q.st_cs); io.v(q.st_off0); io.v(q.st_srow); io.vec(q.st_on); io.vec(q.st_dr); io.vec(q.st_dc);
}
}  // namespace

struct dfx_ctx : public dfx::Ctx {};

extern "C" {

const char* dfx_version(void) { return "dfx 0.1 (gfx950)"; }

const char* dfx_last_error(dfx_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int dfx_create(const dfx_config* cfg, dfx_ctx** out) {
  if (!cfg || !out) return DFX_EINVAL;
  if (cfg->window_size < 1) return DFX_EINVAL;
  if (cfg->auto_window < 0 || (cfg->auto_window > 0 && (cfg->auto_window < cfg->window_size || !cfg->fuse)))
    return DFX_EINVAL;
  if (cfg->jit < 0 || cfg->jit > 2 || (cfg->jit && !cfg->memo)) return DFX_EINVAL;
  dfx_ctx* c = new dfx_ctx();
  c->cfg = *cfg;
  // DFX_JIT=1|2 turns compiled passes on for contexts created with jit = 0
  // (runs an unchanged program on compiled kernels)
  if (const char* j = std::getenv("DFX_JIT"))
    if (!c->cfg.jit && c->cfg.memo && (j[0] == '1' || j[0] == '2') && !j[1]) c->cfg.jit = j[0] - '0';
  c->window_cur = cfg->window_size;
  c->stream = (hipStream_t)cfg->stream;
  c->analysis_only = cfg->device < 0;
  if (!c->analysis_only) {
    if (hipSetDevice(cfg->device) != hipSuccess) { delete c; return DFX_EHIP; }
    if (!g_dummy_stream) {
      if (hipMalloc(&g_dummy_stream, 4096) != hipSuccess) { delete c; return DFX_ENOMEM; }
      if (hipMemset(g_dummy_stream, 0, 4096) != hipSuccess) { delete c; return DFX_EHIP; }
    }
    // the allocation-free flush's scratch array on this device (current)
    if (scratch_address(cfg->device, &c->scratch) != 0) { delete c; return DFX_EHIP; }
    if (!cfg->alloc) {
      hipMemPool_t pool;
      if (hipDeviceGetDefaultMemPool(&pool, cfg->device) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
      }
    }
  }
  *out = c;
  return DFX_OK;
}

int dfx_destroy(dfx_ctx* c) {
  if (!c) return DFX_EINVAL;
  if (c->server) (void)dfx_serve_stop(c);
  int rc = c->capturing ? DFX_OK : flush(*c);
  if (c->batch_rec) batch_record_drop(*c);
  if (!c->analysis_only) {
    drain_deferred_frees(*c);
    for (auto& kv : c->memo) release_plan(*c, *kv.second);
    for (auto& kv : c->stores)
      if (kv.second.ptr && !kv.second.external) dev_free(*c, kv.second.ptr, kv.second.bytes);
    for (auto& g : c->graphs) {
      if (g && g->exec) (void)hipGraphExecDestroy(g->exec);
      if (g && g->graph) (void)hipGraphDestroy(g->graph);
    }
    (void)hipStreamSynchronize(c->stream);
  }
  delete c;
  return rc;
}

static int new_store(dfx_ctx* c, int32_t ndim, const int64_t* shape, int32_t dtype, dfx_store* out,
                     StoreRec** rec) {
  if (!c || !out || ndim < 0 || ndim > DFX_MAX_DIM || (ndim > 0 && !shape))
    return c ? fail(*c, DFX_EINVAL, "bad store arguments") : DFX_EINVAL;
  if (dtype < DFX_F32 || dtype > DFX_I64) return fail(*c, DFX_EINVAL, "bad dtype");
  StoreRec s;
  s.id = c->next_store++;
  s.ndim = ndim;
  s.dtype = dtype;
  s.elems = 1;
  for (int k = 0; k < ndim; ++k) {
    if (shape[k] < 0) return fail(*c, DFX_EINVAL, "negative extent");
    s.shape[k] = shape[k];
    s.elems *= shape[k];
  }
  s.bytes = (size_t)s.elems * dtype_size(dtype);
  auto it = c->stores.emplace(s.id, s).first;
  *out = s.id;
  *rec = &it->second;
  return DFX_OK;
}

int dfx_store_create(dfx_ctx* c, int32_t ndim, const int64_t* shape, int32_t dtype, dfx_store* out) {
  StoreRec* r;
  return new_store(c, ndim, shape, dtype, out, &r);
}

int dfx_store_wrap(dfx_ctx* c, void* dptr, int32_t ndim, const int64_t* shape, int32_t dtype,
                   dfx_store* out) {
  StoreRec* r;
  int rc = new_store(c, ndim, shape, dtype, out, &r);
  if (rc) return rc;
  r->ptr = dptr;
  r->external = true;
  return DFX_OK;
}

static StoreRec* find_store(dfx_ctx* c, dfx_store s) {
  auto it = c->stores.find(s);
  return it == c->stores.end() ? nullptr : &it->second;
}

int dfx_store_write(dfx_ctx* c, dfx_store s, const void* host, size_t bytes) {
  if (!c) return DFX_EINVAL;
  int rc = flush(*c);
  if (rc) return rc;
  StoreRec* r = find_store(c, s);
  if (!r) return fail(*c, DFX_ENOTFOUND, "unknown store");
  if (bytes != r->bytes) return fail(*c, DFX_EINVAL, "byte count differs from the store's size");
  if (c->analysis_only) return fail(*c, DFX_ESTATE, "analysis-only context holds no values");
  if ((rc = ensure_alloc(*c, *r))) return rc;
  if (bytes == 0) return DFX_OK;
  HIPCHK(*c, hipMemcpyAsync(r->ptr, host, bytes, hipMemcpyHostToDevice, c->stream));
  HIPCHK(*c, hipStreamSynchronize(c->stream));
  return DFX_OK;
}

int dfx_store_read(dfx_ctx* c, dfx_store s, void* host, size_t bytes) {
  if (!c) return DFX_EINVAL;
  int rc = flush(*c);
  if (rc) return rc;
  StoreRec* r = find_store(c, s);
  if (!r) return fail(*c, DFX_ENOTFOUND, "unknown store");
  if (bytes != r->bytes) return fail(*c, DFX_EINVAL, "byte count differs from the store's size");
  if (c->analysis_only) return fail(*c, DFX_ESTATE, "analysis-only context holds no values");
  if (bytes == 0) return DFX_OK;
  if (!r->ptr) return fail(*c, DFX_ESTATE, "store was never written");
  HIPCHK(*c, hipMemcpyAsync(host, r->ptr, bytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(*c, hipStreamSynchronize(c->stream));
  return DFX_OK;
}

int dfx_store_device_ptr(dfx_ctx* c, dfx_store s, void** dptr) {
  if (!c || !dptr) return DFX_EINVAL;
  int rc = flush(*c);
  if (rc) return rc;
  StoreRec* r = find_store(c, s);
  if (!r) return fail(*c, DFX_ENOTFOUND, "unknown store");
  if (c->analysis_only) return fail(*c, DFX_ESTATE, "analysis-only context holds no values");
  if ((rc = ensure_alloc(*c, *r))) return rc;
  *dptr = r->ptr;
  return DFX_OK;
}

int dfx_store_release(dfx_ctx* c, dfx_store s) {
  if (!c) return DFX_EINVAL;
  StoreRec* r = find_store(c, s);
  if (!r || r->app_refs <= 0) return fail(*c, DFX_ENOTFOUND, "unknown or released store");
  r->app_refs -= 1;
  maybe_free(*c, s);
  return DFX_OK;
}

int dfx_proj_identity(dfx_ctx* c, int32_t ndim, dfx_proj* out) {
  if (!c || !out || ndim < 0 || ndim > DFX_MAX_DIM) return DFX_EINVAL;
  ProjRec p;
  p.nin = p.nout = ndim;
  for (int k = 0; k < ndim; ++k) p.keep[k] = k;
  *out = intern_proj(*c, p);
  return DFX_OK;
}

int dfx_proj_drop(dfx_ctx* c, int32_t ndim_in, uint32_t keep_mask, dfx_proj* out) {
  if (!c || !out || ndim_in < 0 || ndim_in > DFX_MAX_DIM) return DFX_EINVAL;
  if (keep_mask >> ndim_in) return fail(*c, DFX_EINVAL, "keep mask names dims beyond the launch rank");
  ProjRec p;
  p.nin = ndim_in;
  for (int d = 0; d < ndim_in; ++d)
    if (keep_mask & (1u << d)) p.keep[p.nout++] = d;
  *out = intern_proj(*c, p);
  return DFX_OK;
}

int dfx_part_none(dfx_ctx* c, dfx_part* out) {
  if (!c || !out) return DFX_EINVAL;
  PartRec p;
  p.kind = PK_NONE;
  *out = intern_part(*c, p);
  return DFX_OK;
}

int dfx_part_tiling(dfx_ctx* c, int32_t ndim, const int64_t* tile, const int64_t* offset, dfx_proj proj,
                    dfx_part* out) {
  if (!c || !out || ndim < 0 || ndim > DFX_MAX_DIM || (ndim > 0 && (!tile || !offset))) return DFX_EINVAL;
  if (proj < 0 || proj >= (int)c->projs.size()) return fail(*c, DFX_ENOTFOUND, "unknown projection");
  if (c->projs[proj].nout != ndim) return fail(*c, DFX_EINVAL, "projection output rank differs from tile rank");
  PartRec p;
  p.kind = PK_TILING;
  p.ndim = ndim;
  for (int k = 0; k < ndim; ++k) {
    if (tile[k] < 0) return fail(*c, DFX_EINVAL, "negative tile extent");
    p.tile[k] = tile[k];
    p.off[k] = offset[k];
  }
  p.proj = proj;
  *out = intern_part(*c, p);
  return DFX_OK;
}

int dfx_part_image(dfx_ctx* c, dfx_store src, dfx_part src_part, dfx_part* out) {
  if (!c || !out) return DFX_EINVAL;
  if (!find_store(c, src)) return fail(*c, DFX_ENOTFOUND, "unknown source store");
  if (src_part < 0 || src_part >= (int)c->parts.size()) return fail(*c, DFX_ENOTFOUND, "unknown partition");
  if (c->parts[src_part].kind == PK_IMAGE) return fail(*c, DFX_EINVAL, "nested Image partitions");
  PartRec p;
  p.kind = PK_IMAGE;
  p.img_src = src;
  p.img_part = src_part;
  *out = intern_part(*c, p);
  return DFX_OK;
}

int dfx_submit(dfx_ctx* c, const dfx_task* task) {
  if (!c || !task) return DFX_EINVAL;
  TaskRec t;
  t.op = task->op;
  t.ndim = task->ndim;
  if (t.ndim < 0 || t.ndim > DFX_MAX_DIM || (t.ndim > 0 && !task->launch))
    return fail(*c, DFX_EINVAL, "bad launch domain");
  for (int k = 0; k < t.ndim; ++k) t.launch[k] = task->launch[k];
  if (task->nargs < 0 || (task->nargs > 0 && !task->args) || task->nimm < 0 || (task->nimm > 0 && !task->imm))
    return fail(*c, DFX_EINVAL, "bad argument lists");
  for (int i = 0; i < task->nargs; ++i) t.args.push_back({task->args[i].store, task->args[i].part, task->args[i].priv});
  for (int i = 0; i < task->nimm; ++i) t.imm.push_back(task->imm[i]);
  int rc = validate(*c, t);
  if (rc) return rc;
  t.seq = c->next_seq++;
  std::set<int64_t> seen;
  for (auto& a : t.args)
    if (seen.insert(a.store).second) c->stores.at(a.store).pending += 1;
  c->window.push_back(std::move(t));
  c->stats.tasks_submitted += 1;
  if ((int)c->window.size() >= c->window_cur) return dispatch_one(*c, true);
  return DFX_OK;
}

int dfx_flush(dfx_ctx* c) { return c ? flush(*c) : DFX_EINVAL; }

int dfx_flush_noalloc(dfx_ctx* c) {
  if (!c) return DFX_EINVAL;
  c->no_alloc = true;
  const int rc = flush(*c);
  c->no_alloc = false;
  return rc;
}

// ---- on-disk plan cache ----------------------------------------------------
// File: magic, format version, build stamp, FNV-1a 64 checksum of the body,
// then the body: entry count and, per entry, the canonical key and the plan.
// Plans name stores by canonical index and carry no device state (workspaces
// are allocated at first execution), so a plan is valid for its key in any
// context of the same build.


int dfx_plan_cache_save(dfx_ctx* c, const char* path, int64_t* n_saved) {
  if (!c || !path) return DFX_EINVAL;
  Wr body;
  body.v((uint32_t)c->memo.size());
  for (const auto& kv : c->memo) {
    const Plan& pl = *kv.second;
    body.str(kv.first);
    body.v(pl.prefix);
    body.vec(pl.temps);
    body.v(pl.alg_bytes);
    body.v((uint32_t)pl.passes.size());
    for (const PassPlan& p : pl.passes) {
      PassPlan q = p;   // a pass still being tuned is saved with its default shape
      if (!q.tune_cand.empty()) set_shape(q, q.tune_cand[0]);
      pass_fields(body, q);
    }
  }
  Wr head;
  head.b.append(kPlanMagic, 8);
  head.v((uint32_t)sizeof(PassPlan));
  head.str(build_stamp());
  head.v(fnv1a(body.b.data(), body.b.size()));
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(*c, DFX_EINVAL, std::string("cannot write ") + path);
  const bool ok = std::fwrite(head.b.data(), 1, head.b.size(), f) == head.b.size() &&
                  std::fwrite(body.b.data(), 1, body.b.size(), f) == body.b.size();
  if (std::fclose(f) != 0 || !ok) return fail(*c, DFX_EINVAL, std::string("write failed: ") + path);
  if (n_saved) *n_saved = (int64_t)c->memo.size();
  return DFX_OK;
}

int dfx_plan_cache_load(dfx_ctx* c, const char* path, int64_t* n_loaded) {
  if (!c || !path) return DFX_EINVAL;
  if (!c->cfg.memo || !c->cfg.fuse) return fail(*c, DFX_ESTATE, "the plan cache needs memo = 1 and fuse = 1");
  if (c->capturing) return fail(*c, DFX_ESTATE, "not while a graph is being recorded");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(*c, DFX_ENOTFOUND, std::string("cannot read ") + path);
  std::string data;
  char buf[1 << 16];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) data.append(buf, got);
  std::fclose(f);
  Rd rd{data.data(), data.data() + data.size()};
  if (data.size() < 8 || std::memcmp(data.data(), kPlanMagic, 8) != 0)
    return fail(*c, DFX_EINVAL, "not a plan cache file");
  rd.p += 8;
  uint32_t pp_size = 0;
  std::string stamp;
  uint64_t sum = 0;
  rd.v(pp_size);
  rd.str(stamp);
  rd.v(sum);
  if (!rd.ok || pp_size != sizeof(PassPlan) || stamp != build_stamp())
    return fail(*c, DFX_EINVAL, "plan cache written by another build of the library");
  if (fnv1a(rd.p, (size_t)(rd.e - rd.p)) != sum) return fail(*c, DFX_EINVAL, "plan cache checksum mismatch");
  uint32_t n = 0;
  rd.v(n);
  std::vector<std::pair<std::string, std::unique_ptr<Plan>>> got_plans;
  for (uint32_t i = 0; i < n && rd.ok; ++i) {
    std::string key;
    auto pl = std::make_unique<Plan>();
    uint32_t np = 0;
    rd.str(key);
    rd.v(pl->prefix);
    rd.vec(pl->temps);
    rd.v(pl->alg_bytes);
    rd.v(np);
    if (!rd.ok || np > 64) { rd.ok = false; break; }
    pl->passes.resize(np);
    for (PassPlan& q : pl->passes) {
      pass_fields(rd, q);
      if (!c->cfg.tune) q.tune_cand.clear();
    }
    got_plans.emplace_back(std::move(key), std::move(pl));
  }
  if (!rd.ok || rd.p != rd.e) return fail(*c, DFX_EINVAL, "malformed plan cache");
  int64_t added = 0;
  for (auto& kv : got_plans) {
    if (c->memo.size() >= 4096) break;
    auto ins = c->memo.emplace(std::move(kv.first), std::move(kv.second));
    if (!ins.second) continue;
    ++added;
    // workspaces now, so that a graph can be recorded before any eager run
    for (PassPlan& q : ins.first->second->passes) {
      const int rc = ensure_workspace(*c, q);
      if (rc) return rc;
    }
  }
  if (n_loaded) *n_loaded = added;
  return DFX_OK;
}

int dfx_window_size(dfx_ctx* c, int32_t* out) {
  if (!c || !out) return DFX_EINVAL;
  *out = c->window_cur;
  return DFX_OK;
}

int dfx_sync(dfx_ctx* c) {
  if (!c) return DFX_EINVAL;
  int rc = flush(*c);
  if (rc) return rc;
  if (!c->analysis_only) HIPCHK(*c, hipStreamSynchronize(c->stream));
  return DFX_OK;
}

int dfx_graph_begin(dfx_ctx* c) {
  if (!c) return DFX_EINVAL;
  if (c->analysis_only) return fail(*c, DFX_ESTATE, "analysis-only context");
  if (c->capturing) return fail(*c, DFX_ESTATE, "already recording");
  int rc = flush(*c);
  if (rc) return rc;
  if (!c->stream) return fail(*c, DFX_ESTATE, "graphs need an explicit stream");
  HIPCHK(*c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  c->capturing = true;
  c->capture_launches = 0;
  c->capture_bytes = 0;
  c->capture_compiled = 0;
  return DFX_OK;
}

int dfx_graph_end(dfx_ctx* c, int32_t* graph_id) {
  if (!c || !graph_id) return DFX_EINVAL;
  if (!c->capturing) return fail(*c, DFX_ESTATE, "not recording");
  int rc = flush(*c);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  c->capturing = false;
  if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
  if (e != hipSuccess) return fail(*c, DFX_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  std::unique_ptr<Graph> G(new Graph());
  G->graph = g;
  e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) { (void)hipGraphDestroy(g); return fail(*c, DFX_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)); }
  G->launches = c->capture_launches;
  G->alg_bytes = c->capture_bytes;
  G->compiled = c->capture_compiled;
  c->graphs.push_back(std::move(G));
  *graph_id = (int32_t)c->graphs.size() - 1;
  return DFX_OK;
}

int dfx_graph_launch(dfx_ctx* c, int32_t id) {
  if (!c) return DFX_EINVAL;
  if (id < 0 || id >= (int)c->graphs.size() || !c->graphs[id]) return fail(*c, DFX_ENOTFOUND, "unknown graph");
  int rc = flush(*c);
  if (rc) return rc;
  HIPCHK(*c, hipGraphLaunch(c->graphs[id]->exec, c->stream));
  c->stats.graph_replays += 1;
  c->stats.launches += c->graphs[id]->launches;
  c->stats.alg_bytes += c->graphs[id]->alg_bytes;
  c->stats.compiled_launches += c->graphs[id]->compiled;
  return DFX_OK;
}

int dfx_graph_destroy(dfx_ctx* c, int32_t id) {
  if (!c) return DFX_EINVAL;
  if (id < 0 || id >= (int)c->graphs.size() || !c->graphs[id]) return fail(*c, DFX_ENOTFOUND, "unknown graph");
  (void)hipStreamSynchronize(c->stream);
  (void)hipGraphExecDestroy(c->graphs[id]->exec);
  (void)hipGraphDestroy(c->graphs[id]->graph);
  c->graphs[id].reset();
  return DFX_OK;
}

int dfx_jit_wait(void) {
  jit_wait_idle();
  return DFX_OK;
}

int dfx_jit_info_get(dfx_jit_info* out) {
  if (!out) return DFX_EINVAL;
  const JitCounters n = jit_counters();
  std::memset(out, 0, sizeof(*out));
  out->compiled = n.compiled;
  out->failed = n.failed;
  out->disk_hits = n.disk_hits;
  out->pending = n.pending;
  out->compile_seconds = n.seconds;
  return DFX_OK;
}

int dfx_jit_cache_dir(const char* dir) {
  jit_set_cache_dir(dir ? dir : "");
  return DFX_OK;
}

int dfx_jit_precompile(dfx_ctx* c, int64_t* n_failed) {
  if (!c) return DFX_EINVAL;
  int64_t failed = 0;
  for (auto& kv : c->memo) {
    for (auto& p : kv.second->passes) {
      const int rows = c->analysis_only ? 0 : pick_rows(*c, p);
      const int st_n = staged_streams(p, SIZE_MAX);
      if (!p.jit && !jit_wanted(p, st_n)) continue;
      if (!p.jit) p.jit = request_compiled(p, st_n, rows, true);
      p.jit_checked = true;
      if (jit_state(*p.jit) == 0) jit_wait_idle();
      if (jit_state(*p.jit) < 0) failed += 1;
    }
  }
  if (n_failed) *n_failed = failed;
  return DFX_OK;
}

int dfx_stats_get(dfx_ctx* c, dfx_stats* out) {
  if (!c || !out) return DFX_EINVAL;
  *out = c->stats;
  return DFX_OK;
}

int dfx_stats_reset(dfx_ctx* c) {
  if (!c) return DFX_EINVAL;
  std::memset(&c->stats, 0, sizeof(c->stats));
  c->groups.clear();
  return DFX_OK;
}

int dfx_group_count(dfx_ctx* c, int64_t* n) {
  if (!c || !n) return DFX_EINVAL;
  *n = (int64_t)c->groups.size();
  return DFX_OK;
}

int dfx_group_get(dfx_ctx* c, int64_t i, dfx_group_info* out) {
  if (!c || !out) return DFX_EINVAL;
  if (i < 0 || i >= (int64_t)c->groups.size()) return fail(*c, DFX_ENOTFOUND, "group index out of range");
  *out = c->groups[i];
  return DFX_OK;
}

}  // extern "C"
