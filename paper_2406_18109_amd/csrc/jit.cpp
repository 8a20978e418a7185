// Compiled passes: source generation, hiprtc compilation on a background
// thread, the per-process kernel cache and the optional on-disk cache of
// code objects.
#include "jit.h"

#include <hip/hiprtc.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace dfx {

// The kernel headers as they were when the library was built (vm_exec.h and
// what it includes), written into jit_headers.inc by the build: a compiled
// pass always matches the interpreter it replaces.
#include "jit_headers.inc"

int stream_bucket(int n_in, int tier);

namespace {

uint64_t hash_bytes(const char* p, size_t n, uint64_t h = 1469598103934665603ull) {
  for (size_t i = 0; i < n; ++i) {
    h ^= (unsigned char)p[i];
    h *= 1099511628211ull;
  }
  return h;
}

// Device-code options of the library's own kernels that decide rounding and
// code shape: no contraction, IEEE-rounded FP32 divide and sqrt, denormals
// kept, no packed FP32 instructions.
const char* const kOptions[] = {
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-ffp-contract=off",
    "-fno-fast-math",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-fno-gpu-flush-denormals-to-zero",
    "-mllvm",
    "-structurizecfg-skip-uniform-regions=true",
    "-Xclang",
    "-target-feature",
    "-Xclang",
    "-packed-fp32-ops",
};

constexpr int kMaxDev = 64;

}  // namespace

struct JitEntry {
  std::string src, name_expr;
  uint64_t key = 0;
  std::atomic<int> state{0};   // 0 pending, 1 compiled, -1 failed
  std::string log;             // compiler log of a failure
  std::vector<char> code;      // code object
  std::string lowered;         // the entry's symbol in the code object
  std::mutex mu;               // guards mod/fn/load_failed
  hipModule_t mod[kMaxDev] = {};
  hipFunction_t fn[kMaxDev] = {};
  bool load_failed[kMaxDev] = {};
};

namespace {

struct Compiler {
  std::mutex mu;
  std::condition_variable cv, idle_cv;
  std::deque<std::shared_ptr<JitEntry>> queue;
  // by entry and source text: one program can be instantiated for several
  // variants (FP64 and FP32, say), which are different kernels
  std::unordered_map<std::string, std::shared_ptr<JitEntry>> cache;
  std::thread worker;
  bool stop = false;
  int busy = 0;
  JitCounters n;
  std::string disk_dir;
  uint64_t header_hash = 0;

  Compiler() {
    // the disk cache key covers the headers, the options and the compiler
    uint64_t h = hash_bytes("dfxjit", 6);
    for (int i = 0; i < kJitHeaderCount; ++i) {
      h = hash_bytes(kJitHeaderName[i], std::strlen(kJitHeaderName[i]), h);
      h = hash_bytes(kJitHeaderStr[i], std::strlen(kJitHeaderStr[i]), h);
    }
    for (const char* o : kOptions) h = hash_bytes(o, std::strlen(o), h);
    int maj = 0, min = 0;
    (void)hiprtcVersion(&maj, &min);
    const int ver[2] = {maj, min};
    header_hash = hash_bytes((const char*)ver, sizeof(ver), h);
    if (const char* d = std::getenv("DFX_JIT_CACHE")) disk_dir = d;
  }
  ~Compiler() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    if (worker.joinable()) worker.join();
    // code objects stay loaded: modules are not unloaded while the HIP
    // runtime is being torn down at process exit
  }

  void start_worker() {
    if (worker.joinable()) return;
    worker = std::thread([this] {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        cv.wait(lk, [this] { return stop || !queue.empty(); });
        if (stop) return;
        std::shared_ptr<JitEntry> e = queue.front();
        queue.pop_front();
        busy += 1;
        lk.unlock();
        compile(*e);
        lk.lock();
        busy -= 1;
        n.pending = (int32_t)(queue.size() + busy);
        if (queue.empty() && busy == 0) idle_cv.notify_all();
      }
    });
  }

  std::string disk_path(uint64_t key) {
    char name[64];
    std::snprintf(name, sizeof(name), "/dfxjit-%016llx.co", (unsigned long long)key);
    return disk_dir + name;
  }

  // Disk format: magic, key, symbol length + symbol, code length + code,
  // FNV-1a 64 of symbol and code (a damaged file is compiled again).
  bool disk_load(JitEntry& e) {
    std::string dir;
    {
      std::lock_guard<std::mutex> lk(mu);
      dir = disk_dir;
    }
    if (dir.empty()) return false;
    FILE* f = std::fopen(disk_path(e.key).c_str(), "rb");
    if (!f) return false;
    bool ok = false;
    char magic[8];
    uint64_t key = 0, ls = 0, cs = 0;
    if (std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "DFXJIT1", 8) == 0 &&
        std::fread(&key, 8, 1, f) == 1 && key == e.key && std::fread(&ls, 8, 1, f) == 1 && ls < 4096) {
      std::string sym(ls, '\0');
      if (std::fread(&sym[0], 1, ls, f) == ls && std::fread(&cs, 8, 1, f) == 1 && cs > 0 && cs < (1u << 30)) {
        std::vector<char> code(cs);
        uint64_t sum = 0;
        if (std::fread(code.data(), 1, cs, f) == cs && std::fread(&sum, 8, 1, f) == 1 &&
            sum == hash_bytes(code.data(), cs, hash_bytes(sym.data(), sym.size())) && std::fgetc(f) == EOF) {
          e.lowered = sym;
          e.code.swap(code);
          ok = true;
        }
      }
    }
    std::fclose(f);
    return ok;
  }

  void disk_store(const JitEntry& e) {
    std::string dir;
    {
      std::lock_guard<std::mutex> lk(mu);
      dir = disk_dir;
    }
    if (dir.empty()) return;
    const std::string path = disk_path(e.key);
    const std::string tmp = path + ".tmp" + std::to_string((unsigned long long)std::hash<std::thread::id>()(std::this_thread::get_id()));
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    const uint64_t ls = e.lowered.size(), cs = e.code.size();
    const uint64_t sum = hash_bytes(e.code.data(), cs, hash_bytes(e.lowered.data(), ls));
    bool ok = std::fwrite("DFXJIT1", 1, 8, f) == 8 && std::fwrite(&e.key, 8, 1, f) == 1 &&
              std::fwrite(&ls, 8, 1, f) == 1 && std::fwrite(e.lowered.data(), 1, ls, f) == ls &&
              std::fwrite(&cs, 8, 1, f) == 1 && std::fwrite(e.code.data(), 1, cs, f) == cs &&
              std::fwrite(&sum, 8, 1, f) == 1;
    ok = std::fclose(f) == 0 && ok;
    if (ok) ok = std::rename(tmp.c_str(), path.c_str()) == 0;
    if (!ok) std::remove(tmp.c_str());
  }

  void compile(JitEntry& e) {
    if (disk_load(e)) {
      std::lock_guard<std::mutex> lk(mu);
      n.disk_hits += 1;
      e.state.store(1);
      return;
    }
    const auto t0 = std::chrono::steady_clock::now();
    hiprtcProgram prog = nullptr;
    std::string log;
    bool ok = hiprtcCreateProgram(&prog, e.src.c_str(), "dfx_pass.hip", kJitHeaderCount,
                                  const_cast<const char**>(kJitHeaderStr),
                                  const_cast<const char**>(kJitHeaderName)) == HIPRTC_SUCCESS;
    if (ok) ok = hiprtcAddNameExpression(prog, e.name_expr.c_str()) == HIPRTC_SUCCESS;
    if (ok) {
      const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(kOptions) / sizeof(kOptions[0])),
                                                   const_cast<const char**>(kOptions));
      size_t ls = 0;
      if (hiprtcGetProgramLogSize(prog, &ls) == HIPRTC_SUCCESS && ls > 1) {
        log.assign(ls, '\0');
        (void)hiprtcGetProgramLog(prog, &log[0]);
      }
      ok = r == HIPRTC_SUCCESS;
      if (!ok && log.empty()) log = hiprtcGetErrorString(r);
    }
    if (ok) {
      const char* low = nullptr;
      ok = hiprtcGetLoweredName(prog, e.name_expr.c_str(), &low) == HIPRTC_SUCCESS && low;
      if (ok) e.lowered = low;
      size_t cs = 0;
      ok = ok && hiprtcGetCodeSize(prog, &cs) == HIPRTC_SUCCESS && cs > 0;
      if (ok) {
        e.code.resize(cs);
        ok = hiprtcGetCode(prog, e.code.data()) == HIPRTC_SUCCESS;
      }
    }
    if (prog) (void)hiprtcDestroyProgram(&prog);
    const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (ok) disk_store(e);
    std::lock_guard<std::mutex> lk(mu);
    n.seconds += s;
    if (ok) {
      n.compiled += 1;
      e.state.store(1);
    } else {
      n.failed += 1;
      e.log = log.empty() ? "hiprtc failed" : log;
      e.state.store(-1);
      const char* tr = std::getenv("DFX_TRACE");
      if (tr && tr[0] && tr[0] != '0')
        std::fprintf(stderr, "dfx: compiling %s failed:\n%.4000s\n", e.name_expr.c_str(), e.log.c_str());
    }
  }
};

Compiler& compiler() {
  static Compiler c;
  return c;
}

void put_instr(std::string& s, const VmInstr& I, bool f64) {
  const unsigned op = I.w0 & 0xff, flags = (I.w0 >> 8) & 0xff, slot = (I.w0 >> 16) & 0xff, post = I.w0 >> 24;
  const unsigned d = I.w1 & 0xff, a = (I.w1 >> 8) & 0xff, b = (I.w1 >> 16) & 0xff, c = I.w1 >> 24;
  char buf[256];
  if (f64)
    std::snprintf(buf, sizeof(buf), "    DFX_I(%uu, %uu, %uu, %uu, %uu, %uu, %uu, %uu, 0x%08x%08xull);\n", op, flags, slot,
                  post, d, a, b, c, I.w3, I.w2);
  else
    std::snprintf(buf, sizeof(buf), "    DFX_I(%uu, %uu, %uu, %uu, %uu, %uu, %uu, %uu, 0x%08xu);\n", op, flags, slot, post,
                  d, a, b, c, I.w2);
  s += buf;
}

std::string int_list(const std::vector<int32_t>& v, int n) {
  std::string s = "{";
  for (int i = 0; i < n; ++i) {
    s += std::to_string(i < (int)v.size() ? v[i] : 0);
    if (i + 1 < n) s += ", ";
  }
  return s + "}";
}

}  // namespace

JitVariant jit_variant(int is_f64, int tier, int n_in, int spmv, int st_n, int rows) {
  JitVariant v;
  v.is_f64 = is_f64 ? 1 : 0;
  v.spmv = spmv ? 1 : 0;
  v.nb = stream_bucket(n_in, tier);
  switch (tier) {
    case TIER_ARITH: v.hv = 0; v.nr = VM_NREG_LIGHT; break;
    case TIER_TRANS8: v.hv = 1; v.nr = VM_NREG_LIGHT; break;
    case TIER_TRANS16: v.hv = 1; v.nr = VM_NREG; break;
    default: v.hv = 2; v.nr = VM_NREG; break;
  }
  // as launch_vm / launch_tier: staging takes the wider arithmetic buckets;
  // SpMV steps take one row in every variant
  v.sten = (tier == TIER_ARITH && !spmv && st_n > 0 && v.nb != 2) ? 1 : 0;
  const bool plain = !spmv && !v.sten;
  // transcendental passes: two rows per step in FP64 (Black-Scholes over
  // 2^26 options 0.793 against 0.807 ms with one), one in FP32 (0.361
  // against 0.368 ms with two)
  v.rows = plain ? (tier == TIER_ARITH ? (rows == 1 ? 1 : 0) : (is_f64 ? 2 : 1)) : 0;
  v.waves = spmv ? 4 : 2;
  if (plain) {
    const char* r = std::getenv("DFX_JIT_ROWS");
    if (r && r[0] >= '0' && r[0] <= '2' && !r[1]) v.rows = r[0] - '0';
    const char* w = std::getenv("DFX_JIT_WAVES");
    if (w && w[0] >= '1' && w[0] <= '8' && !w[1]) v.waves = w[0] - '0';
  }
  // transcendental FP32 passes software-pipeline their loads (Black-Scholes
  // FP32: 0.389 against 0.406 ms); FP64 ones do not (0.856 against 0.846 ms)
  const char* pf = std::getenv("DFX_JIT_PF");
  v.heavy_pf = (pf && (pf[0] == '0' || pf[0] == '1') && !pf[1]) ? pf[0] - '0' : (v.hv > 0 && !v.is_f64 ? 1 : 0);
  // parameters reloaded at every step: yes, except in stencil-staged and
  // realigning passes (set in jit_source), whose streaming steps measured
  // faster with them kept live (the 8192^2 Jacobi sweep 0.4443 against
  // 0.4472 ms; Black-Scholes FP64 0.862 against 0.844 ms the other way)
  const char* rl = std::getenv("DFX_JIT_RELOAD");
  v.reload = (rl && (rl[0] == '0' || rl[0] == '1') && !rl[1]) ? rl[0] - '0' : -1;
  return v;
}

std::string jit_source(const JitVariant& v, const JitProgram& g, std::string* name_expr) {
  const bool f64 = v.is_f64 != 0;
  std::string s;
  s += "// One fused pass of the dfx executor, compiled for its op list.\n";
  s += "#include \"vm_exec.h\"\n\nnamespace dfx {\n\nstruct JitPass {\n";
  s += "  static constexpr bool COMPILED = true;\n";
  s += "  static constexpr int WAVES = " + std::to_string(v.waves) + ";\n";
  s += std::string("  static constexpr bool HEAVY_PF = ") + (v.heavy_pf ? "true" : "false") + ";\n";
  s += "  static constexpr int N_IN = " + std::to_string(g.n_in) + ", N_OUT = " + std::to_string(g.n_out) + ";\n";
  bool realigns = false;
  for (int32_t d : g.realign) realigns = realigns || d != 0;
  const bool reload = v.reload >= 0 ? v.reload != 0 : !(v.sten || realigns);
  s += std::string("  static constexpr bool RELOAD = ") + (reload ? "true" : "false") + ";\n";
  s += "  static constexpr int out_reg[VM_MAXOUT] = " + int_list(g.out_reg, VM_MAXOUT) + ";\n";
  s += "  static constexpr int bc_reg[VM_MAXBC] = " + int_list(g.bc_reg, VM_MAXBC) + ";\n";
  s += "  static constexpr int st_on[VM_MAXIN] = " + int_list(g.st_on, VM_MAXIN) + ";\n";
  s += "  static constexpr int st_dr[VM_MAXIN] = " + int_list(g.st_dr, VM_MAXIN) + ";\n";
  s += "  static constexpr int st_dc[VM_MAXIN] = " + int_list(g.st_dc, VM_MAXIN) + ";\n";
  bool any_realign = false;
  for (int32_t d : g.realign) any_realign = any_realign || d != 0;
  s += std::string("  static constexpr bool REALIGN = ") + (any_realign ? "true" : "false") + ";\n";
  s += "  static constexpr int realign[VM_MAXIN] = " + int_list(g.realign, VM_MAXIN) + ";\n";
  s += "  template <typename T, int HV, int NR, int NG, int GS, int E>\n";
  s += "  static __device__ __forceinline__ void run(typename GVec<T, GS>::type (&R0)[NR],\n"
       "                                             typename GVec<T, GS>::type (&R1)[NR],\n"
       "                                             typename GVec<T, GS>::type (&R2)[NR],\n"
       "                                             typename GVec<T, GS>::type (&R3)[NR],\n"
       "                                             VmState<T, NG, GS>& G, const unsigned vmask) {\n";
  s += "#define DFX_I(op, fl, sl, po, d, a, b, c, k) \\\n"
       "    vm_instr<T, HV, NR, NG, GS, E>(R0, R1, R2, R3, G, vmask, op, fl, sl, po, d, a, b, c, __builtin_bit_cast(T, k))\n";
  for (const VmInstr& I : g.code) put_instr(s, I, f64);
  s += "#undef DFX_I\n  }\n};\n\n}  // namespace dfx\n";
  char ne[256];
  std::snprintf(ne, sizeof(ne), "dfx::vm_kernel<%s, %d, %s, %d, %d, %d, %s, dfx::JitPass>", f64 ? "double" : "float",
                v.hv, v.spmv ? "true" : "false", v.nr, v.nb, v.rows, v.sten ? "true" : "false");
  if (name_expr) *name_expr = ne;
  return s;
}

std::shared_ptr<JitEntry> jit_request(const std::string& src, const std::string& name_expr, bool sync) {
  Compiler& C = compiler();
  std::shared_ptr<JitEntry> e;
  {
    std::lock_guard<std::mutex> lk(C.mu);
    const std::string id = name_expr + "\n" + src;
    auto it = C.cache.find(id);
    if (it != C.cache.end()) return it->second;
    e = std::make_shared<JitEntry>();
    e->src = src;
    e->name_expr = name_expr;
    e->key = hash_bytes(id.data(), id.size(), C.header_hash);
    C.cache.emplace(id, e);
    // DFX_JIT_DUMP=<dir>: write each generated source there (inspection)
    if (const char* dump = std::getenv("DFX_JIT_DUMP")) {
      char name[64];
      std::snprintf(name, sizeof(name), "/dfxjit-%016llx.hip", (unsigned long long)e->key);
      if (FILE* f = std::fopen((std::string(dump) + name).c_str(), "w")) {
        std::fprintf(f, "// entry: %s\n%s", name_expr.c_str(), src.c_str());
        std::fclose(f);
      }
    }
    if (!sync) {
      C.queue.push_back(e);
      C.n.pending = (int32_t)(C.queue.size() + C.busy);
      C.start_worker();
    }
  }
  if (sync) C.compile(*e);
  else C.cv.notify_one();
  return e;
}

hipFunction_t jit_function(JitEntry& e, int device, bool may_load) {
  if (e.state.load() != 1 || device < 0 || device >= kMaxDev) return nullptr;
  std::lock_guard<std::mutex> lk(e.mu);
  if (e.fn[device] || e.load_failed[device] || !may_load) return e.fn[device];
  hipModule_t m = nullptr;
  hipFunction_t f = nullptr;
  if (hipModuleLoadData(&m, e.code.data()) != hipSuccess || hipModuleGetFunction(&f, m, e.lowered.c_str()) != hipSuccess) {
    (void)hipGetLastError();
    e.load_failed[device] = true;
    return nullptr;
  }
  e.mod[device] = m;
  e.fn[device] = f;
  return f;
}

int jit_state(const JitEntry& e, std::string* log) {
  const int s = e.state.load();
  if (s < 0 && log) *log = e.log;
  return s;
}

void jit_wait_idle() {
  Compiler& C = compiler();
  std::unique_lock<std::mutex> lk(C.mu);
  C.idle_cv.wait(lk, [&] { return C.queue.empty() && C.busy == 0; });
}

JitCounters jit_counters() {
  Compiler& C = compiler();
  std::lock_guard<std::mutex> lk(C.mu);
  JitCounters n = C.n;
  n.pending = (int32_t)(C.queue.size() + C.busy);
  return n;
}

void jit_set_cache_dir(const std::string& dir) {
  Compiler& C = compiler();
  std::lock_guard<std::mutex> lk(C.mu);
  C.disk_dir = dir;
}

}  // namespace dfx
