// Continuous-batching CG server.
//
// A scheduler thread owns a HIP stream and a set of device slots.  Each round
// it admits queued solves while a slot is free and their HBM footprint fits
// the budget (matrix and right-hand side copied in, state initialised on
// device), launches the four CG phases once for all resident solves (work
// items = (solve, canonical tile)), reads back the per-solve status words and
// retires converged solves (x copied out, memory returned).  Requests that
// arrive while others run join at the next round, so their work overlaps on
// the device.  Every solve's arithmetic depends only on its own data and the
// fixed tiling, so a result is the same alone and in any mix.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>

#include "core.hpp"
#include "serve.h"

namespace dfx {

int launch_serve_phase(const ServeLaunch& L, hipStream_t stream);

static double wall_now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct ServeReq {
  uint64_t ticket;
  int64_t n, nnz;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  std::vector<double> b;
  size_t footprint;
};

struct ServeSlot {
  bool used = false;
  bool fresh = false;
  uint64_t ticket = 0;
  void* mem = nullptr;
  size_t bytes = 0;
  int64_t n = 0;
  int n_tiles = 0;
};

struct ServeResult {
  int status = DFX_SOLVE_QUEUED;
  int iters = 0;
  double rel = 0, t_arrive = 0, t_admit = 0, t_done = 0;
  std::vector<double> x;
};

// Launch-shape tuner: for each phase and batch-size bucket, time the
// candidate items-per-wave values once each, then keep the fastest.  The
// work-item order inside a wave, and therefore every result, is unchanged.
struct Tuner {
  static constexpr int NC = 4;
  static constexpr int cand[NC] = {1, 2, 4, 8};
  struct Entry { float ms[NC] = {0, 0, 0, 0}; int tried = 0; int best = -1; };
  std::unordered_map<int64_t, Entry> tab;
  int pick(int phase, int64_t n_items, int* trial) {
    int b = 0;
    while ((1ll << b) < n_items) ++b;
    Entry& e = tab[(int64_t)phase * 64 + b];
    if (e.best >= 0) { *trial = -1; return cand[e.best]; }
    *trial = e.tried;
    return cand[e.tried];
  }
  void report(int phase, int64_t n_items, int trial, float ms) {
    int b = 0;
    while ((1ll << b) < n_items) ++b;
    Entry& e = tab[(int64_t)phase * 64 + b];
    if (trial < 0 || trial != e.tried) return;
    e.ms[trial] = ms;
    e.tried += 1;
    if (e.tried == NC) {
      int bi = 0;
      for (int i = 1; i < NC; ++i) if (e.ms[i] < e.ms[bi]) bi = i;
      e.best = bi;
    }
  }
};
constexpr int Tuner::cand[Tuner::NC];

struct Server {
  dfx_serve_cfg cfg{};
  int device = 0;
  hipStream_t stream = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  std::string err;
  std::deque<ServeReq> queue;
  std::vector<ServeSlot> slots;
  std::unordered_map<uint64_t, ServeResult> results;
  uint64_t next_ticket = 1;
  size_t used = 0;
  SolveDev* d_solves = nullptr;
  SolveDev* h_solves = nullptr;     // pinned mirror
  int32_t* d_items = nullptr;       // [slot list | tile list]
  int32_t* h_items = nullptr;       // pinned staging
  int32_t* d_fin = nullptr;         // [new solves | all resident solves], max_slots each
  int32_t* h_fin = nullptr;         // pinned staging
  int n_fresh = 0, n_used = 0;
  size_t item_cap = 0;
  Tuner tuner;
  dfx_serve_counters stats{};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

static int64_t tiles_of(int64_t n) {
  const int64_t rows = (n + 127) / 128;
  return (rows + RED_TH - 1) / RED_TH;
}

static size_t footprint_of(int64_t n, int64_t nnz) {
  // CSR + b, x, r, p, q + tile sums, each block 256-byte aligned
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  return al((n + 1) * 4) + al(nnz * 4) + al(nnz * 8) + 5 * al(n * 8) + al(tiles_of(n) * 8);
}

static void fail_locked(Server& S, const std::string& m) {
  if (S.err.empty()) S.err = m;
}

static bool grow_items(Server& S, size_t need) {
  if (need <= S.item_cap) return true;
  size_t cap = std::max<size_t>(need, S.item_cap * 2 + 1024);
  if (S.d_items) (void)hipFreeAsync(S.d_items, S.stream);
  if (S.h_items) { (void)hipStreamSynchronize(S.stream); (void)hipHostFree(S.h_items); }
  S.d_items = nullptr;
  S.h_items = nullptr;
  if (hipMallocAsync((void**)&S.d_items, cap * 2 * sizeof(int32_t), S.stream) != hipSuccess) return false;
  if (hipHostMalloc((void**)&S.h_items, cap * 2 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) return false;
  S.item_cap = cap;
  return true;
}

static bool admit_one(Server& S, ServeReq& q, int slot) {
  ServeSlot& sl = S.slots[slot];
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  const int64_t n = q.n, nnz = q.nnz;
  char* mem = nullptr;
  if (hipMallocAsync((void**)&mem, q.footprint, S.stream) != hipSuccess) return false;
  char* pcur = mem;
  auto take = [&](size_t bytes) { char* r = pcur; pcur += al(bytes); return r; };
  SolveDev d;
  std::memset(&d, 0, sizeof(d));
  d.rowptr = (const int32_t*)take((n + 1) * 4);
  d.col = (const int32_t*)take(nnz * 4);
  d.val = (const double*)take(nnz * 8);
  d.b = (const double*)take(n * 8);
  d.x = (double*)take(n * 8);
  d.r = (double*)take(n * 8);
  d.p = (double*)take(n * 8);
  d.q = (double*)take(n * 8);
  d.partials = (double*)take(tiles_of(n) * 8);
  d.n = n;
  d.n_tiles = (int32_t)tiles_of(n);
  d.max_iter = S.cfg.max_iter;
  d.tol = S.cfg.tol;
  d.status = SOLVE_INIT;
  bool ok = hipMemcpyAsync((void*)d.rowptr, q.rowptr, (n + 1) * 4, hipMemcpyHostToDevice, S.stream) == hipSuccess &&
            hipMemcpyAsync((void*)d.col, q.col, nnz * 4, hipMemcpyHostToDevice, S.stream) == hipSuccess &&
            hipMemcpyAsync((void*)d.val, q.val, nnz * 8, hipMemcpyHostToDevice, S.stream) == hipSuccess &&
            hipMemcpyAsync((void*)d.b, q.b.data(), n * 8, hipMemcpyHostToDevice, S.stream) == hipSuccess;
  S.h_solves[slot] = d;
  ok = ok && hipMemcpyAsync(S.d_solves + slot, S.h_solves + slot, sizeof(SolveDev), hipMemcpyHostToDevice,
                            S.stream) == hipSuccess;
  if (!ok) return false;
  sl.used = true;
  sl.fresh = true;
  sl.ticket = q.ticket;
  sl.mem = mem;
  sl.bytes = q.footprint;
  sl.n = n;
  sl.n_tiles = d.n_tiles;
  return true;
}

static int run_phase(Server& S, int phase, int64_t n_items, int64_t off) {
  if (n_items == 0) return 0;
  const int max_slots = (int)S.slots.size();
  int trial = -1;
  const int ipw = S.tuner.pick(phase, n_items, &trial);
  ServeLaunch L;
  L.solves = S.d_solves;
  L.item_slot = S.d_items + off;
  L.item_tile = S.d_items + S.item_cap + off;
  L.n_items = n_items;
  L.items_per_wave = ipw;
  L.phase = phase;
  L.fin_slots = phase == PH_INIT ? S.d_fin : S.d_fin + max_slots;
  L.n_fin = phase == PH_INIT ? S.n_fresh : S.n_used;
  const int64_t waves = (n_items + ipw - 1) / ipw;
  int64_t grid = std::max<int64_t>(1, (waves + 3) / 4);
  if (grid > 8) grid = (grid + 7) / 8 * 8;
  L.grid = (int)grid;
  if (trial >= 0) (void)hipEventRecord(S.ev0, S.stream);
  int e = launch_serve_phase(L, S.stream);
  if (e) return e;
  if (trial >= 0) {
    (void)hipEventRecord(S.ev1, S.stream);
    (void)hipEventSynchronize(S.ev1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, S.ev0, S.ev1);
    S.tuner.report(phase, n_items, trial, ms);
  }
  S.stats.launches += 1;
  return 0;
}

static void scheduler(Server* Sp) {
  Server& S = *Sp;
  (void)hipSetDevice(S.device);
  // Requests admitted this round.  Their host arrays (the caller's CSR
  // arrays, the request's copy of b) are sources of copies still in flight
  // on the stream, so each is kept, and reported QUEUED, until the round's
  // synchronisation; only then does its status become RUNNING.
  std::vector<ServeReq> staged;
  for (;;) {
    // ---- admission -------------------------------------------------------------
    bool any_active = false;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      while (!S.queue.empty()) {
        ServeReq& q = S.queue.front();
        int slot = -1;
        for (size_t i = 0; i < S.slots.size(); ++i)
          if (!S.slots[i].used) { slot = (int)i; break; }
        if (slot < 0 || S.used + q.footprint > S.cfg.hbm_budget) break;
        if (!admit_one(S, q, slot)) { fail_locked(S, "admission failed (device memory)"); break; }
        S.used += q.footprint;
        S.results[q.ticket].t_admit = wall_now();
        S.stats.admitted += 1;
        S.stats.peak_bytes = std::max<uint64_t>(S.stats.peak_bytes, S.used);
        staged.push_back(std::move(q));
        S.queue.pop_front();
      }
      for (auto& sl : S.slots) any_active = any_active || sl.used;
      if (!any_active) {
        if (S.stop && S.queue.empty()) break;
        S.cv.wait_for(lk, std::chrono::milliseconds(1));
        continue;
      }
    }
    // ---- one round: init new solves, then the three CG phases for all -------
    size_t n_all = 0, n_new = 0;
    for (auto& sl : S.slots)
      if (sl.used) { n_all += sl.n_tiles; if (sl.fresh) n_new += sl.n_tiles; }
    if (!grow_items(S, n_all + n_new)) { std::lock_guard<std::mutex> lk(S.mu); fail_locked(S, "work list allocation failed"); break; }
    size_t k = 0;
    for (size_t i = 0; i < S.slots.size(); ++i)
      if (S.slots[i].used && S.slots[i].fresh)
        for (int t = 0; t < S.slots[i].n_tiles; ++t) { S.h_items[k] = (int32_t)i; S.h_items[S.item_cap + k] = t; ++k; }
    for (size_t i = 0; i < S.slots.size(); ++i)
      if (S.slots[i].used)
        for (int t = 0; t < S.slots[i].n_tiles; ++t) { S.h_items[k] = (int32_t)i; S.h_items[S.item_cap + k] = t; ++k; }
    const size_t ms = S.slots.size();
    S.n_fresh = S.n_used = 0;
    for (size_t i = 0; i < ms; ++i) {
      if (!S.slots[i].used) continue;
      if (S.slots[i].fresh) S.h_fin[S.n_fresh++] = (int32_t)i;
      S.h_fin[ms + S.n_used++] = (int32_t)i;
    }
    bool ok = hipMemcpyAsync(S.d_items, S.h_items, k * sizeof(int32_t), hipMemcpyHostToDevice, S.stream) == hipSuccess &&
              hipMemcpyAsync(S.d_items + S.item_cap, S.h_items + S.item_cap, k * sizeof(int32_t),
                             hipMemcpyHostToDevice, S.stream) == hipSuccess &&
              hipMemcpyAsync(S.d_fin, S.h_fin, 2 * ms * sizeof(int32_t), hipMemcpyHostToDevice, S.stream) == hipSuccess;
    int e = ok ? 0 : 1;
    if (!e) e = run_phase(S, PH_INIT, (int64_t)n_new, 0);
    // several iterations per round amortise the host round trip; a solve that
    // converges inside the round is skipped by the remaining phases
    const int ipr = S.cfg.iters_per_round > 0 ? S.cfg.iters_per_round : 8;
    for (int j = 0; j < ipr && !e; ++j) {
      e = run_phase(S, PH_SPMV_DOT, (int64_t)n_all, (int64_t)n_new);
      if (!e) e = run_phase(S, PH_AXPY_DOT, (int64_t)n_all, (int64_t)n_new);
      if (!e) e = run_phase(S, PH_UPDATE_P, (int64_t)n_all, (int64_t)n_new);
    }
    // one transfer of every slot's state (unused slots are ignored below)
    if (!e) e = hipMemcpyAsync(S.h_solves, S.d_solves, sizeof(SolveDev) * S.slots.size(), hipMemcpyDeviceToHost, S.stream);
    if (!e) e = hipStreamSynchronize(S.stream);
    if (e) { std::lock_guard<std::mutex> lk(S.mu); fail_locked(S, "round failed: " + std::string(hipGetErrorString((hipError_t)e))); break; }
    {
      // the admission copies have completed: the host arrays are free again
      std::lock_guard<std::mutex> lk(S.mu);
      for (const ServeReq& q : staged) S.results[q.ticket].status = DFX_SOLVE_RUNNING;
    }
    staged.clear();
    S.stats.rounds += 1;
    S.stats.row_updates += (int64_t)ipr * n_all * (int64_t)(RED_TH * 128);
    // ---- retire finished solves ---------------------------------------------------
    for (size_t i = 0; i < S.slots.size(); ++i) {
      ServeSlot& sl = S.slots[i];
      if (!sl.used) continue;
      sl.fresh = false;
      const SolveDev& d = S.h_solves[i];
      if (d.status < SOLVE_CONVERGED) continue;
      std::vector<double> x(sl.n);
      bool cp = hipMemcpyAsync(x.data(), d.x, sl.n * 8, hipMemcpyDeviceToHost, S.stream) == hipSuccess &&
                hipStreamSynchronize(S.stream) == hipSuccess;
      (void)hipFreeAsync(sl.mem, S.stream);
      std::lock_guard<std::mutex> lk(S.mu);
      ServeResult& res = S.results[sl.ticket];
      res.status = d.status == SOLVE_CONVERGED ? DFX_SOLVE_CONVERGED
                 : d.status == SOLVE_MAXITER ? DFX_SOLVE_MAXITER : DFX_SOLVE_BREAKDOWN;
      res.iters = d.iters;
      res.rel = d.bnorm > 0 ? std::sqrt(d.rho) / d.bnorm : 0.0;
      res.t_done = wall_now();
      res.x.swap(x);
      if (!cp) fail_locked(S, "copying a solution back failed");
      S.used -= sl.bytes;
      S.stats.completed += 1;
      S.stats.iterations += d.iters;
      sl = ServeSlot();
    }
    S.cv.notify_all();
  }
  std::lock_guard<std::mutex> lk(S.mu);
  S.cv.notify_all();
}

}  // namespace dfx

using namespace dfx;

struct dfx_ctx : public dfx::Ctx {};

extern "C" {

int dfx_serve_start(dfx_ctx* c, const dfx_serve_cfg* cfg) {
  if (!c || !cfg) return DFX_EINVAL;
  if (c->analysis_only) { c->err = "serving needs a device"; return DFX_ESTATE; }
  if (c->server) { c->err = "server already running"; return DFX_ESTATE; }
  if (cfg->max_slots < 1 || cfg->hbm_budget == 0 || !(cfg->tol > 0) || cfg->max_iter < 1 || cfg->iters_per_round < 0) {
    c->err = "bad serving configuration";
    return DFX_EINVAL;
  }
  Server* S = new Server();
  S->cfg = *cfg;
  S->device = c->cfg.device;
  S->slots.resize(cfg->max_slots);
  bool ok = hipSetDevice(S->device) == hipSuccess &&
            hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) == hipSuccess &&
            hipMalloc((void**)&S->d_solves, sizeof(SolveDev) * cfg->max_slots) == hipSuccess &&
            hipHostMalloc((void**)&S->h_solves, sizeof(SolveDev) * cfg->max_slots, hipHostMallocDefault) == hipSuccess &&
            hipMalloc((void**)&S->d_fin, sizeof(int32_t) * 2 * cfg->max_slots) == hipSuccess &&
            hipHostMalloc((void**)&S->h_fin, sizeof(int32_t) * 2 * cfg->max_slots, hipHostMallocDefault) == hipSuccess &&
            hipEventCreate(&S->ev0) == hipSuccess && hipEventCreate(&S->ev1) == hipSuccess;
  if (!ok) {
    if (S->d_solves) (void)hipFree(S->d_solves);
    if (S->h_solves) (void)hipHostFree(S->h_solves);
    if (S->d_fin) (void)hipFree(S->d_fin);
    if (S->h_fin) (void)hipHostFree(S->h_fin);
    if (S->ev0) (void)hipEventDestroy(S->ev0);
    if (S->ev1) (void)hipEventDestroy(S->ev1);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
    c->err = "serving set-up failed";
    return DFX_EHIP;
  }
  std::memset(S->h_solves, 0, sizeof(SolveDev) * cfg->max_slots);
  c->server = S;
  S->th = std::thread(scheduler, S);
  return DFX_OK;
}

int dfx_serve_submit(dfx_ctx* c, const dfx_csr_desc* A, const double* b, uint64_t* ticket) {
  if (!c || !A || !b || !ticket) return DFX_EINVAL;
  Server* S = (Server*)c->server;
  if (!S) { c->err = "server not running"; return DFX_ESTATE; }
  if (A->n < 1 || A->nnz < 1 || !A->rowptr || !A->col || !A->val) { c->err = "bad CSR descriptor"; return DFX_EINVAL; }
  // structural check on the host: the device kernels trust these bounds
  if (A->rowptr[0] != 0 || A->rowptr[A->n] != A->nnz) { c->err = "rowptr must run from 0 to nnz"; return DFX_EINVAL; }
  for (int64_t i = 0; i < A->n; ++i)
    if (A->rowptr[i + 1] < A->rowptr[i]) { c->err = "rowptr must be non-decreasing"; return DFX_EINVAL; }
  for (int64_t k = 0; k < A->nnz; ++k)
    if (A->col[k] < 0 || A->col[k] >= A->n) { c->err = "column index out of range"; return DFX_EINVAL; }
  if (tiles_of(A->n) > S_MAXTILES) { c->err = "solve too large for the batched executor"; return DFX_EUNSUPPORTED; }
  const size_t fp = footprint_of(A->n, A->nnz);
  std::lock_guard<std::mutex> lk(S->mu);
  if (!S->err.empty()) { c->err = S->err; return DFX_EHIP; }
  if (fp > S->cfg.hbm_budget) { c->err = "solve footprint exceeds the HBM budget"; return DFX_ENOMEM_BUDGET; }
  ServeReq q;
  q.ticket = S->next_ticket++;
  q.n = A->n;
  q.nnz = A->nnz;
  q.rowptr = A->rowptr;
  q.col = A->col;
  q.val = A->val;
  q.b.assign(b, b + A->n);
  q.footprint = fp;
  ServeResult& r = S->results[q.ticket];
  r.status = DFX_SOLVE_QUEUED;
  r.t_arrive = wall_now();
  *ticket = q.ticket;
  S->queue.push_back(std::move(q));
  S->stats.submitted += 1;
  S->cv.notify_all();
  return DFX_OK;
}

static int fill_result(const ServeResult& r, dfx_solve_result* out) {
  out->status = r.status;
  out->iterations = r.iters;
  out->rel_residual = r.rel;
  out->t_arrive = r.t_arrive;
  out->t_admit = r.t_admit;
  out->t_done = r.t_done;
  return DFX_OK;
}

int dfx_serve_poll(dfx_ctx* c, uint64_t ticket, dfx_solve_result* out) {
  if (!c || !out) return DFX_EINVAL;
  Server* S = (Server*)c->server;
  if (!S) { c->err = "server not running"; return DFX_ESTATE; }
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->results.find(ticket);
  if (it == S->results.end()) { c->err = "unknown ticket"; return DFX_ENOTFOUND; }
  return fill_result(it->second, out);
}

int dfx_serve_wait(dfx_ctx* c, uint64_t ticket, double timeout_s, dfx_solve_result* out) {
  if (!c || !out) return DFX_EINVAL;
  Server* S = (Server*)c->server;
  if (!S) { c->err = "server not running"; return DFX_ESTATE; }
  std::unique_lock<std::mutex> lk(S->mu);
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
  for (;;) {
    auto it = S->results.find(ticket);
    if (it == S->results.end()) { c->err = "unknown ticket"; return DFX_ENOTFOUND; }
    if (it->second.status >= DFX_SOLVE_CONVERGED) return fill_result(it->second, out);
    if (!S->err.empty()) { c->err = S->err; return DFX_EHIP; }
    if (S->cv.wait_until(lk, deadline) == std::cv_status::timeout) {
      fill_result(S->results[ticket], out);
      c->err = "timed out";
      return DFX_ESTATE;
    }
  }
}

int dfx_serve_read_x(dfx_ctx* c, uint64_t ticket, double* host, size_t n) {
  if (!c || !host) return DFX_EINVAL;
  Server* S = (Server*)c->server;
  if (!S) { c->err = "server not running"; return DFX_ESTATE; }
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->results.find(ticket);
  if (it == S->results.end()) { c->err = "unknown ticket"; return DFX_ENOTFOUND; }
  if (it->second.status < DFX_SOLVE_CONVERGED) { c->err = "solve not finished"; return DFX_ESTATE; }
  if (it->second.x.size() != n) { c->err = "length differs from the solve's size"; return DFX_EINVAL; }
  std::memcpy(host, it->second.x.data(), n * 8);
  return DFX_OK;
}

int dfx_serve_release(dfx_ctx* c, uint64_t ticket) {
  if (!c) return DFX_EINVAL;
  Server* S = (Server*)c->server;
  if (!S) { c->err = "server not running"; return DFX_ESTATE; }
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->results.find(ticket);
  if (it == S->results.end() || it->second.status < DFX_SOLVE_CONVERGED) { c->err = "unknown or unfinished ticket"; return DFX_ENOTFOUND; }
  S->results.erase(it);
  return DFX_OK;
}

int dfx_serve_stats(dfx_ctx* c, dfx_serve_counters* out) {
  if (!c || !out) return DFX_EINVAL;
  Server* S = (Server*)c->server;
  if (!S) { c->err = "server not running"; return DFX_ESTATE; }
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->stats;
  out->resident_bytes = S->used;
  out->queued = (int64_t)S->queue.size();
  return DFX_OK;
}

int dfx_serve_stop(dfx_ctx* c) {
  if (!c) return DFX_EINVAL;
  Server* S = (Server*)c->server;
  if (!S) return DFX_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  std::string err = S->err;
  (void)hipStreamSynchronize(S->stream);
  if (S->d_items) (void)hipFree(S->d_items);
  if (S->h_items) (void)hipHostFree(S->h_items);
  (void)hipFree(S->d_solves);
  (void)hipHostFree(S->h_solves);
  if (S->d_fin) (void)hipFree(S->d_fin);
  if (S->h_fin) (void)hipHostFree(S->h_fin);
  (void)hipEventDestroy(S->ev0);
  (void)hipEventDestroy(S->ev1);
  (void)hipStreamDestroy(S->stream);
  delete S;
  c->server = nullptr;
  if (!err.empty()) { c->err = err; return DFX_EHIP; }
  return DFX_OK;
}

}  // extern "C"
