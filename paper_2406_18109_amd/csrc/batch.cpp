// Host side of the persistent batched executor (batch.h, batch.hip).
//
// A context records into a batch instead of launching: every pass its
// dispatches lower between dfx_batch_record_begin and dfx_batch_record_end
// is kept (its kernel parameters, its reductions' result stores) as one task
// stream of the batch.  dfx_batch_run launches the persistent kernel over
// every recorded stream at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "batch.h"
#include "core.hpp"

namespace dfx {

int launch_batch(const BatchPass* passes, BatchStream* streams, BatchCtl* ctl, int grid, int heavy,
                 hipStream_t stream);
int batch_waves_per_cu(int heavy);

struct BatchRec {
  dfx_batch* b = nullptr;
  size_t pass0 = 0;
  long loop_at = -1;   // first pass of the repeated body, or -1
  int rc = DFX_OK;     // first recording error
  std::string err;
};

}  // namespace dfx

using namespace dfx;

struct dfx_ctx : public dfx::Ctx {};

struct dfx_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  std::vector<BatchPass> passes;
  std::vector<char> pass_heavy;       // the pass needs the transcendental op set
  std::vector<BatchStream> streams;   // host copy: tables, and the state read back by dfx_batch_wait
  std::vector<int64_t> max_tiles;     // per stream
  BatchCtl ctl{};
  BatchPass* d_passes = nullptr;
  BatchStream* d_streams = nullptr;
  BatchCtl* d_ctl = nullptr;
  std::vector<void*> d_tsum;
  size_t up_passes = 0, up_streams = 0;   // table sizes on the device
  int recording = 0;
  bool started = false;
  bool pending = false;   // a launch not yet waited for
  int grid = 0;
  int grid_hv[2] = {0, 0};   // resident blocks of the arithmetic / transcendental kernel
  int n_xcd = 1;          // XCDs (L2 domains) of the device; stream s runs on XCD s % n_xcd
  std::string err;
};

namespace dfx {

static int bfail(dfx_batch* b, int rc, const std::string& m) {
  b->err = m;
  return rc;
}

// Called by run_pass for a context that is recording: keep the pass instead
// of launching it.
int batch_record_pass(Ctx& c, const VmParams& P, const VmFinal& F, int dtype, int tier) {
  BatchRec* r = (BatchRec*)c.batch_rec;
  if (r->rc != DFX_OK) return DFX_OK;   // already failed: report at record_end
  if (dtype != DFX_F64 || (tier != TIER_ARITH && tier != TIER_TRANS8) || P.n_in > 6) {
    r->rc = DFX_EUNSUPPORTED;
    r->err = "batched execution takes FP64 passes of at most 8 registers and 6 input streams";
    return DFX_OK;
  }
  BatchPass B;
  std::memset(&B, 0, sizeof(B));
  B.P = P;
  int64_t tpw = 1;
  while (tpw < VM_MAXTPW && (P.n_tiles + tpw - 1) / tpw > BATCH_MAX_RUNS) tpw *= 2;
  if ((P.n_tiles + tpw - 1) / tpw > BATCH_MAX_RUNS) {
    r->rc = DFX_EUNSUPPORTED;
    r->err = "pass too large for batched execution";
    return DFX_OK;
  }
  B.P.tiles_per_wave = tpw;
  B.P.sp_coop = 0;   // the batch kernel computes SpMV rows per wave
  B.n_runs = (int32_t)((P.n_tiles + tpw - 1) / tpw);
  for (int k = 0; k < VM_MAXRED; ++k) B.P.red_partials[k] = nullptr;
  for (int k = 0; k < F.n_red; ++k) {
    B.init[k] = F.init[k];
    B.result[k] = F.result[k];
  }
  r->b->passes.push_back(B);
  r->b->pass_heavy.push_back(tier == TIER_TRANS8 ? 1 : 0);
  return DFX_OK;
}

// A context destroyed while recording: its stream is abandoned.
void batch_record_drop(Ctx& c) {
  BatchRec* r = (BatchRec*)c.batch_rec;
  c.batch_rec = nullptr;
  if (!r) return;
  r->b->passes.resize(r->pass0);
  r->b->pass_heavy.resize(r->pass0);
  r->b->recording -= 1;
  delete r;
}

}  // namespace dfx

extern "C" {

int dfx_batch_create(int32_t device, void* stream, dfx_batch** out) {
  if (!out) return DFX_EINVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return DFX_EHIP;
  dfx_batch* b = new dfx_batch();
  b->device = device;
  b->stream = (hipStream_t)stream;
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || n_cu <= 0) {
    delete b;
    return DFX_EHIP;
  }
  // every block resident; gfx950 has 32 compute units per XCD, and blocks
  // are dispatched to the XCDs in turn, so each XCD gets grid / n_xcd of them
  b->n_xcd = std::max(1, std::min(BATCH_MAX_XCD, n_cu / 32));
  for (int h = 0; h < 2; ++h)
    b->grid_hv[h] = std::max(b->n_xcd, n_cu * std::max(batch_waves_per_cu(h), 4) / (BLOCK / WAVE));
  b->grid = b->grid_hv[1];
  *out = b;
  return DFX_OK;
}

int dfx_batch_destroy(dfx_batch* b) {
  if (!b) return DFX_EINVAL;
  (void)hipStreamSynchronize(b->stream);
  if (b->d_passes) (void)hipFree(b->d_passes);
  if (b->d_streams) (void)hipFree(b->d_streams);
  if (b->d_ctl) (void)hipFree(b->d_ctl);
  for (void* p : b->d_tsum) (void)hipFree(p);
  delete b;
  return DFX_OK;
}

const char* dfx_batch_last_error(dfx_batch* b) { return b ? b->err.c_str() : "null batch"; }

int dfx_batch_record_begin(dfx_batch* b, dfx_ctx* c) {
  if (!b || !c) return DFX_EINVAL;
  if (c->analysis_only) return bfail(b, DFX_ESTATE, "an analysis-only context cannot record into a batch");
  if (c->batch_rec) return bfail(b, DFX_ESTATE, "the context is already recording");
  if (b->recording) return bfail(b, DFX_ESTATE, "another context is recording into the batch");
  if (c->capturing) return bfail(b, DFX_ESTATE, "the context is recording a graph");
  int rc = dfx_flush(c);
  if (rc) return bfail(b, rc, std::string("flush before recording: ") + dfx_last_error(c));
  BatchRec* r = new BatchRec();
  r->b = b;
  r->pass0 = b->passes.size();
  c->batch_rec = r;
  b->recording += 1;
  return DFX_OK;
}

int dfx_batch_loop_begin(dfx_batch* b, dfx_ctx* c) {
  if (!b || !c) return DFX_EINVAL;
  BatchRec* r = (BatchRec*)c->batch_rec;
  if (!r || r->b != b) return bfail(b, DFX_ESTATE, "the context is not recording into this batch");
  if (r->loop_at >= 0) return bfail(b, DFX_ESTATE, "the repeated body has already begun");
  int rc = dfx_flush(c);
  if (rc) return bfail(b, rc, std::string("flush: ") + dfx_last_error(c));
  r->loop_at = (long)b->passes.size();
  return DFX_OK;
}

static const double* conv_ptr(dfx_ctx* c, dfx_store s) {
  auto it = c->stores.find(s);
  if (it == c->stores.end() || it->second.ndim != 0 || it->second.dtype != DFX_F64 || !it->second.ptr) return nullptr;
  return (const double*)it->second.ptr;
}

int dfx_batch_record_end(dfx_batch* b, dfx_ctx* c, int32_t max_iter, dfx_store conv_a, dfx_store conv_b,
                         double tol, int32_t* stream_id) {
  if (!b || !c) return DFX_EINVAL;
  BatchRec* r = (BatchRec*)c->batch_rec;
  if (!r || r->b != b) return bfail(b, DFX_ESTATE, "the context is not recording into this batch");
  int rc = dfx_flush(c);
  if (rc == DFX_OK && r->rc == DFX_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = DFX_EHIP;
  const double* ca = nullptr;
  const double* cb = nullptr;
  if (rc == DFX_OK && r->rc == DFX_OK && (conv_a > 0 || conv_b > 0)) {
    ca = conv_ptr(c, conv_a);
    cb = conv_ptr(c, conv_b);
    if (!ca || !cb) {
      r->rc = DFX_EINVAL;
      r->err = "convergence operands must be allocated 0-d FP64 stores of the recording context";
    }
  }
  c->batch_rec = nullptr;
  b->recording -= 1;
  if (rc != DFX_OK || r->rc != DFX_OK) {
    b->passes.resize(r->pass0);   // drop what this stream recorded
    b->pass_heavy.resize(r->pass0);
    const std::string m = rc != DFX_OK ? std::string("flush: ") + dfx_last_error(c) : r->err;
    const int e = rc != DFX_OK ? rc : r->rc;
    delete r;
    return bfail(b, e, m);
  }
  BatchStream st;
  std::memset(&st, 0, sizeof(st));
  const size_t end = b->passes.size();
  const size_t body0 = r->loop_at >= 0 ? (size_t)r->loop_at : end;
  st.pass0 = (int32_t)r->pass0;
  st.n_pre = (int32_t)(body0 - r->pass0);
  st.n_body = (int32_t)(end - body0);
  st.max_iter = st.n_body > 0 ? std::max(0, max_iter) : 0;
  st.conv_a = ca;
  st.conv_b = cb;
  st.tol = tol;
  int64_t mt = 1;
  for (size_t i = r->pass0; i < end; ++i) mt = std::max<int64_t>(mt, b->passes[i].P.n_tiles);
  delete r;
  b->streams.push_back(st);
  b->max_tiles.push_back(mt);
  if (stream_id) *stream_id = (int32_t)b->streams.size() - 1;
  return DFX_OK;
}

// Launch every stream.  restart != 0: every stream starts from its first
// pass; 0: streams paused by a round limit resume, finished ones stay done.
int dfx_batch_run(dfx_batch* b, int32_t round_limit, int32_t restart) {
  if (!b) return DFX_EINVAL;
  if (b->recording) return bfail(b, DFX_ESTATE, "a context is still recording into the batch");
  if (hipSetDevice(b->device) != hipSuccess) return bfail(b, DFX_EHIP, "hipSetDevice failed");
  if (b->pending) {
    const int rc = dfx_batch_wait(b);
    if (rc) return rc;
  }
  const size_t ns = b->streams.size();
  if (ns == 0) return DFX_OK;
  // tables: passes are immutable once recorded; stream tables grow
  if (b->up_passes != b->passes.size()) {
    if (b->d_passes) (void)hipFree(b->d_passes);
    b->d_passes = nullptr;
    if (hipMalloc(&b->d_passes, b->passes.size() * sizeof(BatchPass)) != hipSuccess)
      return bfail(b, DFX_ENOMEM, "batch pass table");
    if (hipMemcpy(b->d_passes, b->passes.data(), b->passes.size() * sizeof(BatchPass), hipMemcpyHostToDevice) !=
        hipSuccess)
      return bfail(b, DFX_EHIP, "batch pass table upload");
    b->up_passes = b->passes.size();
  }
  if (b->up_streams != ns) {
    if (b->d_streams) (void)hipFree(b->d_streams);
    b->d_streams = nullptr;
    if (hipMalloc(&b->d_streams, ns * sizeof(BatchStream)) != hipSuccess)
      return bfail(b, DFX_ENOMEM, "batch stream table");
    while (b->d_tsum.size() < ns) {
      const size_t i = b->d_tsum.size();
      const int64_t mt = b->max_tiles[i];
      // tile sums of every reduction slot, then the chunk sums of the tree
      const int64_t elems = (int64_t)VM_MAXRED * mt + 2 * (mt / 256 + 256);
      void* p = nullptr;
      if (hipMalloc(&p, (size_t)elems * sizeof(double)) != hipSuccess) return bfail(b, DFX_ENOMEM, "tile sums");
      b->d_tsum.push_back(p);
      b->streams[i].tsum = (double*)p;
      b->streams[i].tsum_stride = mt;
    }
    b->up_streams = ns;
    restart = 1;   // new streams start from their first pass
  }
  if (!b->d_ctl && hipMalloc(&b->d_ctl, sizeof(BatchCtl)) != hipSuccess) return bfail(b, DFX_ENOMEM, "batch control");
  size_t settled = 0;
  for (auto& st : b->streams) {
    if (restart || !b->started) {
      st.claim = 0;
      st.done = 0;
      st.iters = 0;
      st.status = (st.n_pre == 0 && (st.n_body == 0 || st.max_iter == 0)) ? BS_DONE : BS_RUNNING;
    } else if (st.status == BS_PAUSED) {
      st.status = BS_RUNNING;
      st.claim = (st.claim >> 32) << 32;   // reopen the next pass
    }
    st.round_iters = 0;
    if (st.status != BS_RUNNING) {
      settled += 1;
      st.claim = ((st.claim >> 32) << 32) | 0x80000000ull;   // closed: nothing to claim
    }
  }
  std::memset(&b->ctl, 0, sizeof(b->ctl));
  b->ctl.n_streams = (uint32_t)ns;
  b->ctl.n_xcd = (uint32_t)b->n_xcd;
  b->ctl.round_limit = std::max(0, round_limit);
  for (size_t i = 0; i < ns; ++i) {
    BatchXcd& X = b->ctl.x[i % b->n_xcd];
    X.n_streams += 1;
    if (b->streams[i].status != BS_RUNNING) X.n_settled += 1;
  }
  b->started = true;
  // order after the recording contexts' work (writes of inputs, earlier passes)
  if (hipDeviceSynchronize() != hipSuccess) return bfail(b, DFX_EHIP, "device synchronise before the batch");
  if (hipMemcpy(b->d_streams, b->streams.data(), ns * sizeof(BatchStream), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_ctl, &b->ctl, sizeof(BatchCtl), hipMemcpyHostToDevice) != hipSuccess)
    return bfail(b, DFX_EHIP, "batch state upload");
  if (settled == ns) return DFX_OK;
  const int heavy = std::find(b->pass_heavy.begin(), b->pass_heavy.end(), 1) != b->pass_heavy.end() ? 1 : 0;
  b->grid = b->grid_hv[heavy];
  const int e = launch_batch(b->d_passes, b->d_streams, b->d_ctl, b->grid, heavy, b->stream);
  if (e != 0) return bfail(b, DFX_EHIP, std::string("batch launch: ") + hipGetErrorString((hipError_t)e));
  b->pending = true;
  return DFX_OK;
}

// Wait for the last run and read the streams' states back.
int dfx_batch_wait(dfx_batch* b) {
  if (!b) return DFX_EINVAL;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, DFX_EHIP, "batch run failed");
  if (!b->d_streams || !b->pending) return DFX_OK;
  b->pending = false;
  if (hipMemcpy(b->streams.data(), b->d_streams, b->streams.size() * sizeof(BatchStream), hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(&b->ctl, b->d_ctl, sizeof(BatchCtl), hipMemcpyDeviceToHost) != hipSuccess)
    return bfail(b, DFX_EHIP, "batch state read-back");
  for (int x = 0; x < b->n_xcd; ++x)
    if (b->ctl.x[x].error) {
      std::string m = "batch stopped: no pass completed for a long time (stall detector); XCD ids seen 0x";
      char buf[512];
      std::snprintf(buf, sizeof(buf), "%x; waves per XCD id:", b->ctl.xcc_seen);
      m += buf;
      for (int k = 0; k < 16; ++k) {
        std::snprintf(buf, sizeof(buf), " %u", b->ctl.waves[k]);
        m += buf;
      }
      for (int k = 0; k < b->n_xcd; ++k) {
        std::snprintf(buf, sizeof(buf), "; xcd %d: %u streams, %u settled, %u passes, error %d", k,
                      b->ctl.x[k].n_streams, b->ctl.x[k].n_settled, b->ctl.x[k].progress, b->ctl.x[k].error);
        m += buf;
      }
      return bfail(b, DFX_EHIP, m);
    }
  return DFX_OK;
}

int dfx_batch_stream_info(dfx_batch* b, int32_t stream_id, int32_t* iterations, int32_t* status) {
  if (!b || stream_id < 0 || (size_t)stream_id >= b->streams.size()) return DFX_EINVAL;
  const BatchStream& st = b->streams[stream_id];
  if (iterations) *iterations = st.iters;
  if (status) *status = st.status;
  return DFX_OK;
}

int dfx_batch_counts(dfx_batch* b, int32_t* n_streams, int32_t* n_passes, int32_t* grid) {
  if (!b) return DFX_EINVAL;
  if (n_streams) *n_streams = (int32_t)b->streams.size();
  if (n_passes) *n_passes = (int32_t)b->passes.size();
  if (grid) *grid = b->grid;
  return DFX_OK;
}

}  // extern "C"
