// Batched persistent execution: the device tables of one batch.
//
// A batch holds independent task streams, each a list of fused passes that
// were lowered by the ordinary planner and recorded instead of launched:
// passes [pass0, pass0 + n_pre) run once, then [pass0 + n_pre,
// pass0 + n_pre + n_body) repeat up to max_iter times, stopping early when a
// 0-d FP64 value falls to tol times another.  One persistent launch runs every
// stream: each wave repeatedly claims a work item (stream, current pass, tile
// run) of a stream of its XCD and executes it; the wave that finishes a
// pass's last run reduces the pass's tile sums with the canonical tree and
// advances the stream.  No wave waits for another: a wave with nothing to
// claim looks at the XCD's other streams.
#pragma once
#include <stdint.h>

#include "vm.h"

namespace dfx {

constexpr int BATCH_MAX_RUNS = 4096;  // work items per pass (runs of tiles_per_wave tiles)

struct BatchPass {
  VmParams P;                    // red_partials unused: tile sums go to the stream's tsum
  int32_t n_runs;                // ceil(n_tiles / tiles_per_wave)
  int32_t init[VM_MAXRED];       // reduction k starts from zero (else accumulates)
  void* result[VM_MAXRED];       // 0-d FP64 result of reduction k
};

enum BatchStatus : int32_t { BS_RUNNING = 0, BS_DONE = 1, BS_PAUSED = 2 };

struct BatchStream {
  int32_t pass0, n_pre, n_body, max_iter;
  const double* conv_a;          // stop once *conv_a <= tol * *conv_b after a repetition (null: never)
  const double* conv_b;
  double tol;
  double* tsum;                  // tile sums: [VM_MAXRED][tsum_stride], then one chunk-sum row
  int64_t tsum_stride;
  // device state, kept across launches
  unsigned long long claim;      // (passes completed << 32) | next run to claim
  uint32_t done;                 // runs finished of the current pass
  int32_t iters;                 // repetitions of the body completed
  int32_t round_iters;           // repetitions completed in this launch
  int32_t status;                // BatchStatus
};

// Streams are pinned to XCDs: stream s runs on the compute units of XCD
// s % n_xcd, whose L2 is the coherence point of everything the stream's
// waves exchange inside a launch.  Each XCD's counters sit in their own
// 256-byte line.
constexpr int BATCH_MAX_XCD = 8;
struct BatchXcd {
  uint32_t n_streams;            // streams of this XCD
  uint32_t n_settled;            // of them, done or paused in this launch
  uint32_t progress;             // passes completed: the stall detector's clock
  int32_t error;                 // 1: the stall detector fired
  uint32_t pad[60];
};
struct BatchCtl {
  BatchXcd x[BATCH_MAX_XCD];
  uint32_t n_streams, n_xcd;
  int32_t round_limit;           // > 0: a stream pauses after this many repetitions in one launch
  uint32_t xcc_seen;             // bit k: some wave ran on XCD k (diagnostics)
  uint32_t waves[16];            // waves that started, per XCD id (diagnostics)
};

}  // namespace dfx
