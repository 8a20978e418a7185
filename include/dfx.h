/*
 * dfx -- fused execution of task windows over logical arrays on AMD MI355X.
 *
 * The calls follow the statement of the problem in "Composing Distributed
 * Computations Through Task and Kernel Fusion" (Yadav et al., ASPLOS 2025):
 *
 *   - stores, projection functions, partitions, privileges and index tasks
 *     are the IR of section 3 (the syntax figure of section 3, data model in
 *     section 3.1, computational model in section 3.2);
 *   - submitted tasks are buffered in a task window and a fusible prefix is
 *     found with the four fusion constraints of section 4.2;
 *   - stores made temporary by fusion (section 5.1) get no device memory;
 *     application references are counted separately from references held by
 *     pending tasks (split reference counts, section 5.1);
 *   - analysis and the executable plan are memoised on the canonical form of
 *     the window (section 5.2);
 *   - flush and release are the `flush_window` and `del` of section 5.1.
 *
 * Conventions
 *   Every call returns int: DFX_OK (0) or a negative DFX_E* code; the text of
 *   the last error is available from dfx_last_error(ctx).  A rejected call
 *   changes nothing (a rejected submit leaves the window as it was).  A
 *   context is used from one host thread at a time.  Host buffers passed in
 *   remain owned by the caller and are copied before the call returns, with
 *   one exception: the CSR arrays of a serving request are borrowed until
 *   the request leaves the QUEUED state (dfx_csr_desc).
 *   Device memory of stores is owned by the library (allocated through the
 *   configured callbacks, default a stream-ordered hipMallocAsync pool),
 *   except for stores made with dfx_store_wrap, whose memory is borrowed and
 *   never freed.  Handles are never reused within a context.
 */
#ifndef DFX_H
#define DFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DFX_MAX_DIM 4

enum {
  DFX_OK = 0,
  DFX_EINVAL = -1,        /* malformed call, illegal task, shape/partition mismatch */
  DFX_ENOMEM = -2,        /* device or host allocation failed */
  DFX_EHIP = -3,          /* a HIP runtime call failed */
  DFX_ESTATE = -4,        /* call not valid in the current state (e.g. values in an analysis-only context) */
  DFX_ENOMEM_BUDGET = -5, /* a serving request can never fit the HBM budget */
  DFX_EBREAKDOWN = -6,    /* CG breakdown (p.q <= 0 or non-finite) */
  DFX_EMAXITER = -7,      /* iteration limit reached before the tolerance */
  DFX_ENOTFOUND = -8,     /* unknown handle or ticket */
  DFX_EUNSUPPORTED = -9   /* legal in the IR but not executable by this library */
};

typedef int64_t dfx_store;   /* store handle (section 3.1: Store(id, shape)) */
typedef int32_t dfx_part;    /* interned partition handle */
typedef int32_t dfx_proj;    /* interned projection-function handle */
typedef struct dfx_ctx dfx_ctx;

typedef enum { DFX_F32 = 0, DFX_F64 = 1, DFX_I32 = 2, DFX_I64 = 3 } dfx_dtype;

/* Privileges of section 3.2: read, write, read-write, reduce (one operator, +). */
typedef enum { DFX_R = 1, DFX_W = 2, DFX_RW = 3, DFX_RD = 4 } dfx_priv;

/*
 * Operation table.  Each op lists its arguments in order with the privilege
 * each must carry; k is imm[0].  All floating arguments of one task share one
 * dtype (F32 or F64); arithmetic is in that dtype with IEEE rounding of every
 * operation (no contraction into fused multiply-adds).
 *   unary  (a R, out W):     NEG ABS SQRT EXP LOG ERF SQUARE(a*a) COPY
 *   binary (a R, b R, out W): ADD SUB MUL DIV POW MAX MIN
 *   immediate (a R, out W):  ADD_IMM a+k  SUB_IMM a-k  RSUB_IMM k-a
 *                            MUL_IMM a*k  DIV_IMM a/k  RDIV_IMM k/a
 *   FILL (out W):            out = k
 *   AXPY (alpha R, x R, y RW): y = y + alpha*x if k >= 0, y = y - alpha*x if k < 0
 *   SUM   (x R, s Rd)        s = s + sum(x)          (s = sum(x) if k != 0)
 *   SUMSQ (x R, s Rd)        s = s + sum(x*x)        (init flag as SUM)
 *   DOT   (x R, y R, s Rd)   s = s + sum(x*y)        (init flag as SUM)
 *   SPMV_CSR (rowptr R, col R, val R, x R, y W): y = A x for the rows of y's
 *            sub-store; rowptr/col are I32, val/x/y floating; each row is
 *            summed sequentially in CSR order.
 * Reductions produce a 0-d store through the None partition with privilege
 * Rd.  The sum's rounding order is a fixed tree determined only by the
 * element index (so fused and unfused execution agree bit for bit).
 */
typedef enum {
  DFX_OP_NEG = 1, DFX_OP_ABS, DFX_OP_SQRT, DFX_OP_EXP, DFX_OP_LOG, DFX_OP_ERF,
  DFX_OP_SQUARE, DFX_OP_COPY,
  DFX_OP_ADD = 16, DFX_OP_SUB, DFX_OP_MUL, DFX_OP_DIV, DFX_OP_POW, DFX_OP_MAX, DFX_OP_MIN,
  DFX_OP_ADD_IMM = 32, DFX_OP_SUB_IMM, DFX_OP_RSUB_IMM, DFX_OP_MUL_IMM, DFX_OP_DIV_IMM,
  DFX_OP_RDIV_IMM,
  DFX_OP_FILL = 48, DFX_OP_AXPY,
  DFX_OP_SUM = 64, DFX_OP_SUMSQ, DFX_OP_DOT,
  DFX_OP_SPMV_CSR = 80
} dfx_op;

/* Device allocation callbacks: return NULL on failure.  `stream` is the
 * context's hipStream_t; frees are stream-ordered. */
typedef void* (*dfx_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*dfx_free_fn)(void* ptr, size_t bytes, void* stream, void* user);

typedef struct {
  int32_t device;        /* HIP device ordinal; -1 = analysis-only context (no GPU, no values) */
  void* stream;          /* hipStream_t all work is ordered on (NULL: the null stream) */
  dfx_alloc_fn alloc;    /* NULL: hipMallocAsync on `stream` */
  dfx_free_fn dealloc;   /* NULL: hipFreeAsync on `stream` */
  void* alloc_user;
  int32_t window_size;   /* tasks buffered before analysis runs (>= 1) */
  int32_t fuse;          /* 0: unfused baseline, one task per launch, every store materialised */
  int32_t memo;          /* 1: memoise analysis and plan on the window's canonical form */
  int32_t tune;          /* 1: a memoised pass times tiles-per-wave candidates (1x, 2x, 4x the
                            default) on its first 7 executions and keeps the fastest (a
                            candidate must beat the default by 3 %).  Results do not depend on
                            the choice: every candidate keeps each block's tiles an aligned
                            subtree of the reduction tree. */
  int32_t auto_window;   /* 0: the window holds window_size tasks.  > 0: automatic window
                            sizing (the evaluation's choice of window sizes): when a full
                            window fuses as a whole, it is not dispatched; its size doubles,
                            up to auto_window (>= window_size, else EINVAL), and the tasks
                            stay buffered.  Once a full window does not fuse as a whole, the
                            size stays.  Flushes are not affected.  Needs fuse = 1. */
  int32_t jit;           /* compiled passes (section 6's JIT code generation): 0 off, every
                            pass interpreted.  1: a pass's first execution queues its kernel
                            for compilation on a background thread; it runs interpreted until
                            the kernel is ready, then compiled.  2: the first execution
                            compiles it in the caller.  Needs memo = 1 (else EINVAL).  A
                            compiled pass returns the same bits as the interpreted one.
                            The environment variable DFX_JIT=1 or 2 sets it for contexts
                            created with jit = 0 and memo = 1. */
  int32_t reserved[6];
} dfx_config;

typedef struct {
  dfx_store store;
  dfx_part part;
  int32_t priv;          /* dfx_priv */
} dfx_arg;

/* IndexTask(domain, [(S, P, Pr)]) of section 3.2; ndim = 0 is a single task. */
typedef struct {
  uint32_t op;           /* dfx_op */
  int32_t ndim;          /* launch-domain rank, 0..DFX_MAX_DIM */
  const int64_t* launch; /* launch-domain extents (ndim entries, each >= 1) */
  int32_t nargs;
  const dfx_arg* args;
  int32_t nimm;
  const double* imm;
} dfx_task;

typedef struct {
  int64_t tasks_submitted;
  int64_t tasks_dispatched;
  int64_t groups_dispatched;     /* fused tasks issued (one per analysed prefix) */
  int64_t launches;              /* kernel launches (graph replays count their nodes) */
  int64_t temporaries_eliminated;
  int64_t memo_hits;
  int64_t memo_misses;
  int64_t graph_replays;
  int64_t alg_bytes;             /* algorithmic HBM bytes of everything launched */
  double analysis_seconds;       /* host time in analysis + lowering (misses only) */
  int64_t compiled_launches;     /* pass launches that ran a compiled kernel */
} dfx_stats;

#define DFX_INFO_MAX 64
typedef struct {
  int64_t first_task;            /* sequence number (0-based) of the group's first task */
  int32_t prefix_len;            /* tasks fused into this group */
  int32_t memo_hit;
  int32_t n_passes;              /* kernel launches for the group */
  int32_t pass_kind[8];          /* 0 elementwise/reduction, 1 SpMV, 2 single task */
  int32_t n_temporaries;
  dfx_store temporaries[DFX_INFO_MAX];
  int64_t alg_bytes;             /* algorithmic bytes of the group's launches */
} dfx_group_info;

/* ---- context ---------------------------------------------------------- */
/* Section 4 (task window) and the configuration above.  Destroy flushes. */
int dfx_create(const dfx_config* cfg, dfx_ctx** out);
int dfx_destroy(dfx_ctx* ctx);
const char* dfx_last_error(dfx_ctx* ctx);
const char* dfx_version(void);

/* ---- stores (section 3.1) --------------------------------------------- */
/* Create a store of the given shape (ndim 0 = scalar).  Memory is allocated
 * lazily, when a dispatched task first writes it or on dfx_store_write; the
 * application reference count starts at 1. */
int dfx_store_create(dfx_ctx* ctx, int32_t ndim, const int64_t* shape, int32_t dtype,
                     dfx_store* out);
/* Borrow C-contiguous device memory `dptr` as a store (never freed). */
int dfx_store_wrap(dfx_ctx* ctx, void* dptr, int32_t ndim, const int64_t* shape,
                   int32_t dtype, dfx_store* out);
/* Copy `bytes` (= the store's full size) from host memory into the store.
 * Flushes the window first. */
int dfx_store_write(dfx_ctx* ctx, dfx_store s, const void* host, size_t bytes);
/* Flush, synchronise, copy the whole store to host memory. */
int dfx_store_read(dfx_ctx* ctx, dfx_store s, void* host, size_t bytes);
/* Flush and return the store's device address (allocating it if needed). */
int dfx_store_device_ptr(dfx_ctx* ctx, dfx_store s, void** dptr);
/* Drop the application's reference (Python `del`, section 5.1). */
int dfx_store_release(dfx_ctx* ctx, dfx_store s);

/* ---- projections and partitions (section 3.1) -------------------------- */
int dfx_proj_identity(dfx_ctx* ctx, int32_t ndim, dfx_proj* out);
/* Point -> Point keeping the launch dims whose bits are set in keep_mask, in
 * increasing order (e.g. ndim_in=2, mask=0b10 maps (i, j) to (j)). */
int dfx_proj_drop(dfx_ctx* ctx, int32_t ndim_in, uint32_t keep_mask, dfx_proj* out);
/* None: every point maps to the whole store (replication). */
int dfx_part_none(dfx_ctx* ctx, dfx_part* out);
/* Tiling(tile, offset, proj): point p maps to [proj(p)*tile, proj(p+1)*tile) + offset
 * (the sub-store-bounds formula of section 3.1); ndim is the store's rank. */
int dfx_part_tiling(dfx_ctx* ctx, int32_t ndim, const int64_t* tile, const int64_t* offset,
                    dfx_proj proj, dfx_part* out);
/* Image(src, src_part): the entries named by the coordinates stored in
 * src[src_part, p] (the gathered operand of a sparse product).  Never equal
 * to a None or Tiling partition. */
int dfx_part_image(dfx_ctx* ctx, dfx_store src, dfx_part src_part, dfx_part* out);

/* ---- tasks ------------------------------------------------------------ */
/* Validate and append an index task to the window; when the window holds
 * window_size tasks, analyse it and dispatch its longest fusible prefix. */
int dfx_submit(dfx_ctx* ctx, const dfx_task* task);
/* Analyse and dispatch until the window is empty (flush_window, section 5.1). */
int dfx_flush(dfx_ctx* ctx);
/* Flush and wait for all dispatched work. */
int dfx_sync(dfx_ctx* ctx);

/* Allocation-free flush, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same analysis and dispatch as dfx_flush, but:
 *   - the block sums of every reduction go to a fixed array in the library's
 *     device memory (one per device, set up by dfx_create, kept until the
 *     process ends), not to the plan's workspace: at most 16384 blocks per
 *     pass with a reduction (a pass over about 2^26 FP64 elements uses
 *     4096); a larger pass gives DFX_EUNSUPPORTED;
 *   - a group that would need device memory (a store's first allocation,
 *     e.g. the output of a task never run before) is not launched:
 *     DFX_ESTATE, and that group and the rest stay in the window (groups
 *     dispatched before it stay dispatched);
 *   - device frees that retiring stores would make are deferred to the next
 *     dfx_flush, dfx_submit that dispatches, or dfx_destroy.
 * No hipMalloc, hipFree or allocation callback is called.  Host-side
 * analysis of a window not seen before still uses the C++ heap.  Every
 * context on one device shares the array and each call overwrites it:
 * allocation-free flushes that overlap on one device (different streams or
 * threads) race.  Nothing in the array needs clearing: every block sum is
 * written before it is read. */
int dfx_flush_noalloc(dfx_ctx* ctx);

/* ---- whole-region graphs ----------------------------------------------- */
/* Flush, then record every launch dispatched until dfx_graph_end into one
 * hipGraph.  No store may need new memory while recording (DFX_ESTATE). */
int dfx_graph_begin(dfx_ctx* ctx);
int dfx_graph_end(dfx_ctx* ctx, int32_t* graph_id);
/* Replay a recorded region on the context's stream (same stores, same order). */
int dfx_graph_launch(dfx_ctx* ctx, int32_t graph_id);
int dfx_graph_destroy(dfx_ctx* ctx, int32_t graph_id);

/* ---- introspection ---------------------------------------------------- */
int dfx_stats_get(dfx_ctx* ctx, dfx_stats* out);
int dfx_stats_reset(dfx_ctx* ctx);
/* On-disk plan cache (the paper's stated future work: reuse analysis and
 * lowering across runs).  save writes every memoised plan with its
 * canonical key (partitions encoded by structure, stores by first
 * appearance, so a key means the same in every context); load adds the
 * file's plans to the memo table (keys already present are kept) and
 * reports how many it added.  The file is bound to the library build that
 * wrote it: another build's file, a wrong magic, a checksum mismatch or a
 * truncated body is rejected with DFX_EINVAL and nothing is added; a
 * missing file gives DFX_ENOTFOUND.  load needs memo = 1 and fuse = 1
 * (DFX_ESTATE) and is refused while a graph is being recorded (DFX_ESTATE).
 * Loaded plans get their device workspaces at load, so a graph can be
 * recorded from them with no eager run first.  A pass saved while its
 * launch shape was being tuned is
 * stored with the default shape.  The file is trusted input: it is meant to
 * be one that dfx_plan_cache_save wrote. */
int dfx_plan_cache_save(dfx_ctx* ctx, const char* path, int64_t* n_saved);
int dfx_plan_cache_load(dfx_ctx* ctx, const char* path, int64_t* n_loaded);
/* ---- compiled passes (jit = 1 or 2) ----------------------------------- */
/* Section 6 generates and JIT-compiles a kernel per fused task.  Here a
 * memoised pass's op list is written out as the body of the op-list kernel
 * template (one call per instruction, its fields as constants) and compiled
 * with hiprtc for gfx950; tiling, loads, stores and the reduction tree are
 * the template's, so the bits do not change.  Kernels are shared by every
 * context of the process (keyed by their instantiation and source text) and, when a cache
 * directory is set (dfx_jit_cache_dir or the DFX_JIT_CACHE environment
 * variable), stored there as code objects and reused by later processes.
 * A kernel that fails to compile or load leaves its pass interpreted.
 * Which passes run compiled (measured on MI355X): those with transcendental
 * ops, those of fewer than 1024 tiles (latency-bound) and stencil-staged ones;
 * large arithmetic and SpMV passes stream as fast interpreted and stay so.
 * DFX_JIT_ALL=1 compiles every pass. */
typedef struct {
  int64_t compiled;              /* kernels compiled by this process */
  int64_t failed;                /* kernels that failed to compile */
  int64_t disk_hits;             /* kernels read from the cache directory */
  int32_t pending;               /* queued or compiling */
  int32_t reserved;
  double compile_seconds;        /* time spent compiling (disk hits excluded) */
} dfx_jit_info;
/* Blocks until no compilation is queued or running (process-wide). */
int dfx_jit_wait(void);
int dfx_jit_info_get(dfx_jit_info* out);
/* Directory for code objects ("" or NULL: no disk cache).  The directory
 * must exist; files are named by a hash of the kernel source, the embedded
 * headers, the compile options and the hiprtc version. */
int dfx_jit_cache_dir(const char* dir);
/* Compiles, in the caller, the kernel of every pass of every memoised plan
 * of the context that would run compiled and has none yet (also in an
 * analysis-only context, which compiles without loading); *n_failed counts
 * those that failed. */
int dfx_jit_precompile(dfx_ctx* ctx, int64_t* n_failed);

/* Current window size: window_size, or what automatic sizing has grown it to. */
int dfx_window_size(dfx_ctx* ctx, int32_t* out);
/* Number of groups recorded since the last reset, and the i-th one. */
int dfx_group_count(dfx_ctx* ctx, int64_t* n);
int dfx_group_get(dfx_ctx* ctx, int64_t i, dfx_group_info* out);


/* ---- batched persistent execution of independent task streams ---------- */
/* Not in the paper (the executor's batching): many independent task streams
 * of uneven sizes run in one persistent launch.  A stream is what one
 * context dispatches between dfx_batch_record_begin and dfx_batch_record_end:
 * its windows are analysed, fused and lowered as usual (section 4's fused
 * tasks, section 5's temporaries and memoisation), but the passes are kept in
 * the batch instead of launched.  Passes recorded before dfx_batch_loop_begin
 * run once; those after it form a body repeated up to max_iter times, which
 * stops early once *conv_a <= tol * *conv_b (two 0-d FP64 stores of the
 * context, compared in FP64 after each repetition; conv_a = conv_b = 0: no
 * test).  dfx_batch_run launches one persistent kernel over every stream:
 * waves claim (stream, pass, tile run) work items from per-stream claim
 * counters, and the wave that completes a pass's last run reduces its tile
 * sums with the same canonical tree as the ordinary path and advances the
 * stream; no wave waits on another.  Every result is therefore bit-identical
 * to the same stream run through dfx_flush.
 * Limits: FP64 passes of at most 8 live values and 6 input streams (tiers
 * with more registers or pow give DFX_EUNSUPPORTED at record_end) and at most
 * 4096 x 64 tiles per pass.  Streams of one batch run concurrently: no
 * stream may write memory another stream reads or writes.  The stores a
 * stream uses must stay alive (not released by every reference) until the
 * batch is destroyed; the batch keeps device addresses, not references.
 * Recording is exclusive: one context at a time (DFX_ESTATE otherwise).
 * dfx_batch_run synchronises the device first (the recording contexts' work
 * is complete before the launch), then launches asynchronously on the
 * batch's stream.  restart != 0 starts every stream from its first pass;
 * restart = 0 resumes streams paused by round_limit (> 0: a stream pauses
 * after that many body repetitions in one launch) and leaves finished ones.
 * dfx_batch_wait synchronises and reads the stream states back; it returns
 * DFX_EHIP if the kernel's stall detector ended the launch (no pass of any
 * stream completed for several seconds).  Errors: dfx_batch_last_error. */
typedef struct dfx_batch dfx_batch;
enum { DFX_BATCH_RUNNING = 0, DFX_BATCH_DONE = 1, DFX_BATCH_PAUSED = 2 };
int dfx_batch_create(int32_t device, void* stream, dfx_batch** out);
int dfx_batch_destroy(dfx_batch* b);
const char* dfx_batch_last_error(dfx_batch* b);
int dfx_batch_record_begin(dfx_batch* b, dfx_ctx* ctx);
int dfx_batch_loop_begin(dfx_batch* b, dfx_ctx* ctx);
int dfx_batch_record_end(dfx_batch* b, dfx_ctx* ctx, int32_t max_iter, dfx_store conv_a, dfx_store conv_b,
                         double tol, int32_t* stream_id);
int dfx_batch_run(dfx_batch* b, int32_t round_limit, int32_t restart);
int dfx_batch_wait(dfx_batch* b);
/* After dfx_batch_wait: body repetitions completed and DFX_BATCH_* status. */
int dfx_batch_stream_info(dfx_batch* b, int32_t stream_id, int32_t* iterations, int32_t* status);
int dfx_batch_counts(dfx_batch* b, int32_t* n_streams, int32_t* n_passes, int32_t* grid);

/* ---- serving: continuous batching of independent CG solves -------------- */
/* Not in the paper: a request loop over the same arithmetic.  A scheduler
 * thread admits queued solves while a slot is free and their HBM footprint
 * fits `hbm_budget`, runs one CG iteration per round for every resident solve
 * in shared launches (work items = (solve, canonical tile)), and retires
 * solves that reach sqrt(rho_k) <= tol * ||b|| (or max_iter, or breakdown).
 * Solves arriving while others run join at the next round.  A solve's
 * arithmetic depends only on its own data, so its result is bit-identical
 * alone and in any mix.  submit/poll/wait/read_x/release/stats are
 * thread-safe with respect to the scheduler.  Matrices are FP64 CSR with I32
 * indices; x0 = 0. */
enum {
  DFX_SOLVE_QUEUED = 0,
  DFX_SOLVE_RUNNING = 1,
  DFX_SOLVE_CONVERGED = 2,
  DFX_SOLVE_MAXITER = 3,
  DFX_SOLVE_BREAKDOWN = 4
};

typedef struct {
  uint64_t hbm_budget;   /* bytes resident solves may hold at once */
  int32_t max_slots;     /* solves resident at once */
  int32_t max_iter;      /* iteration limit per solve */
  double tol;            /* relative residual target */
  int32_t iters_per_round;  /* CG iterations per scheduling round, 0 for the default
                               (8); status checks, retirement and admission happen
                               between rounds, and a solve that converges inside a
                               round stops iterating on the device, so results do
                               not depend on it */
  int32_t reserved[7];
} dfx_serve_cfg;

/* Host CSR arrays: validated and referenced (not copied) by submit; they must
 * stay valid, unchanged, until the solve leaves the QUEUED state.  The solve
 * is reported QUEUED until the copies of its arrays to the device have
 * completed, so a status of RUNNING or later means they may be freed. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t* rowptr;  /* n+1 entries, rowptr[0] = 0, rowptr[n] = nnz */
  const int32_t* col;     /* nnz entries in [0, n) */
  const double* val;      /* nnz entries */
} dfx_csr_desc;

typedef struct {
  int32_t status;         /* DFX_SOLVE_* */
  int32_t iterations;
  double rel_residual;    /* sqrt(rho)/||b|| of the recursive residual */
  double t_arrive, t_admit, t_done;  /* steady-clock seconds */
} dfx_solve_result;

typedef struct {
  int64_t submitted, admitted, completed, rounds, launches, iterations;
  int64_t row_updates;    /* rows touched per CG phase, summed over rounds */
  uint64_t peak_bytes, resident_bytes;
  int64_t queued;
} dfx_serve_counters;

int dfx_serve_start(dfx_ctx* ctx, const dfx_serve_cfg* cfg);
/* Queue a solve; b (n doubles) is copied.  DFX_ENOMEM_BUDGET if its
 * footprint can never fit, DFX_EINVAL for a malformed CSR. */
int dfx_serve_submit(dfx_ctx* ctx, const dfx_csr_desc* A, const double* b, uint64_t* ticket);
int dfx_serve_poll(dfx_ctx* ctx, uint64_t ticket, dfx_solve_result* out);
/* Block until the solve finishes or timeout_s passes (DFX_ESTATE on timeout). */
int dfx_serve_wait(dfx_ctx* ctx, uint64_t ticket, double timeout_s, dfx_solve_result* out);
int dfx_serve_read_x(dfx_ctx* ctx, uint64_t ticket, double* host, size_t n);
int dfx_serve_release(dfx_ctx* ctx, uint64_t ticket);
int dfx_serve_stats(dfx_ctx* ctx, dfx_serve_counters* out);
/* Finish every queued and resident solve, then stop the scheduler. */
int dfx_serve_stop(dfx_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* DFX_H */
