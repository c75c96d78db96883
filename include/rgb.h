/*
 * rgb.h - C ABI of the batched two-dimensional LP solver for MI355X (gfx950).
 *
 * Each LP k of a batch is (Eq. (1)-(2), Sec. 2.1 of Charlton, Maddock and
 * Richmond, "Two-Dimensional Batch Linear Programming on the GPU"):
 *
 *     maximize  cx[k]*x + cy[k]*y
 *     subject to ax[i]*x + ay[i]*y <= b[i]   for offsets[k] <= i < offsets[k+1]
 *
 * Solved with Seidel's randomized incremental method (Sec. 2.1) as a batch on
 * the GPU (Sec. 3): constraints are taken in the order given, so the caller
 * supplies them in random order (Sec. 2.1 needs a random order for the
 * expected O(m) cost; the solver itself never shuffles).
 *
 * Result (per LP): x* is the lexicographically smallest maximiser (among the
 * optimal points the one with the smallest x, then the smallest y); the
 * paper's bounding rows x <= M, x >= -M (Sec. 2.1) are taken with M -> infinity.
 *   RGB_OPTIMAL    x*, y* written
 *   RGB_INFEASIBLE no point satisfies every row (x, y = NaN)
 *   RGB_UNBOUNDED  feasible, no lexicographic optimum (x, y = NaN)
 *   RGB_INVALID    a non-finite ax/ay/b/cx/cy in the LP, malformed offsets
 *                  for this LP, or a vertex on the method's path whose
 *                  coordinates exceed the FP32 range (x, y = NaN)
 * A row with ax = ay = 0 means 0 <= b: it empties the LP if b < 0 and is
 * ignored otherwise.  An LP with no rows is RGB_UNBOUNDED.
 *
 * Memory: every buffer argument of the solve calls is DEVICE memory of the
 * context's device, owned by the caller, and must stay valid until the work
 * on `stream` completes.  Layout is CSR-offset SoA:
 *   offsets  int64[num_lps + 1], offsets[0] = 0, non-decreasing,
 *            offsets[num_lps] = num_constraints
 *   ax, ay, b float32[num_constraints]   (rows of LP k are contiguous)
 *   cx, cy    float32[num_lps]
 *   x_out, y_out float32[num_lps], status_out int32[num_lps] (rgb_status_t)
 * Rows are read only inside [0, num_constraints): an LP whose offsets fall
 * outside, decrease, or span more than 2^30 rows gets RGB_INVALID instead of
 * being read.
 *
 * Arithmetic is FP32 on the FP32 inputs, with the decisions that FP32 cannot
 * settle (a row parallel to a violated line, u_left within rounding of
 * u_right, a position beyond the FP32 range) taken in FP64; the statuses are
 * those of a serial FP64 Seidel on the same rows.  Rows are expected to be
 * scaled so that |b_i| / |a_i| and |a_i|^2 stay inside the FP32 normal range.
 *
 * Errors: calls return rgb_err_t synchronously for argument errors and never
 * throw across the ABI.  Launch failures return RGB_ERR_DEVICE; a fault
 * during asynchronous execution surfaces at the caller's next
 * synchronisation.  rgb_ctx_last_error() gives a message for the last error
 * on that context.  A context is not thread-safe: use one per host thread or
 * lock around it.
 */
#ifndef RGB_H_
#define RGB_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RGB_OPTIMAL = 0,
    RGB_INFEASIBLE = 1,
    RGB_UNBOUNDED = 2,
    RGB_INVALID = 3
} rgb_status_t;

typedef enum {
    RGB_OK = 0,
    RGB_ERR_INVALID_ARG = -1,
    RGB_ERR_OOM = -2,
    RGB_ERR_DEVICE = -3,
    RGB_ERR_BUSY = -4,
    RGB_ERR_TOO_LARGE = -5,
    RGB_ERR_NOT_FOUND = -6
} rgb_err_t;

/* Kernel families (Sec. 3).  PLAIN is the one-LP-per-lane form the paper
 * calls NaiveRGB; BATCHED gives each LP a group of lanes that scan its rows
 * and split every 1D LP's work units among themselves;
 * PERSISTENT bins LPs by size class (lanes per LP chosen per class) and
 * runs one persistent launch that deals the bulk of the work round-robin and
 * the tail from a device queue, largest LPs first; BINNED bins the same way
 * and launches one wave per sub-batch of the queue, leaving the balancing
 * to the hardware dispatcher.  POOLED gives each LP a small scan group (4, 8
 * or 16 lanes) and serves the 1D LPs of all LPs of a wave that wait with a
 * violated row in one round, their work units dealt over the whole wave.
 * AUTO = the context's tuning (BINNED unless retuned or set). */
typedef enum {
    RGB_VARIANT_AUTO = 0,
    RGB_VARIANT_PLAIN = 1,
    RGB_VARIANT_BATCHED = 2,
    RGB_VARIANT_PERSISTENT = 3,
    RGB_VARIANT_BINNED = 4,
    RGB_VARIANT_POOLED = 5
} rgb_variant_t;

typedef struct rgb_ctx rgb_ctx_t;

/* Optional per-call settings; pass NULL for defaults.  Zero means "default"
 * for every numeric field. */
typedef struct {
    int32_t variant;        /* rgb_variant_t */
    int32_t lanes_per_lp;   /* BATCHED: lanes per LP, one of 4, 8, 16, 32, 64; POOLED: 4, 8 or 16 */
    int32_t pool_wait;      /* POOLED: a wave keeps scanning until this many eighths (1..8) of its
                               live LPs wait with a violated row; -1 = serve every violation at once */
    int32_t pool_rows;      /* POOLED: rows each lane tests per scan step (1, 2 or 4) */
    int32_t chunk;          /* PERSISTENT: sub-batches taken per queue pop */
    int32_t grid;           /* PERSISTENT: workgroups launched */
    int32_t queue_share;    /* PERSISTENT: share of the sub-batches handed out by the device queue,
                               in 1/1024 (the rest are dealt round-robin); -1 = none */
    int32_t* n_1dlp_out;    /* optional device int32[num_lps]: 1D LPs solved per LP (0 for INVALID LPs) */
    void* ev_begin;         /* optional hipEvent_t recorded on the stream right before the solve kernel */
    void* ev_end;           /* optional hipEvent_t recorded right after it and the FP64 fix-up kernel
                               that follows every solve (binning kernels excluded) */
} rgb_solve_opts_t;

/* A launch configuration: kernel family and shape.  rgb_autotune() fills one
 * by measurement; AUTO solves use the context's current one. */
typedef struct {
    int32_t variant;        /* RGB_VARIANT_PERSISTENT, _BINNED, _BATCHED or _POOLED */
    int32_t log2_lanes[16]; /* PERSISTENT/BINNED: lanes per LP = 2^v (v in 2..6) for size class c,
                               which holds LPs with 2^(c-1) < m <= 2^c rows (class 0: m <= 1,
                               class 15: m > 2^14); v = 8: each LP of the class is solved by a
                               workgroup of 128 lanes (two waves) that keeps the LP's first
                               1,650 rows in LDS (Sec. 3's block-wide work units), before the
                               other classes */
    int32_t batched_lanes;  /* BATCHED: lanes per LP (4, 8, 16, 32 or 64) */
    int32_t queue_share;    /* PERSISTENT: sub-batches handed out by the device queue, in 1/1024 */
    int32_t chunk;          /* PERSISTENT: sub-batches per queue pop (>= 1) */
    int32_t grid;           /* PERSISTENT: workgroups, 0 = all that fit on the device at once */
    int32_t pool_lanes;     /* POOLED: scan lanes per LP (4, 8 or 16) */
    int32_t pool_wait;      /* POOLED: wait threshold in eighths, 0 = serve every violation at once */
    int32_t pool_rows;      /* POOLED: rows each lane tests per scan step (1, 2 or 4) */
    float ms;               /* rgb_autotune: measured time of one solve with this configuration */
} rgb_tuning_t;

/* Version string of the library. */
const char* rgb_version(void);

/* Options of a context; pass NULL for defaults. */
typedef struct {
    const char* tuning_table; /* path of a tuning table written by rgb_autotune (JSON, see there), or
                                 NULL: the context starts with the entry the table holds for its
                                 device, if any, as its AUTO configuration; a missing file or a
                                 table without this device leaves the defaults */
    int32_t reserved[4];      /* zero */
} rgb_ctx_opts_t;

/* Create a context on HIP device `device` (the caller's current device is
 * left unchanged).  *out receives the context.  The table named by
 * opts->tuning_table is read once, here; the context keeps no reference to
 * it.  Errors: INVALID_ARG (bad device, NULL out, a table that cannot be
 * parsed or whose entry for this device is not a valid configuration),
 * DEVICE. */
rgb_err_t rgb_ctx_create(int device, const rgb_ctx_opts_t* opts, rgb_ctx_t** out);

/* Free the context and its workspace.  Waits for no stream: the caller
 * synchronises the streams it used first.  NULL is a no-op. */
rgb_err_t rgb_ctx_destroy(rgb_ctx_t* ctx);

/* Message for the last error on ctx (empty if none; static text if ctx is NULL). */
const char* rgb_ctx_last_error(const rgb_ctx_t* ctx);

/* Solve num_lps LPs (Eq. (1)-(2)); enqueues work on `stream` (a hipStream_t,
 * NULL = the null stream) and returns without waiting.  Layout, ownership and
 * per-LP status as described at the top of this file.  num_lps = 0 is a
 * no-op.  Workspace is taken from the context and grown with hipMalloc when
 * needed (never during stream capture: INVALID_ARG then).  Errors:
 * INVALID_ARG (NULL pointer with num_lps > 0, negative counts, bad option),
 * OOM, DEVICE. */
rgb_err_t rgb_solve_batch(rgb_ctx_t* ctx, int64_t num_lps, int64_t num_constraints,
                          const int64_t* offsets, const float* ax, const float* ay, const float* b,
                          const float* cx, const float* cy, float* x_out, float* y_out,
                          int32_t* status_out, const rgb_solve_opts_t* opts, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as rgb_solve_batch, same arguments, layout, results and errors, but
 * it allocates nothing.  PERSISTENT and BINNED solves keep their binning and
 * queue state in a static device array of the library (about 5 MiB, one
 * copy per device, held until the process ends) instead of a context
 * workspace; the other families need no workspace.  num_lps is limited to
 * 2^20 (1,048,576): larger batches return RGB_ERR_TOO_LARGE before anything
 * is enqueued.  Every call on one device shares that device's array and the
 * binning kernels of each call rewrite all of the state it reads, so
 * back-to-back calls need no clearing; calls whose work overlaps on one
 * device (different streams or host threads without ordering) race on the
 * array and may return wrong results: order them on one stream.  The
 * caller passes every input and output buffer as for rgb_solve_batch.
 * Errors: as rgb_solve_batch (never OOM), TOO_LARGE, and DEVICE if the
 * array's device address could not be obtained when ctx was created. */
rgb_err_t rgb_solve_batch_noalloc(rgb_ctx_t* ctx, int64_t num_lps, int64_t num_constraints,
                                  const int64_t* offsets, const float* ax, const float* ay, const float* b,
                                  const float* cx, const float* cy, float* x_out, float* y_out,
                                  int32_t* status_out, const rgb_solve_opts_t* opts, void* stream);

/* Read or replace the configuration AUTO solves on ctx use.  set validates
 * every field (INVALID_ARG otherwise). */
rgb_err_t rgb_ctx_get_tuning(const rgb_ctx_t* ctx, rgb_tuning_t* out);
rgb_err_t rgb_ctx_set_tuning(rgb_ctx_t* ctx, const rgb_tuning_t* tuning);

/* Choose the fastest configuration for this batch by measurement and make
 * it ctx's AUTO configuration (the paper fixes its block size at compile
 * time, Sec. 5; here the launch shape is measured on the target).  Arguments
 * as rgb_solve_batch (the outputs are overwritten by the trial solves); the
 * kernel families are compared first, then lanes per LP class by class for
 * the class-aware families (classes holding >= 4% of the rows, largest
 * first), then the queue share and chunk of the persistent kernel.  Each
 * candidate is timed `reps` times with HIP events on `stream` (the median
 * counts) until `budget_ms` of wall time is spent.  Blocks until done.
 * *best (may be NULL) receives the winner.
 *
 * table_path (may be NULL): a tuning table, created if missing, into which
 * the result is merged; a later rgb_ctx_create with opts->tuning_table =
 * table_path starts from it without searching.  The table is JSON:
 *   {"format": "rgb-tuning-1", "devices": {"<device name> <gfx arch> <CUs>cu":
 *     {"variant": "binned", "batched_lanes": 16, "queue_share": 128, "chunk": 1,
 *      "grid": 0, "pool_lanes": 4, "pool_wait": 2, "pool_rows": 4, "ms": 1.43,
 *      "classes": {"13": {"log2_lanes": 6}, ...}}}}
 * keyed by device and size class (class c holds LPs with 2^(c-1) < m <= 2^c
 * rows).  The family and scalar knobs are the winner's; "classes" lists the
 * classes whose lanes per LP this or an earlier run measured (this run's
 * replace earlier ones; others are kept).  Entries of other devices are
 * kept.  The file is replaced atomically (written beside it, then renamed).
 * Errors as rgb_solve_batch, and INVALID_ARG when the table cannot be read
 * or written. */
rgb_err_t rgb_autotune(rgb_ctx_t* ctx, int64_t num_lps, int64_t num_constraints, const int64_t* offsets,
                       const float* ax, const float* ay, const float* b, const float* cx, const float* cy,
                       float* x_out, float* y_out, int32_t* status_out, int32_t reps, double budget_ms,
                       const char* table_path, void* stream, rgb_tuning_t* best);

/* A solve captured once as a HIP graph (binning, queue set-up and the solve
 * kernel) and replayed with rgb_plan_launch: same buffers, same launch
 * configuration, no host-side argument work.  The plan owns its workspace,
 * so launches of different plans may overlap; launches of one plan must not
 * (issue them on one stream).  Buffers must stay valid while the plan
 * exists.  The configuration is ctx's at creation time unless opts selects
 * one.  opts->n_1dlp_out and the events are captured too. */
typedef struct rgb_plan rgb_plan_t;
rgb_err_t rgb_plan_create(rgb_ctx_t* ctx, int64_t num_lps, int64_t num_constraints, const int64_t* offsets,
                          const float* ax, const float* ay, const float* b, const float* cx, const float* cy,
                          float* x_out, float* y_out, int32_t* status_out, const rgb_solve_opts_t* opts,
                          rgb_plan_t** out);
rgb_err_t rgb_plan_launch(rgb_plan_t* plan, void* stream);
rgb_err_t rgb_plan_destroy(rgb_plan_t* plan);

/* ---------------------------------------------------------------------------
 * Served mode: continuous batching of LP requests.
 *
 * A server owns a device arena of `hbm_budget` bytes, its own context (with
 * the creating context's tuning), `n_streams` streams and one scheduler
 * thread.  A submitted request is copied once, into pinned host rings
 * (`host_ring_mib`, three quarters for rows at 12 B, a quarter for LPs at
 * 16 B), and queued; the scheduler admits queued requests in arrival order
 * into micro-batches as soon as a stream is free and the arena has room (a
 * request that arrives while others are on the GPU joins the next
 * micro-batch, and micro-batches on different streams overlap on the
 * device), copies each micro-batch's ring spans straight into the arena,
 * solves it with rgb_solve_batch, copies the results back and frees the arena
 * block and the ring space.  Results are exactly those of solving each
 * request alone.  All calls are thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct rgb_server rgb_server_t;

typedef struct {
    uint64_t hbm_budget;           /* device bytes for request data; 0 = 1 GiB */
    int32_t n_streams;             /* micro-batches in flight at once, 1..16; 0 = 4 */
    int32_t max_batch_lps;         /* LPs per micro-batch at most; 0 = 65536 */
    int32_t max_pending;           /* queued, not yet admitted requests; 0 = 65536 */
    int32_t variant;               /* kernel family of the micro-batches; AUTO = the tuning */
    int32_t one_request_per_batch; /* 1: every micro-batch holds a single request (no batching) */
    int32_t host_ring_mib;         /* pinned host memory holding queued requests, MiB; 0 = 256 */
} rgb_server_opts_t;

typedef struct {
    uint64_t submitted, completed, rejected_busy, rejected_too_large;
    uint64_t lps_completed, micro_batches;
    uint64_t arena_bytes_in_use, arena_bytes_peak;
    int32_t pending, in_flight;    /* requests queued / admitted and not yet finished */
} rgb_server_stats_t;

/* Start a server on ctx's device (ctx itself is not used afterwards).  The
 * pinned host rings and staging buffers are written once here, so that the
 * first requests do not pay the first touch of their pages (creation takes
 * about as long as a host memset of host_ring_mib).
 * Errors: INVALID_ARG (bad option), OOM (arena or pinned buffers), DEVICE. */
rgb_err_t rgb_server_create(rgb_ctx_t* ctx, const rgb_server_opts_t* opts, rgb_server_t** out);

/* Queue one request.  Pointers are HOST memory in the layout of
 * rgb_solve_batch and are copied before the call returns.  *ticket receives
 * the request's id.  Errors: INVALID_ARG; TOO_LARGE if the request can never
 * fit (more LPs than max_batch_lps, more bytes than the arena, or more than
 * the host rings hold); BUSY if max_pending requests are already queued or
 * the host rings are full (retry later). */
rgb_err_t rgb_server_submit(rgb_server_t* srv, int64_t num_lps, int64_t num_constraints, const int64_t* offsets,
                            const float* ax, const float* ay, const float* b, const float* cx, const float* cy,
                            uint64_t* ticket);

/* Wait up to wait_ms (-1: forever, 0: just look) for request `ticket`.  When
 * it is done, *done = 1, the results are copied to the HOST arrays x_out,
 * y_out, status_out (num_lps each), *latency_ms (may be NULL) receives the
 * time from submission to completion, and the ticket is released.
 * Otherwise *done = 0.  Errors: NOT_FOUND (unknown or released ticket),
 * DEVICE (the micro-batch of this request failed). */
rgb_err_t rgb_server_poll(rgb_server_t* srv, uint64_t ticket, int32_t wait_ms, float* x_out, float* y_out,
                          int32_t* status_out, double* latency_ms, int32_t* done);

rgb_err_t rgb_server_stats(rgb_server_t* srv, rgb_server_stats_t* out);

/* Stop the scheduler after the admitted micro-batches finish and free
 * everything; requests not yet admitted are dropped.  NULL is a no-op. */
rgb_err_t rgb_server_destroy(rgb_server_t* srv);

/* Solve a batch held in HOST memory and return the results to host memory
 * (the transfer-inclusive path; Sec. 4 counts transfers in its timings).
 * Blocking.  Arguments as rgb_solve_batch, but every pointer is host memory;
 * the offsets must be non-decreasing with offsets[0] >= 0 and
 * offsets[num_lps] <= num_constraints (the batch is cut into chunks of whole
 * LPs of about `chunk_rows` rows, 0 = 8 Mi rows).  Chunks go through three
 * streams so that copies overlap solves; buffers allocated with hipHostMalloc
 * (pinned) are copied by DMA directly, other memory is staged through pinned
 * buffers with a parallel memcpy.  Results are exactly those of
 * rgb_solve_batch on the same data.  opts as for rgb_solve_batch except that
 * n_1dlp_out and the events must be NULL.  *ms_out (may be NULL) receives the
 * wall time of the call.  Errors: INVALID_ARG, OOM, DEVICE. */
rgb_err_t rgb_solve_batch_host(rgb_ctx_t* ctx, int64_t num_lps, int64_t num_constraints, const int64_t* offsets,
                               const float* ax, const float* ay, const float* b, const float* cx, const float* cy,
                               float* x_out, float* y_out, int32_t* status_out, const rgb_solve_opts_t* opts,
                               int64_t chunk_rows, double* ms_out);

/* ---------------------------------------------------------------------------
 * Crowd time step on the device (the collision-avoidance use that motivates
 * the paper, Sec. 1 and 5): every agent's velocity is the optimum of a 2D LP
 * built from its neighbours.
 *
 * rgb_crowd_step, on `stream`, for agents at (px, py) with preferred
 * velocities (gx, gy):
 *   1. bins the agents into square cells of side `cell` over `bounds`;
 *   2. for agent i finds its k_i nearest other agents, exactly, ordered by
 *      the FP32 squared distance (dx*dx + dy*dy) and then by index;
 *   3. writes LP i: for each neighbour j, the half-plane n.v <= (d - radius)/2
 *      with n the unit vector from i towards j and d their distance (n =
 *      (1, 0) when d = 0), then the speed disc |v| <= vmax as n_disc tangent
 *      half-planes (normals at angles 2 pi q / n_disc), all rows ordered by
 *      SplitMix64 keys: row t of agent i at step s gets key
 *      splitmix64_nth(seed, (s << 40) + (i << 8) + t + 1), rows are sorted by
 *      the key's bits 7..63, then by t;
 *   4. solves the LPs (rgb_solve_batch, objective (gx, gy)), writing x* to
 *      (vx, vy) and the status to `status`;
 *   5. sets v = 0 where the LP is not OPTIMAL, moves p += dt v and clamps p
 *      to `bounds`.
 * px, py, gx, gy, vx, vy, status: device arrays of n_agents.  Positions must
 * lie inside `bounds` (the kNN search relies on it; step 5 keeps them there).
 * `step` (0 .. 2^23 - 1) feeds the row-order keys; step = -1 takes it from
 * the crowd's device step counter (0 at creation) and advances the counter,
 * so that a step captured in a HIP graph is a new step on every replay (the
 * step allocates nothing and records no memset).  opts as for
 * rgb_solve_batch without n_1dlp_out or events.  Errors: INVALID_ARG, DEVICE.
 * ------------------------------------------------------------------------- */
typedef struct rgb_crowd rgb_crowd_t;

typedef struct {
    float radius;    /* 0 = 0.3 */
    float vmax;      /* 0 = 1 */
    float dt;        /* 0 = 0.1 */
    float cell;      /* grid cell side; 0 = 2 */
    int32_t n_disc;  /* speed-disc rows, 3..63; 0 = 16 */
    int32_t reserved;
    uint64_t seed;   /* row-order keys */
} rgb_crowd_opts_t;

/* n_agents >= 2; k: HOST int32[n_agents], neighbours per agent, 1..64 and
 * below n_agents; bounds: HOST float[4] = {x0, y0, x1, y1}.  Allocates the
 * device buffers of the step (rows, grid) on ctx's device; ctx must outlive
 * the crowd.  Errors: INVALID_ARG, OOM, DEVICE. */
rgb_err_t rgb_crowd_create(rgb_ctx_t* ctx, int64_t n_agents, const int32_t* k, const float bounds[4],
                           const rgb_crowd_opts_t* opts, rgb_crowd_t** out);
rgb_err_t rgb_crowd_step(rgb_crowd_t* crowd, float* px, float* py, const float* gx, const float* gy, float* vx,
                         float* vy, int32_t* status, int64_t step, const rgb_solve_opts_t* opts, void* stream);
/* Total rows of the crowd's LPs (sum of k_i + n_disc). */
rgb_err_t rgb_crowd_num_rows(const rgb_crowd_t* crowd, int64_t* num_constraints);
/* Copy the LPs built by the last step into DEVICE buffers (offsets:
 * n_agents + 1, rows: rgb_crowd_num_rows), enqueued on `stream`. */
rgb_err_t rgb_crowd_rows(const rgb_crowd_t* crowd, int64_t* offsets, float* ax, float* ay, float* b, void* stream);
rgb_err_t rgb_crowd_destroy(rgb_crowd_t* crowd);

/* ---------------------------------------------------------------------------
 * Reduction microbenchmark (the bound-combining step of Sec. 3).
 *
 * rgb_reduce_bench_run computes out[s] = min(in[s c .. s c + c - 1]) for every
 * segment s of `contention` = c consecutive values, with one of four
 * methods, so their cost can be compared as c grows (c = how many work units
 * meet in one bound).  in: device float[n], out: device float[n / c]; c a
 * power of two in [2, 4096], n a multiple of c.  Enqueued on `stream`;
 * results are the exact minima for every method.  Errors: INVALID_ARG, DEVICE.
 * ------------------------------------------------------------------------- */
typedef enum {
    RGB_REDUCE_LDS_ATOMIC = 0,    /* LDS min per value, the paper's shared-memory atomics */
    RGB_REDUCE_GLOBAL_ATOMIC = 1, /* device-memory min per value */
    RGB_REDUCE_DPP = 2,           /* DPP butterfly in the wave, LDS across the block's waves */
    RGB_REDUCE_SERIAL = 3         /* one lane per segment */
} rgb_reduce_method_t;

rgb_err_t rgb_reduce_bench_run(int32_t method, int32_t contention, int64_t n, const float* in, float* out,
                               void* stream);

/* ---------------------------------------------------------------------------
 * Batched three-dimensional LPs (the method of Sec. 2.1 with n = 3; the paper
 * names higher dimensions as its next step in Sec. 6).
 *
 * LP k: maximize c_k.x over x in R^3 subject to a_i.x <= b_i for its rows
 * offsets[k] <= i < offsets[k+1], and the bounding rows |x_j| <= box of
 * Sec. 2.1 (one box for the batch; the rows are not stored).  The result is
 * the lexicographically smallest maximiser: among the points maximising c.x
 * the one with the smallest x, then y, then z.  Rows are taken in the order
 * given (the caller's random order gives Seidel's expected bound).
 *
 * Layout as rgb_solve_batch, with a third normal component: offsets int64
 * [num_lps + 1]; ax, ay, az, b float [num_constraints]; cx, cy, cz float
 * [num_lps]; outputs x, y, z float and status int32 [num_lps].  All pointers
 * are DEVICE memory owned by the caller.  Status: OPTIMAL; INFEASIBLE (x
 * NaN); UNBOUNDED when the optimum lies on a face of the box (the LP without
 * the box is unbounded, or its optimum lies outside the box), with x the
 * optimum inside the box; INVALID (x NaN) for non-finite rows or objective
 * and offsets that are out of range, decreasing or span more than 2^30 rows.
 * Arithmetic is FP64 on the FP32 inputs.
 *
 * lanes_per_lp: 0 (= 16) or 4, 8, 16, 32, 64 lanes per LP.  ev_begin,
 * ev_end: optional hipEvent_t recorded on `stream` around the kernel.
 * Enqueued on `stream` (0 = null stream) on ctx's device; returns before the
 * solve completes.  Errors (synchronous, nothing enqueued): INVALID_ARG for
 * a null context or pointer, negative sizes, box not positive or above the
 * largest FP32 value (x is written in FP32) or
 * an unsupported lanes_per_lp; TOO_LARGE above 2^31 - 1 LPs; DEVICE when
 * the launch fails.
 * ------------------------------------------------------------------------- */
rgb_err_t rgb_solve3_batch(rgb_ctx_t* ctx, int64_t num_lps, int64_t num_constraints, const int64_t* offsets,
                           const float* ax, const float* ay, const float* az, const float* b, const float* cx,
                           const float* cy, const float* cz, double box, float* x_out, float* y_out, float* z_out,
                           int32_t* status_out, int32_t lanes_per_lp, void* stream, void* ev_begin, void* ev_end);

/* ---------------------------------------------------------------------------
 * Batched LPs in n = 2..5 dimensions (the method of Sec. 2.1 in n
 * dimensions, recursive in the dimension; the paper names higher dimensions
 * as its next step in Sec. 6).
 *
 * LP k: maximize c_k.x over x in R^n subject to a_i.x <= b_i for its rows
 * offsets[k] <= i < offsets[k+1], and the bounding rows |x_j| <= box of
 * Sec. 2.1 (one box for the batch; the rows are not stored).  The result is
 * the lexicographically smallest maximiser: among the points maximising c.x
 * the one with the smallest x_1, then x_2, and so on.  Rows are taken in the
 * order given (the caller's random order gives Seidel's expected bound).
 *
 * Layout (coordinate-major SoA): offsets int64 [num_lps + 1]; a float
 * [dim * num_constraints] with component j of row i at a[j * num_constraints
 * + i]; b float [num_constraints]; c float [dim * num_lps] with component j
 * of LP k's objective at c[j * num_lps + k]; outputs x float [dim * num_lps]
 * (same layout as c) and status int32 [num_lps].  All pointers are DEVICE
 * memory owned by the caller.  Status: OPTIMAL; INFEASIBLE (x NaN);
 * UNBOUNDED when the optimum lies on a face of the box (max_j |x_j| >= box
 * (1 - 1e-9): the LP without the box is unbounded, or its optimum lies
 * outside the box), with x the optimum inside the box; INVALID (x NaN) for
 * non-finite rows or objective and offsets that are out of range, decreasing
 * or span more than 2^30 rows.  Arithmetic is FP64 on the FP32 inputs, with
 * relative tolerances of 1e-11 on row violations and 1e-12 on parallel rows
 * and ties.
 *
 * lanes_per_lp: 0 (= 16, or 8 for dim 5: the measured best) or 4, 8, 16,
 * 32, 64 lanes per LP.  ev_begin, ev_end: optional hipEvent_t recorded on
 * `stream` around the kernel.
 * Enqueued on `stream` (0 = null stream) on ctx's device; returns before the
 * solve completes.  Errors (synchronous, nothing enqueued): INVALID_ARG for
 * a null context or pointer, negative sizes, dim outside 2..5, box not
 * positive or above the largest FP32 value (x is written in FP32) or an
 * unsupported lanes_per_lp; TOO_LARGE above
 * 2^31 - 1 LPs; DEVICE when the launch fails.
 * ------------------------------------------------------------------------- */
rgb_err_t rgb_solven_batch(rgb_ctx_t* ctx, int32_t dim, int64_t num_lps, int64_t num_constraints,
                           const int64_t* offsets, const float* a, const float* b, const float* c, double box,
                           float* x_out, int32_t* status_out, int32_t lanes_per_lp, void* stream, void* ev_begin,
                           void* ev_end);

#ifdef __cplusplus
}
#endif

#endif /* RGB_H_ */
