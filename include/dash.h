/*
 * dash.h -- C ABI of the MI355X (gfx950) dual-way streaming PARAFAC2 library.
 *
 * The operations follow "Fast and Accurate Dual-Way Streaming PARAFAC2 for
 * Irregular Tensors" (DASH): an irregular tensor {X_k}, slices X_k of shape
 * I_k x J sharing J columns, modelled as X_k ~ U_k S_k V^T with S_k diagonal
 * (row k of W), V shared and U_k free (Sec. 2.1).  Updates bring new rows of
 * existing slices and whole new slices (Problem 1, Sec. 2.2); each update
 * solves Lemma 1 (new rows of U_k), Lemma 2 (S_k) and Lemma 3 (V) under a
 * forgetting factor lambda (Sec. 3.1, eq. [new_loss]) without revisiting old
 * rows (Algorithm 1).
 *
 * Conventions for every call:
 *  - Matrices are dense row-major.  "device" pointers are HIP device memory of
 *    the context's device; "host" pointers are ordinary CPU memory.
 *  - Input buffers are borrowed: the library never frees them.  Device row
 *    buffers handed to dash_ingest_rows / dash_ingest_slices must stay valid and
 *    unmodified until the dash_update (or dash_wait) that consumes them returns.
 *  - Output buffers are owned by the caller and sized from dash_get_dims.
 *  - No call throws; every failure returns a dash_status and leaves a message
 *    for dash_last_error.  A failed call leaves the context unchanged unless its
 *    description says otherwise.
 *  - A context is not thread-safe: serialise calls on one context.  Work is
 *    enqueued on the context's HIP stream.
 */
#ifndef DASH_H
#define DASH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dash_status {
  DASH_OK = 0,
  DASH_E_INVALID_ARG = 1,   /* bad argument; nothing changed                       */
  DASH_E_OUT_OF_MEMORY = 2, /* device or pinned allocation failed                  */
  DASH_E_BAD_STATE = 3,     /* call not allowed in the context's current state     */
  DASH_E_CAPACITY = 4,      /* a capacity fixed at dash_create would be exceeded   */
  DASH_E_NUMERIC = 5,       /* non-finite factors; the update was rolled back      */
  DASH_E_DEVICE = 6,        /* a HIP runtime call failed                           */
  DASH_E_IO = 7             /* checkpoint file could not be read or written        */
} dash_status;

enum { DASH_PREC_FP32 = 0, DASH_PREC_MIXED = 1 };
enum { DASH_STATS_EXACT = 0, DASH_STATS_LAGGED = 1 };

typedef struct dash_config {
  int32_t J;                 /* columns shared by all slices, 1 <= J <= 256              */
  int32_t R;                 /* target rank, 1 <= R <= 32                                */
  double lambda;             /* forgetting factor, 0 < lambda <= 1 (Sec. 3.1)            */
  int32_t n_iter;            /* ALS passes per update; 1 is Algorithm 1                  */
  int32_t init_max_iter;     /* PARAFAC2-ALS iterations of dash_init (paper: 10)         */
  double init_tol;           /* stop when |d loss| <= init_tol * loss                   */
  int32_t precision;         /* DASH_PREC_FP32, or DASH_PREC_MIXED: the new rows' products
                                (Lemma 1's x V (V^T V)^{-1} and U_new^T X_new, U_new^T U_new)
                                on BF16 MFMA with FP32 sums; the running sums Y_k, D_k
                                FP32 plus an FP32 compensation word each, folded in
                                FP64 (twice the state bytes); R x R solves FP64       */
  int32_t stats_mode;        /* DASH_STATS_EXACT: Lemmas 2-3 evaluated exactly from the
                                running sums Y_k = sum lambda^age U^T X, D_k with the
                                current V, S_k (reads every Y_k each pass);
                                DASH_STATS_LAGGED: Algorithm 1's recursions
                                (eq. [obtain_CandC], [obtain_FandF], [obtain_FandG]):
                                c_k, F, G keep the terms of past updates as they were
                                computed, scaled by lambda, so a pass reads only the new
                                rows and each slice's D_k, c_k; the reported fit then
                                evaluates eq. [new_loss] with those F, G                */
  int64_t max_slices;        /* capacity in slices (K never exceeds it)                  */
  int64_t max_rows_per_update;   /* capacity in rows staged for one update               */
  int64_t max_groups_per_update; /* capacity in row groups staged for one update         */
  int64_t max_init_rows;     /* capacity of dash_init's initial tensor (rows)            */
  int32_t device;            /* HIP device ordinal                                       */
  void *stream;              /* hipStream_t to enqueue on; NULL: the library makes a
                                blocking one (ordered after the null stream's work)     */
} dash_config;

typedef struct dash_ctx dash_ctx;

typedef struct dash_update_report {
  int64_t step;      /* 1-based index of the update this report describes           */
  int64_t rows;      /* rows consumed by the update (sum of I_{k,new})              */
  int32_t K;         /* slices after the update                                     */
  int32_t committed; /* 1 if the update's state was committed                       */
  double fit;        /* 1 - sqrt(loss)/sqrt(sum_n) after the update                 */
  double loss;       /* eq. [new_loss] with compounding weights, closed form        */
  double sum_n;      /* sum over slices of the forgetting-weighted squared norms    */
  double device_us;  /* device time of the update: from its first launch starting
                        to its final phase ending (device realtime clock)       */
  /* anomaly scores (dash_anomaly on, else 0), Sec. 3.4 with the threshold of
     Sec. 4.5: */
  double te;            /* tensor-level error (Definition 2): mean over the slices
                           that received rows of their se_k (Definition 1)        */
  double te_threshold;  /* mean + population std of the previous `window` te of
                           this context (+inf while there is none)             */
  int32_t te_anomaly;   /* 1 if te > te_threshold                               */
  int32_t n_anomalies;  /* slices whose se_k exceeded their own moving threshold */
} dash_update_report;

typedef struct dash_init_report {
  int32_t iters;     /* PARAFAC2-ALS iterations run                                 */
  double loss;       /* loss of the initial decomposition                           */
  double fit;
} dash_init_report;

typedef struct dash_dims {
  int32_t J, R;
  int32_t K;           /* committed slices                                           */
  int32_t K_pending;   /* slices including those staged by dash_ingest_slices        */
  int64_t step;        /* committed updates                                          */
  int64_t m_last;      /* rows of the last committed update (rows of U_new)          */
  int64_t rows_pending;
  int32_t initialized;
} dash_dims;

/* Fill *cfg with defaults for the given J, R: lambda 0.7, n_iter 1,
 * init_max_iter 10, init_tol 1e-10 (Sec. 4.1 hyperparameters), FP32 exact mode,
 * capacities 65536 slices / 1M rows / 65536 groups / 4M initial rows, device 0. */
void dash_config_default(dash_config *cfg, int32_t J, int32_t R);

/* Create a context: validates cfg (J, R, lambda in (0,1], n_iter >= 1,
 * capacities >= 1) and allocates every state buffer up front, so later calls
 * allocate nothing on the device.  Errors: DASH_E_INVALID_ARG,
 * DASH_E_OUT_OF_MEMORY, DASH_E_DEVICE.  On success *out owns the context. */
dash_status dash_create(const dash_config *cfg, dash_ctx **out);

/* Wait for outstanding work and free the context.  NULL is a no-op. */
dash_status dash_destroy(dash_ctx *ctx);

/* Initial decomposition of the initial tensor {X_k}_{k<K} (Sec. 3.2.1):
 * PARAFAC2-ALS (V0 = top-R eigenvectors of sum_k X_k^T X_k unless V0 is given,
 * H = I, S_k = I; then per iteration the Procrustes step Q_k = polar(X_k V S_k H^T)
 * and a CP-ALS sweep H -> V -> W on Y_k = Q_k^T X_k), then the helper terms of
 * eq. [updateC_init]-[updateG_init] in the exact form Y_k = U_k^T X_k,
 * D_k = U_k^T U_k, n_k = ||X_k||^2 with U_k = Q_k H.
 *   row_ptr  int64[K+1] in device or host memory, row_ptr[0] = 0,
 *            non-decreasing; slice k is rows row_ptr[k] .. row_ptr[k+1]-1 of X
 *            (each slice needs >= 1 row).  A device array is copied to the host
 *            (the passes are planned there) once the context's stream is idle;
 *            borrowed for the call only.
 *   X        device float[row_ptr[K] * J].
 *   V0       device float[J*R] or NULL.
 *   report   host, may be NULL.
 * Blocking.  Errors: DASH_E_BAD_STATE if already initialised, DASH_E_CAPACITY,
 * DASH_E_INVALID_ARG, DASH_E_NUMERIC (context stays uninitialised). */
dash_status dash_init(dash_ctx *ctx, int32_t K, const int64_t *row_ptr, const float *X,
                      const float *V0, dash_init_report *report);

/* dash_init for callers that cannot allocate device memory (code under HIP
 * graph capture elsewhere in the process, tight serving loops, harnesses that
 * forbid hipMalloc): the same initialisation, with the same results, but its
 * workspace is a fixed array the library holds on each device it runs on
 * (dash_init_noalloc_limit() bytes, kept until the process ends) instead of a
 * per-call allocation; no hipMalloc, hipFree or other allocating call.  The
 * workspace needs (2 J^2 + J + 4 R^2 + K R^2 + ~(K/1024 + 1)(max(2R^2, JR)+2)
 * doubles, plus a Gram matrix's partials when V0 is NULL); larger problems get
 * DASH_E_CAPACITY with nothing done.  The call is synchronous and every call
 * on a device shares that device's array: calls that overlap on one device
 * (from several threads) race.  row_ptr must be host memory here (a device
 * array would need a host copy): DASH_E_INVALID_ARG otherwise.  Other errors
 * as dash_init. */
dash_status dash_init_noalloc(dash_ctx *ctx, int32_t K, const int64_t *row_ptr, const float *X,
                              const float *V0, dash_init_report *report);
/* Bytes of dash_init_noalloc's per-device workspace. */
size_t dash_init_noalloc_limit(void);

/* Helper terms from caller-given factors of the initial tensor
 * (eq. [updateC_init]-[updateG_init]): Y_k = U_k^T X_k, D_k = U_k^T U_k,
 * n_k = ||X_k||^2.  row_ptr/X as for dash_init; U device float[row_ptr[K]*R]
 * (rows aligned with X), W device float[K*R], V device float[J*R].  Blocking. */
dash_status dash_init_from_factors(dash_ctx *ctx, int32_t K, const int64_t *row_ptr,
                                   const float *X, const float *U, const float *W,
                                   const float *V);

/* Stage new rows of existing slices (Problem 1, "Given" item 2).
 *   n         number of row groups (n >= 0).
 *   slice_id  host int32[n]; each in [0, K_pending) -- a slice created by a
 *             staged dash_ingest_slices may be extended too.
 *   row_ptr   host int64[n+1], non-decreasing; group g is rows
 *             row_ptr[g] .. row_ptr[g+1]-1 of rows (empty groups are allowed).
 *   rows      device float[row_ptr[n] * J], borrowed until the update returns.
 * Rows of one slice are appended in ingest order.  Errors:
 * DASH_E_INVALID_ARG, DASH_E_CAPACITY, DASH_E_BAD_STATE (not initialised). */
dash_status dash_ingest_rows(dash_ctx *ctx, int32_t n, const int32_t *slice_id,
                             const int64_t *row_ptr, const float *rows);

/* Stage L new slices (Problem 1, "Given" item 1); they receive ids
 * K_pending, K_pending+1, ... in order and *first_id (host) gets the first.
 *   row_ptr host int64[L+1] with row_ptr[l+1] > row_ptr[l] (>= 1 row each).
 *   rows    device float[row_ptr[L] * J], borrowed as for dash_ingest_rows. */
dash_status dash_ingest_slices(dash_ctx *ctx, int32_t L, const int64_t *row_ptr,
                               const float *rows, int32_t *first_id);

/* Run one update (Algorithm 1 with Lemmas 1-3, n_iter ALS passes) on all
 * staged data and wait for it.  No staged rows: no-op, DASH_OK, report->rows 0
 * and no forgetting applied.  On non-finite factors the update is rolled back
 * (staged data dropped, state as before) and DASH_E_NUMERIC is returned.
 * report: host, may be NULL. */
dash_status dash_update(dash_ctx *ctx, dash_update_report *report);

/* Enqueue the update and return without waiting; staged pointers stay borrowed
 * until dash_wait.  Several updates may be in flight.  If one of them fails
 * numerically, it and every later in-flight update are discarded and dash_wait
 * reports DASH_E_NUMERIC with the failing step in report->step. */
dash_status dash_update_async(dash_ctx *ctx);

/* Wait for all enqueued updates; *report (may be NULL) describes the last one. */
dash_status dash_wait(dash_ctx *ctx, dash_update_report *report);

/* Copy the current factors into caller-owned device buffers (any may be NULL):
 *   V      float[J*R];  W float[K*R] (row k = diagonal of S_k);
 *   U_new  float[m_last*R], the rows of U_{k,new} of the last committed update
 *          in ingest order (new-slice groups and row groups interleaved exactly
 *          as they were staged).  U_{k,old} is not retained (Sec. 3.2.2).
 *   m_last host int64, may be NULL.
 * Waits for outstanding updates first. */
dash_status dash_get_factors(dash_ctx *ctx, float *V, float *W, float *U_new, int64_t *m_last);

dash_status dash_get_dims(const dash_ctx *ctx, dash_dims *dims);

/* Export / import the streaming state in float64 host arrays:
 *   V [J*R], W [K*R], Y [K*R*J] (Y_k = sum lambda^age U_k^T X_k), D [K*R*R]
 *   (D_k = sum lambda^age U_k^T U_k), n [K] (sum lambda^age ||x||^2).
 * dash_get_state returns the values as of the last committed update (any
 * pointer may be NULL).  dash_set_state replaces the whole state (marks the
 * context initialised, K slices, step kept) -- it is how a checkpoint is
 * restored and how tests start both implementations from one state. */
dash_status dash_get_state(dash_ctx *ctx, double *V, double *W, double *Y, double *D, double *n);
dash_status dash_set_state(dash_ctx *ctx, int32_t K, const double *V, const double *W,
                           const double *Y, const double *D, const double *n);

/* Checkpoint the committed state to a file and restore it.  The file holds the
 * state exactly as the device keeps it (float32 Y_k, D_k, float64 n_k, W, V,
 * and the update index at which each slice was last folded), so a restored
 * context continues bit for bit like the one that was saved.  dash_load needs
 * a context with the same J, R and lambda and enough max_slices; it replaces
 * the state and the update counter.  Errors: DASH_E_IO, DASH_E_INVALID_ARG. */
dash_status dash_save(dash_ctx *ctx, const char *path);
dash_status dash_load(dash_ctx *ctx, const char *path);

/* Per-kernel device time of the update path, measured with HIP events recorded
 * around each launch on the context's stream.  dash_profile(ctx, every) clears
 * the counters and, for every > 0, records the launches of the updates whose
 * index (dash_update_report.step) is a multiple of `every` (1: all of them;
 * timing events perturb the launches they bracket, so sampling keeps the
 * others undisturbed); dash_profile(ctx, 0) stops.  dash_profile_read waits for
 * outstanding work and returns the sums since the last clear. */
typedef struct dash_profile_stats {
  int64_t updates;
  int64_t pass_launches, reduce_launches, solve_launches, commit_launches, upload_launches;
  double pass_ms, reduce_ms, solve_ms, commit_ms, upload_ms;
} dash_profile_stats;

dash_status dash_profile(dash_ctx *ctx, int32_t every);
dash_status dash_profile_read(dash_ctx *ctx, dash_profile_stats *out);

const char *dash_status_string(dash_status s);
const char *dash_last_error(const dash_ctx *ctx);

/* Fault injection, for tests of the error paths: the next call that reaches
 * `site` fails there as the real failure would, then the injection is spent.
 * Sites: DASH_SITE_INGEST -- the next dash_ingest_rows / dash_ingest_slices
 * with work to stage returns DASH_E_CAPACITY, nothing staged;
 * DASH_SITE_LAUNCH -- the next dash_update / dash_update_async with staged
 * rows returns DASH_E_DEVICE before enqueuing anything, the rows stay staged;
 * DASH_SITE_COMMIT -- the next enqueued update's commit check (final phase,
 * on the device) treats its factors as non-finite: the update is rolled back
 * exactly as for NaN input (DASH_E_NUMERIC, staged data dropped, state as
 * before); DASH_SITE_INIT_ALLOC -- the next dash_init's scratch allocation
 * fails (DASH_E_OUT_OF_MEMORY, context stays uninitialised).  DASH_SITE_NONE
 * cancels a pending injection.  Host only; no device call.  Errors:
 * DASH_E_INVALID_ARG (NULL ctx, unknown site). */
typedef enum dash_fail_site {
  DASH_SITE_NONE = 0,
  DASH_SITE_INGEST = 1,
  DASH_SITE_LAUNCH = 2,
  DASH_SITE_COMMIT = 3,
  DASH_SITE_INIT_ALLOC = 4
} dash_fail_site;
dash_status dash_debug_fail_next(dash_ctx *ctx, int32_t site);

/* Non-blocking completion check (Algorithm 1's outputs as they become ready):
 * reaps, in order, the enqueued updates that have finished, up to cap, and
 * writes their reports to reports[0 .. *n_done).  If one of them was not
 * committed (non-finite factors), the call drains the context like dash_wait,
 * reports that update last and returns DASH_E_NUMERIC.  reports is host memory
 * (may be NULL when cap == 0). */
dash_status dash_poll(dash_ctx *ctx, dash_update_report *reports, int32_t cap, int32_t *n_done);

/* Autotuning of the launch schedule: with trials > 0 the next updates run in
 * turn with every candidate -- the sweep variant (the fused one-wave-per-slice
 * sweep where it applies, or the split sweep), twice the default slices per F
 * chunk or not, the final phase fused into the sweep launch or separate, the
 * split sweep's solve chunks at the default size or a quarter of it -- each
 * `trials` times; every candidate is scored by device time per algorithmic
 * byte of its updates and the best is kept for the updates after that.  Every
 * schedule computes the same update; results differ between schedules only by
 * the order of the FP64 partial sums.  trials = 0 returns to the default
 * schedule.  With a cache (dash_autotune_cache) the shape of the first update
 * of the run -- J, R, precision, statistics mode, passes, and log2 buckets of
 * the mean rows per touched slice and of the slice count -- is looked up
 * first: a cached schedule is taken at once, and a finished run stores its
 * winner.  dash_autotune_read reports the schedule in force. */
typedef struct dash_schedule {
  int32_t variant;     /* 0: one wave per slice, 1: one workgroup per slice     */
  int32_t spread;      /* slices per chunk relative to the default (1 or 2)     */
  int32_t fused;       /* 1: the final phase runs in the sweep launch           */
  int32_t solve_div;   /* split sweep: solve chunks of 1/solve_div the default   */
  int32_t from_cache;  /* 1: the schedule came from the autotuner's cache        */
  int32_t tuned;       /* 1: chosen by a finished autotuning run                */
  int32_t candidates;  /* schedules of the last autotuning run                  */
  double ns_per_kb;    /* measured device ns per KiB of algorithmic traffic of
                          the schedule in force (0 if not measured)             */
} dash_schedule;
dash_status dash_autotune(dash_ctx *ctx, int32_t trials);
dash_status dash_autotune_read(dash_ctx *ctx, dash_schedule *out);
/* The autotuner's cache file (JSON lines, one tuned schedule per shape key;
 * read at the start of a tuning run, rewritten when a run finishes), or NULL
 * for none.  Errors: DASH_E_INVALID_ARG. */
dash_status dash_autotune_cache(dash_ctx *ctx, const char *path);

/* Graph mode (enable = 1): each update's launches -- descriptor fetch, the
 * n_iter sweeps and final phases -- are replayed from one executable HIP graph
 * captured at the first update, with every kernel node's grid and arguments
 * rewritten for the update at hand (no allocation, no memset node).  Updates
 * that dash_profile times are launched directly.  Waits for the context's
 * work; enable = 0 drops the graph. */
dash_status dash_graph(dash_ctx *ctx, int32_t enable);

/* Per-update device spans: with dash_spans(ctx, 1) the device_us of every
 * update reaped from then on by dash_update, dash_wait or dash_poll is kept;
 * dash_spans_read copies them (milliseconds, in update order), at most cap.
 * dash_spans(ctx, 0) stops; either call clears the list. */
dash_status dash_spans(dash_ctx *ctx, int32_t enable);
dash_status dash_spans_read(dash_ctx *ctx, float *ms, int32_t cap, int32_t *n);

/* Anomaly scores (Sec. 3.4, Definitions 1-2; threshold of Sec. 4.5): with
 * window >= 1 every later update also computes, with its updated S_k and V,
 *   se_k = sum_{i,j} |X_{k,new} - U_{k,new} S_k V^T|_{ij} / (I_{k,new} J)
 * for each slice that received rows, flags the slices whose se_k exceeds the
 * mean plus the population standard deviation of that slice's previous
 * `window` scores, and reports te (the mean of se_k) with the same threshold
 * over the context's previous te (dash_update_report).  The kernel re-reads
 * the update's rows (J floats per row) after the final phase; updates with
 * scores on are launched directly (no graph replay).  window = 0 turns the
 * scores off; enabling clears every history.  Allocates its buffers here.
 * Errors: DASH_E_INVALID_ARG (window < 0), DASH_E_OUT_OF_MEMORY. */
dash_status dash_anomaly(dash_ctx *ctx, int32_t window);

/* The slice-level scores of the last committed update that was scored: for
 * at most cap of its slices, in ascending slice id, slice[i] (host int32),
 * se[i] (host float) and flag[i] (host int32, 1 = anomaly); *n receives the
 * count.  Waits for outstanding updates.  Errors: DASH_E_BAD_STATE when
 * scores are off, DASH_E_INVALID_ARG. */
dash_status dash_get_slice_errors(dash_ctx *ctx, int32_t *slice, float *se, int32_t *flag, int32_t cap,
                                  int32_t *n);

/* Device bytes that dash_create allocates for cfg (the admission footprint of
 * a served stream).  Errors: DASH_E_INVALID_ARG. */
dash_status dash_footprint(const dash_config *cfg, int64_t *bytes);

/* ---------------------------------------------------------------------------
 * Serving: many independent streams on one device.  Every stream is an
 * irregular tensor of its own with its own J, R, lambda and precision
 * (Problem 1 per stream), decomposed by a context of its own.  Clients submit
 * rows at any time; a tick cuts one update per stream from the rows it has
 * and runs the updates of all streams together, each stage of the update as
 * one launch per kernel class over every stream.  A stream's workgroup counts
 * and reduction order depend on the stream alone, so its results are bit for
 * bit the same alone and in any mix.  Served streams always run the split
 * sweep.  All server calls are thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct dash_server dash_server;

typedef struct dash_server_report {
  int32_t stream;        /* stream id                                            */
  int32_t committed;     /* as dash_update_report.committed                     */
  int64_t step;          /* the stream's update index                            */
  int64_t rows;          /* rows the update consumed                             */
  double fit;            /* the stream's fit after the update                    */
  double latency_us;     /* host time from the submit of the update's first
                            request to the moment the server saw it committed */
  int64_t last_request;  /* the last request the update consumed: the device
                            buffers of this stream's requests up to it are free */
  double device_us;      /* device time of the update (its tick's span)          */
} dash_server_report;

typedef struct dash_server_stats {
  int64_t ticks;         /* ticks launched                                        */
  int64_t launches;      /* kernel launches of those ticks                       */
  int64_t updates;       /* updates reported                                     */
  int64_t rows;          /* rows of those updates                                */
  int64_t budget, used;  /* device bytes: budget, admitted footprints            */
  int32_t queued;        /* streams waiting for admission                        */
  int32_t open;          /* admitted streams                                     */
} dash_server_stats;

/* A server on `device` whose streams may together allocate at most
 * budget_bytes of device memory.  Its HIP stream is a blocking one: ordered
 * after work the caller put on the null stream.  Errors: DASH_E_INVALID_ARG,
 * DASH_E_OUT_OF_MEMORY, DASH_E_DEVICE. */
dash_status dash_server_create(int32_t device, int64_t budget_bytes, dash_server **out);
/* Stop the loop, wait for every update in flight, close every stream, free. */
dash_status dash_server_destroy(dash_server *srv);
/* Open a stream for cfg (device and stream fields are replaced by the
 * server's).  If its footprint (dash_footprint) fits the unused budget and no
 * stream is waiting, its context is created now (state 2, open).  Otherwise,
 * with queue = 1 it waits in a FIFO admission queue (state 1) and is admitted
 * when closes free enough budget; with queue = 0 DASH_E_CAPACITY is returned
 * and nothing changes.  *stream receives its id either way.  A stream whose
 * footprint exceeds the whole budget is refused.  Errors: as dash_create,
 * DASH_E_CAPACITY. */
dash_status dash_server_open(dash_server *srv, const dash_config *cfg, int32_t queue, int32_t *stream);
/* *state: 0 closed or unknown, 1 waiting for admission, 2 open. */
dash_status dash_server_state(dash_server *srv, int32_t stream, int32_t *state);
/* Close a stream: its updates in flight finish and are reported, requests not
 * yet in an update are dropped, its context is freed and its budget returned;
 * waiting streams are admitted.  Errors: DASH_E_INVALID_ARG. */
dash_status dash_server_close(dash_server *srv, int32_t stream);
/* The context of an open stream, or NULL.  The caller initialises it with
 * dash_init* and reads it with dash_get_* (only while none of its requests is
 * waiting or in flight, e.g. after dash_server_drain); dash_ingest_*,
 * dash_update* and dash_poll/dash_wait are the server's. */
dash_ctx *dash_server_context(dash_server *srv, int32_t stream);
/* Submit rows to an open, initialised stream: n_groups row groups as
 * dash_ingest_rows (host slice_id and row_ptr, device rows) and n_new new
 * slices as dash_ingest_slices (host new_ptr, device new_rows); the groups may
 * name the new slices, whose ids start at *first_new_id (may be NULL).  The
 * host arrays are copied; the device buffers stay the caller's and must not
 * change until an update of this stream reports last_request >= *request.
 * producer: the HIP stream the rows were written on (the update waits for
 * it), or NULL for the null stream.  Errors: DASH_E_INVALID_ARG,
 * DASH_E_BAD_STATE (not open or not initialised), DASH_E_CAPACITY (more rows,
 * groups or slices than the stream's configuration allows). */
dash_status dash_server_submit(dash_server *srv, int32_t stream, int32_t n_groups, const int32_t *slice_id,
                               const int64_t *row_ptr, const float *rows, int32_t n_new, const int64_t *new_ptr,
                               const float *new_rows, void *producer, int64_t *request, int32_t *first_new_id);
/* One tick on the calling thread: every open stream with submitted rows (and
 * fewer than four updates in flight) gets one update of the requests that fit
 * its per-update capacity.  *launched (may be NULL) receives the count. */
dash_status dash_server_tick(dash_server *srv, int32_t *launched);
/* Finished updates into out[0 .. *n), at most cap, in completion order.
 * wait = 1 (no loop running): first wait for everything in flight.  A stream
 * whose update was rolled back reports it and the updates after it with
 * committed = 0; the first such status is returned. */
dash_status dash_server_poll(dash_server *srv, int32_t wait, dash_server_report *out, int32_t cap,
                             int32_t *n);
/* Run ticks and completion polling on a host thread of the server's own: a
 * tick starts when rows are waiting, tick_us microseconds have passed since the
 * last one (0: at once) and either no tick is in flight or one is and
 * every open stream has rows waiting.  Errors: DASH_E_BAD_STATE
 * when already running. */
dash_status dash_server_start(dash_server *srv, int32_t tick_us);
/* Stop the loop thread (updates in flight continue; poll with wait = 1). */
dash_status dash_server_stop(dash_server *srv);
/* Wait until every submitted request is in a committed, collected update
 * (reports stay for dash_server_poll).  timeout_ms < 0: no limit; on timeout
 * DASH_E_BAD_STATE. */
dash_status dash_server_drain(dash_server *srv, int32_t timeout_ms);
dash_status dash_server_get_stats(dash_server *srv, dash_server_stats *out);
/* Device time of the server's kernels, per kernel instantiation. */
typedef struct dash_kernel_stat {
  char name[48];        /* e.g. "k_solve<16>" (stage kernel and template arguments) */
  int64_t launches;     /* timed launches                                          */
  double ms;            /* their summed device time (HIP events around each launch,
                           on the server's stream)                                 */
  double bytes;         /* their summed algorithmic bytes                          */
} dash_kernel_stat;
/* Time every launch of every `every`-th tick from now on (0: stop); clears the
 * statistics.  Events sit between the timed launches, so the timed ticks run
 * slightly slower than the others. */
dash_status dash_server_profile(dash_server *srv, int32_t every);
/* The statistics so far (waits for the timed ticks): at most cap entries into
 * out, *n the count, *ticks (may be NULL) the ticks timed. */
dash_status dash_server_profile_read(dash_server *srv, dash_kernel_stat *out, int32_t cap, int32_t *n,
                                     int64_t *ticks);
/* Text of the server's last launch error ("" if none). */
const char *dash_server_last_error(dash_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* DASH_H */
