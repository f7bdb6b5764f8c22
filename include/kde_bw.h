/*
 * kde_bw.h -- C ABI of the MI355X (gfx950) engine for exact bandwidth-selection
 * pair sums of univariate Gaussian kernel density estimates.
 *
 * Method: Andrzejewski, Gramacki, Gramacki, "Density Estimations for
 * Approximate Query Processing on SIMD Architectures" (arXiv 1505.01998).
 * The selectors are those of its Section 4.4: the normal-reference rule, the
 * direct plug-in chain of Section 4.4.1 and the least-squares cross-validation
 * objective g(h) of Section 4.4.2 minimised over a grid, with the O(n^2) pair
 * sums of Section 5.4 evaluated on the GPU.
 *
 * Conventions shared by every call
 *  - Every call returns a kde_status; nothing throws across the ABI.  On any
 *    status other than KDE_OK, kde_last_error() describes the failure.
 *  - A context is bound to one device and is not thread-safe: calls on one
 *    context must not overlap.  Independent contexts may be used from
 *    different threads.
 *  - Synchronous calls borrow their inputs for the duration of the call only
 *    and return after the results are in the caller's (host) output buffers.
 *  - A sample column is n >= 2 finite values, float32 or float64, contiguous,
 *    in host memory (on_device = 0) or in device memory of the context's
 *    device (on_device = 1; the pointer must be valid on the context's stream).
 *    n is limited to KDE_MAX_N.  A non-finite sample or n < 2 gives
 *    KDE_E_INVAL.
 *  - Bandwidth grids are float64 host arrays in data units: the kernel at h is
 *    the N(0, h^2) density, the same h as the estimator of Section 4.2
 *    (eq. kde-def).  Entries must be finite, > 0 and strictly ascending, else
 *    KDE_E_INVAL.  1 <= n_h <= KDE_MAX_NH.
 *  - Device failures (launch or copy errors) give KDE_E_DEVICE; the context
 *    must then be destroyed.
 */
#ifndef KDE_BW_H
#define KDE_BW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KDE_MAX_N ((int64_t)1 << 30)
#define KDE_MAX_NH 65536
#define KDE_MAX_BATCH 65535
#define KDE_MAX_QUERIES (1 << 24) /* query points or ranges per kde_density / kde_range_aggregates call */
#define KDE_MAX_D 16 /* dimensions of a sample matrix (kde_lscv_md_curve) */
#define KDE_MAX_H_EVAL 65536 /* bandwidth matrices per kde_lscv_H_eval call */

typedef enum {
  KDE_OK = 0,
  KDE_E_INVAL = 1,      /* bad argument or sample column */
  KDE_E_DEGENERATE = 2, /* sigma = 0, or a functional estimate of the wrong sign */
  KDE_E_NOMEM = 3,      /* device or pinned allocation failed; a served request larger than the
                         * server's whole HBM budget; a kde_lscv_curve_noalloc column larger than
                         * its fixed scratch */
  KDE_E_DEVICE = 4,     /* HIP runtime error */
  KDE_E_BUSY = 5,       /* reserved: result not ready */
  KDE_E_CANCELLED = 6   /* reserved: request cancelled */
} kde_status;

typedef enum { KDE_F32 = 0, KDE_F64 = 1 } kde_dtype;

typedef enum {
  /* Pair terms in FP32 (hardware exp2), FP32 running sums folded into
   * Kahan-compensated FP32 per-lane accumulators, FP64 across lanes, tiles and
   * blocks, FP64 for every scalar step and for g(h) = difference of sums.  A
   * plug-in stage whose pair sum is badly conditioned is re-run in FP64. */
  KDE_PREC_MIXED = 0,
  /* Every pair term and every sum in FP64. */
  KDE_PREC_FP64 = 1
} kde_prec;

typedef struct kde_ctx kde_ctx;

typedef struct {
  const void* data; /* n samples */
  int64_t n;
  kde_dtype dtype;
  int on_device; /* 0: host pointer, 1: device pointer */
} kde_column;

/* Plug-in diagnostics.  Stage order is (psi_8, psi_6, psi_4); for stages = 2
 * slot 0 holds the normal-scale psi_8 of eq. (PLUGIN-Psi8Estimate) and g[0],
 * kappa[0] are NaN.  g[s] is the pilot bandwidth of stage s (eq. PLUGIN-g1,
 * PLUGIN-g2), psi[s] its estimate (eq. PLUGIN-Psi6Estimate, PLUGIN-Psi4Estimate),
 * kappa[s] = sum|t| / |sum t| over its pair terms (condition number of the
 * pair sum), precision_used[s] the kde_prec the stage's pair sum was taken in
 * (-1 where no pair sum was taken). */
typedef struct {
  double sigma, h_rot;
  int stages;
  double g[3], psi[3], kappa[3];
  int precision_used[3];
  double h;
} kde_plugin_info;

/* Create a context on HIP device `device` computing in precision `prec`.
 * The context owns a HIP stream of default priority, a device workspace that
 * grows on demand, and per-kernel timing counters. */
kde_status kde_ctx_create(int device, kde_prec prec, kde_ctx** out);
/* Stops a running server, then releases every prepared LSCV_H sample
 * (kde_lscv_H_prepare) and every resumable job (kde_job_create) created on
 * the context and not yet released; those handles must not be used after. */
void kde_ctx_destroy(kde_ctx* ctx);

/* Text of the last failure on this context; owned by the context and valid
 * until its next call.  Never NULL. */
const char* kde_last_error(const kde_ctx* ctx);

/* Run on an external stream (a hipStream_t of the context's device, e.g. the
 * caller's framework stream) instead of the context's own; NULL restores it. */
kde_status kde_ctx_set_stream(kde_ctx* ctx, void* hip_stream);

/* Change the precision used by later calls. */
kde_status kde_ctx_set_precision(kde_ctx* ctx, kde_prec prec);

/* Tuning knobs by name (value < 0 restores the default):
 *   "lscv_hc"      bandwidths per pass of the LSCV pair kernel (8, 16 or 32)
 *   "lscv_tj"      samples per LDS tile of the persistent dense LSCV sweep
 *                  (256, 512 or 1024; other than 512 only with lscv_hc 16,
 *                  else the pass falls back to sliced launches).  Results
 *                  are bitwise those of any tile size.
 *   "seg"          j-range per work item, rounded to the tile (0 = whole row)
 *   "launch_evals" pair-term evaluations per kernel launch (launch splitting)
 *   "fp64_kappa"   mixed precision: kappa above which a plug-in stage is re-run
 *                  in FP64 (0 = never)
 *   "lscv_mfma"    1: form the LSCV exponent arguments on the matrix cores
 *                  (mixed precision with lscv_hc 16; results identical in
 *                  value to rounding, not bitwise, to the vector-ALU kernel)
 *   "serve_iter_evals" server: minimum pair-term evaluations per scheduler
 *                  iteration (an iteration also holds at least 24 rounds of
 *                  1024 blocks of its largest work unit).  Pruned sweeps are
 *                  counted at their dense size, so with "prune" an iteration
 *                  does less work than it counts; a larger value keeps the
 *                  per-iteration host work small against it.
 *   "serve_iter_ms" server: target duration of a full scheduler iteration
 *                  (0: off, iterations sized by serve_iter_evals alone).  The
 *                  server measures each iteration that used its whole
 *                  budget and moves the next budget towards this duration,
 *                  within [1, 64] x serve_iter_evals: with "prune", whose
 *                  sweeps do less than they count, iterations keep their
 *                  length.  Results do not depend on it.
 *   "serve_aging_ms" server: aging of the smallest-remaining-work order: a
 *                  request's remaining evaluations count divided by
 *                  1 + waited / tau (tau in ms; 0: plain order), so large
 *                  requests are not held back indefinitely under load
 *   "serve_fail_ticket" server, failure handling: the request with this
 *                  ticket (tickets count from 1 per server) is treated as if
 *                  its pass had failed: it ends with KDE_E_DEVICE and frees
 *                  its slot while the requests sharing its launches complete
 *                  (0: off).  Forced from the host; every kernel runs as usual.
 *   "autotune"     1: synchronous calls and kde_batch run the LSCV pass in
 *                  the variant (bandwidths per block, tile size) that
 *                  kde_autotune measured fastest for the job's largest LSCV
 *                  column (tuning that shape on first use when the job holds
 *                  at least 1e13 pair-term evaluations; smaller jobs use a
 *                  cached decision or lscv_hc / lscv_tj).  Results are
 *                  bitwise those of any variant.
 *   "prune"        1: LSCV tile pruning on sorted samples (mixed precision;
 *                  synchronous calls, kde_batch, the server and jobs).
 *                  Each LSCV column is sorted on the device (the pair
 *                  sums do not depend on the order); the first j-tile of every
 *                  row gives lower bounds L(h) of the positive pair sums; a
 *                  256 x 512 tile farther from its row than the chunk's cut
 *                  is skipped when even its largest possible terms add up,
 *                  over all skipped tiles, to less than 2^-34 L(h) for S1 and
 *                  S2 and every h of the chunk.  Results stay within 2^-34 of
 *                  the dense sums on top of the arithmetic error;
 *                  kde_result.lscv_evals counts what was evaluated.  The
 *                  plug-in passes are unchanged.  A column's pruned results
 *                  are bitwise the same alone, in a batch, served or run as
 *                  a job.
 *   "persistent"   1 (default): the dense mixed-precision LSCV pass of a job
 *                  (synchronous call, batch, server iteration, job slice) is
 *                  one launch of about as many blocks as the device holds,
 *                  which take the pass's work units in order, largest first,
 *                  from a device counter; 0: launches of bounded work
 *                  ("launch_evals").  Results are bitwise the same.
 *   "graph"        1: the kernel launches of a synchronous call or kde_batch
 *                  are captured into a HIP graph; a later call with the same
 *                  signature (per request: validity, n, dtype, host/device,
 *                  methods, stages, grid kind and size, log-grid range; the
 *                  options) replays it instead of planning and launching
 *                  again.  Samples, grid values and device column addresses
 *                  are copied in around the graph, so a replay computes on the
 *                  new inputs; results are bitwise those without the option.
 *                  Up to 8 graphs are kept per context (least recently used
 *                  replaced); a graph whose device buffers were reallocated
 *                  by a larger job is captured again.  Inactive while timing
 *                  is on or when the context runs on the null stream.
 * Unknown keys give KDE_E_INVAL. */
kde_status kde_ctx_set_option(kde_ctx* ctx, const char* key, int64_t value);

/* Counters of the "graph" option since the context was created: jobs whose
 * launches were captured into a new graph, and jobs that replayed one. */
kde_status kde_ctx_graph_stats(kde_ctx* ctx, int64_t* captures, int64_t* replays);

/* Tile autotuner of the LSCV pair pass (eq. LSCV-gh over a grid, every h
 * from one pair distance as in Section 4.5).  Times the persistent dense
 * sweep in five variants (bandwidths per block, samples per LDS tile) =
 * (8, 512), (16, 256), (16, 512), (16, 1024), (32, 512) on trial launches of
 * a column shaped like n samples with an n_h-point grid (rows of an evenly
 * spread column of min(n, 8192) samples in buffers of the context; B and 2B
 * units differenced) and caches the fastest per shape (quarter octave of n,
 * n_h) in the context (each variant timed twice, keeping its better rate);
 * the default (16, 512) is kept unless another is 3% faster.  A variant is
 * a candidate only if its trial partial sums for the first 8 bandwidths are
 * bitwise those of the default (in both trials): the variant never
 * changes a result, since items and summation order do not depend on it.
 * out->hc and out->tj receive the choice, out->evals_per_s[v] the measured
 * rate of variant v in the order above (pair-term evaluations per second,
 * scaled by the share of its bandwidth slots the grid fills; 0 if the
 * variant could not run), out->parity[v] 1 when it passed the gate.  A cached
 * shape returns at once.  KDE_E_INVAL for n outside [2, KDE_MAX_N], n_h
 * outside [1, KDE_MAX_NH] or a context in FP64 precision; KDE_E_BUSY while a
 * server runs. */
typedef struct {
  int32_t hc;
  int32_t tj;
  double evals_per_s[5];
  int32_t parity[5];
  int32_t pad0;
} kde_tune_info;
kde_status kde_autotune(kde_ctx* ctx, int64_t n, int32_t n_h, kde_tune_info* out);
/* Measures the ceiling of the LSCV sweep's inner loop on this device: the
 * kernel's own per-(pair, h) code (Section 4.5: the pair distance formed once
 * and reused for hc bandwidths; FP32 exp2, S1 add, S2 fma, 64-term runs
 * folded into FP64) repeated over one LDS tile staged once, without tile
 * staging, barriers, masks or partial-sum writes.  *evals_per_s receives its
 * pair-term evaluations per second: launches of R and 2R repetitions (~0.1
 * and ~0.25 s) timed with events on the context's stream, the rate taken
 * over the extra R of the second so that launch start and drain cancel.
 * The rate bounds what the sweep can
 * reach with this instruction mix.  It measures the mixed form's kernel
 * whatever the context's precision.  KDE_E_INVAL for hc other than 8, 16,
 * 32; KDE_E_BUSY while a server runs. */
kde_status kde_lscv_ceiling(kde_ctx* ctx, int32_t hc, double* evals_per_s);
/* Issue-rate probe of the vector ALU on this device: the rates that bound
 * the pair kernels of Section 4.4 (psi_r sums, LSCV sums with the pair
 * distance reused across bandwidths as in Section 4.5), which run from
 * registers and LDS.  Register-only loops of eight independent chains per
 * lane, about 0.05-0.2 s per case, timed with events on the context's stream;
 * results are per clock and per compute unit at the device's reported engine
 * clock (clock_hz) over its cus compute units.  add_f32, mul_f32, fma_f32:
 * plain (unpacked) FP32 vector lanes issued; exp_f32: v_exp_f32 lanes;
 * lscv_mix: LSCV pair-bandwidth terms (one mul, one exp2, one add, one fma)
 * with exponents spread over (2^-71, 1]; lscv_mix_zero: the same loop with
 * every distance 0 (every exponential is exp2(0)).  KDE_E_BUSY while a
 * server runs; KDE_E_DEVICE on a HIP error. */
typedef struct {
  double clock_hz;
  int32_t cus;
  int32_t pad0;
  double add_f32, mul_f32, fma_f32, exp_f32;
  double lscv_mix, lscv_mix_zero;
} kde_issue_info;
kde_status kde_issue_rates(kde_ctx* ctx, kde_issue_info* out);

/* Kernel timing.  While enabled, every launch of the pair kernels is bracketed
 * by HIP events on the stream it runs on.  kde_ctx_kernel_time reports, for
 * kernel family "lscv_pairs", "psi_pairs" or "md_pairs" (the d-dimensional
 * pair kernels: LSCV_h, LSCV_H, density with a bandwidth matrix), the number
 * of launches, their
 * summed duration in ms and the summed pair-term evaluations since timing was
 * last enabled. */
kde_status kde_ctx_set_timing(kde_ctx* ctx, int enable);
kde_status kde_ctx_kernel_time(kde_ctx* ctx, const char* family, int64_t* launches, double* total_ms,
                               double* evals);

/* Normal-reference bandwidth h = (4/3)^(1/5) sigma n^(-1/5): eq. (LSCV-H-start)
 * with d = 1, equal to sigma * h0 of eq. (LSCV-h0); sigma from
 * eq. (PLUGIN-VarianceEstimator)/(PLUGIN-StdDevEstimator), n-1 denominator.
 * KDE_E_DEGENERATE when sigma = 0. */
kde_status kde_bw_rot(kde_ctx* ctx, kde_column x, double* h_out);

/* Direct plug-in bandwidth, Section 4.4.1, eq. (PLUGIN-VarianceEstimator)
 * through (PLUGIN-Final_h).  stages = 2 is the printed chain (normal-scale
 * psi_8, pairwise psi_6 and psi_4); stages = 3 starts from the normal-scale
 * psi_10 and estimates psi_8 pairwise as well.  psi_r(g) is read as
 * n^-2 g^-(r+1) sum over all (i, j) of K^(r)((X_i - X_j)/g), i.e. the diagonal
 * term n K^(r)(0) inside the normalisation.  info may be NULL.
 * KDE_E_DEGENERATE when sigma = 0 or a pilot/final radicand is not positive. */
kde_status kde_bw_plugin(kde_ctx* ctx, kde_column x, int stages, double* h_out, kde_plugin_info* info);

/* LSCV objective over a grid, eq. (LSCV-gh) with (LSCV-Tx), (LSCV-Kx),
 * (LSCV-KKx), in data units for d = 1:
 *   g(h) = h^-1 [ 2 n^-2 sum_{i<j} T((X_i - X_j)/h) + n^-1 (4 pi)^(-1/2) ],
 *   T = K*K - 2K.
 * The pair distance is formed once per pair and reused for every h of the grid
 * (the rewrite of Section 4.5), nothing is stored per pair.
 * h_grid == NULL selects the default grid: n_h points (150 if n_h <= 0)
 * spaced linearly over sigma * [h0/4, 4 h0] (eq. LSCV-Zh0, LSCV-h0).
 * g_out[n_h] receives g(h); gscale_out[n_h] (may be NULL) receives the same
 * expression with the two pair sums added instead of subtracted, the scale
 * against which errors in g are measured.  grid_out[n_h] (may be NULL)
 * receives the grid used. */
kde_status kde_lscv_curve(kde_ctx* ctx, kde_column x, const double* h_grid, int32_t n_h, double* g_out,
                          double* gscale_out, double* grid_out);

/* For callers that cannot allocate memory (code whose harness forbids
 * hipMalloc, tight serving loops): kde_lscv_curve computed with no device,
 * pinned or other HIP allocation in the call.  Same arguments and results as
 * kde_lscv_curve without grid_out; the values are bitwise those of
 * kde_lscv_curve on the same context options.  The job's device workspace
 * (the column's working copy, partial sums, grid, work list) lives in a fixed
 * device array of KDE_NOALLOC_SCRATCH_BYTES that every GPU the library runs
 * on holds from the library's load until the process ends; the host side
 * stages through pageable buffers of the context, kept between calls.  Every
 * call on one GPU shares that GPU's array and leaves the last call's contents
 * in it (the call initialises all it reads): calls that overlap on one GPU,
 * from any contexts or threads, race and must be serialised by the caller.
 * KDE_E_NOMEM (no allocation attempted) when the column needs more than the
 * array holds: every n <= 131072 with n_h <= 512 fits, in either precision;
 * KDE_E_INVAL as kde_lscv_curve, and while the autotune option is on (its
 * trials allocate); KDE_E_BUSY while a server runs on the context. */
#define KDE_NOALLOC_SCRATCH_BYTES ((uint64_t)32 << 20)
kde_status kde_lscv_curve_noalloc(kde_ctx* ctx, kde_column x, const double* h_grid, int32_t n_h, double* g_out,
                                  double* gscale_out);

/* The two raw pair sums behind g(h): s1[k] = sum_{i<j} exp(-D^2/(4 h_k^2)),
 * s2[k] = sum_{i<j} exp(-D^2/(2 h_k^2)), D = X_i - X_j.  h_grid must not be
 * NULL. */
kde_status kde_lscv_sums(kde_ctx* ctx, kde_column x, const double* h_grid, int32_t n_h, double* s1_out,
                         double* s2_out);

/* Diagnostic view of the LSCV pass: runs exactly the pass kde_lscv_sums runs
 * (same work list and launch slicing for this n, grid and context options)
 * and returns the FP64 partial sums of selected work items.  A work item is
 * one block of the i < j triangle: samples i in [i_begin, i_begin + 256) and
 * j in [j_begin, j_end), pairs with j <= i or an index >= n excluded.
 * sel[n_sel] are item indices in [0, n_items), or negative to count from the
 * end (-1 = last); items are ordered longest first.  n_items_out receives
 * the item count.  ranges_out[3*k..3*k+2] receives
 * (i_begin, j_begin, j_end) of item sel[k]; sums_out[(k*n_h + h)*2 + {0,1}]
 * receives its s1/s2 partials for grid point h. */
kde_status kde_lscv_item_sums(kde_ctx* ctx, kde_column x, const double* h_grid, int32_t n_h, const int32_t* sel,
                              int32_t n_sel, int32_t* n_items_out, int32_t* ranges_out, double* sums_out);

/* ---------------------------------------------------------------- batches
 * Many columns in one job: their moment passes, plug-in stages and LSCV
 * passes run as shared launches whose work units mix columns, largest first.
 * Each column keeps the work decomposition and reduction order it has when
 * run alone, so every result of a batch is bitwise identical to the same
 * request made on its own. */

typedef enum {
  KDE_GRID_EXPLICIT = 0, /* h[n_h], host float64, finite, > 0, strictly ascending */
  KDE_GRID_PAPER = 1,    /* n_h points linear over sigma * [h0/4, 4 h0], eq. (LSCV-Zh0) */
  KDE_GRID_LOG_ROT = 2   /* n_h points log-spaced over h_rot * [lo, hi], 0 < lo < hi */
} kde_grid_kind;

typedef struct {
  kde_grid_kind kind;
  const double* h;
  int32_t n_h;
  double lo, hi;
} kde_grid;

#define KDE_METHOD_ROT 1u
#define KDE_METHOD_PLUGIN 2u
#define KDE_METHOD_LSCV 4u

typedef struct {
  kde_column x;
  unsigned methods; /* KDE_METHOD_* bits; ROT is always computed */
  int stages;       /* plug-in stages, 2 or 3 */
  kde_grid grid;    /* LSCV grid */
} kde_request;

typedef struct {
  kde_status status;       /* per request */
  double sigma, h_rot, h_plugin, h_lscv;
  int32_t k_lscv;
  int at_edge;
  kde_plugin_info plugin;
  double* g_out;           /* caller-owned [n_h] for g(h), or NULL */
  double* gscale_out;      /* caller-owned [n_h], or NULL */
  double t_queue_s, t_service_s; /* served requests: time queued, time admitted to done */
  double lscv_evals_dense;  /* LSCV pair-term evaluations of the method: n(n-1)/2 * n_h */
  double lscv_evals;        /* of them performed (less with the "prune" option) */
} kde_result;

/* ---------------------------------------------------------------- resumable jobs
 * One request run on the caller's thread in slices of work, with checkpoints.
 * A job owns its column's device block and walks the request's work in a
 * fixed order (moments, plug-in stages, LSCV units, reductions, finalisation);
 * every work unit writes its own partial sums and each reduction runs in a
 * fixed order once its inputs are complete, so results are bitwise those of
 * the same request in kde_batch however the work is sliced, and a job
 * resumed from a checkpoint finishes with the results of an uninterrupted
 * one.  A job uses its context's stream and workspace: destroy it before the
 * context; while a server runs on the context, job calls return KDE_E_BUSY.
 * The options in force at kde_job_create (lscv_hc, lscv_mfma, prune,
 * fp64_kappa) stay the job's; a checkpoint carries its fp64_kappa and resumes
 * only in a job of the same precision, lscv_hc, lscv_mfma and prune. */
typedef struct kde_job kde_job;
/* Plans the request and copies its samples (host or device) and explicit grid
 * into the job's device block; the caller may free them on return.
 * KDE_E_INVAL for an invalid request. */
kde_status kde_job_create(kde_ctx* ctx, const kde_request* req, kde_job** out);
/* Runs the next work units until about max_evals pair-term evaluations are
 * issued (at least one unit), and synchronises.  *done_out (may be NULL) is 1
 * once the request is finished.  A device error makes the job unusable. */
kde_status kde_job_run(kde_job* job, double max_evals, int* done_out);
/* Pair-term evaluations issued so far and in all (any argument may be NULL). */
kde_status kde_job_progress(const kde_job* job, double* evals_done, double* evals_total, int* done_out);
/* The result of a finished job (as kde_poll fills it); KDE_E_BUSY before. */
kde_status kde_job_result(kde_job* job, kde_result* out);
/* Size of a checkpoint: a header, the column block (samples, working copies,
 * partial sums: about kde_request_footprint bytes) and the curve. */
kde_status kde_job_checkpoint_bytes(const kde_job* job, uint64_t* bytes);
/* Writes the job's cursor, device state and block into buf[bytes] (host). */
kde_status kde_job_checkpoint(kde_job* job, void* buf, uint64_t bytes);
/* Loads a checkpoint into a job created for a request of the same shape
 * (n, dtype, methods, stages, grid kind and size) on a context with the
 * same precision and options, before its first kde_job_run; the job then
 * continues the checkpointed request (its samples come with the
 * checkpoint).  KDE_E_INVAL for a foreign, truncated or mismatched buffer. */
kde_status kde_job_resume(kde_job* job, const void* buf, uint64_t bytes);
void kde_job_destroy(kde_job* job);

/* Device memory one request needs in a job or a server slot (its column
 * block: working copies of the samples, partial sums, grid, results), under
 * the options of ctx, or the defaults (mixed precision) when ctx is NULL.
 * Host-only: no device is touched, so it also runs without a GPU.  This is
 * the size the server's admission compares with its HBM budget.
 * KDE_E_INVAL for an invalid request (same checks as the calls that run it);
 * KDE_E_BUSY while a server runs on ctx. */
kde_status kde_request_footprint(const kde_ctx* ctx, const kde_request* req, uint64_t* bytes);

/* Work items of the pair triangle i < j of a column of n samples, as the
 * planner cuts it for the LSCV pass over an n_h-point grid (n_h > 0) or for a
 * plug-in stage (n_h = 0); Section 5.4 walks the same triangle in tiles.
 * Item k covers i in [row_begin[k], row_begin[k] + 256) and j in
 * [j_begin[k], j_end[k]) with j > i, holds pairs[k] such pairs, and the items
 * are ordered longest first.  seg: j-range per item as the "seg" option
 * (0 = whole rows, > 0 rounded up to a multiple of 512, < 0 = automatic under
 * the default launch size, lengthened when the pass would exceed 2^24 work
 * units).  Writes min(cap, count) items and sets *n_items = count.
 * Host-only.  KDE_E_INVAL for n outside [2, KDE_MAX_N], n_h outside
 * [0, KDE_MAX_NH], cap < 0, or NULL arrays with cap > 0. */
kde_status kde_plan_items(int64_t n, int32_t n_h, int64_t seg, int32_t cap, int32_t* n_items, int32_t* row_begin,
                          int32_t* j_begin, int32_t* j_end, double* pairs);

/* Run n_req (<= KDE_MAX_BATCH) requests as one job.  Per-request argument errors and degenerate
 * samples are reported in out[k].status (the other requests still run); a
 * degenerate plug-in chain does not stop the LSCV pass of the same request
 * (its h_lscv is still filled).  The call itself returns KDE_OK unless the
 * device fails or an argument of the call is invalid.  out[k].g_out / gscale_out, when not NULL, must hold n_h
 * doubles and are filled for LSCV requests. */
kde_status kde_batch(kde_ctx* ctx, const kde_request* reqs, int32_t n_req, kde_result* out);

/* ---------------------------------------------------------------- serving
 * A server runs on a context (one at a time; while it runs, the synchronous
 * calls and option setters of that context return KDE_E_BUSY).  The server
 * reserves hbm_budget_bytes of device memory when it starts (KDE_E_NOMEM if
 * the device cannot) and places every admitted request's block inside it.
 * Requests submitted from any thread queue in arrival order and are admitted
 * while the sum of the device footprints (kde_request_footprint) of admitted
 * requests stays within the budget and fewer than max_slots are resident (a
 * request larger than the whole budget is rejected with KDE_E_NOMEM).  The
 * first queued request that does not fit keeps its room: later requests are
 * admitted before it only within the rest of the budget, so it is admitted as
 * soon as enough resident work has finished.  Admitted requests stay resident
 * on the device (samples, partial sums, state) until done.  Continuous
 * batching: every scheduler iteration launches, in shared launches, the next
 * work units of every resident request, smallest remaining work first,
 * within the iteration's evaluation budget; requests admitted while others
 * run join the next iteration, and the next iteration is enqueued before the
 * previous one has ended.  Each result is bitwise identical to the same
 * request run alone through kde_batch. */
kde_status kde_server_start(kde_ctx* ctx, uint64_t hbm_budget_bytes, int32_t max_slots);
/* Copies the column (host or device) and grid; the caller may free them on
 * return.  Invalid requests are rejected here with KDE_E_INVAL. */
kde_status kde_submit(kde_ctx* ctx, const kde_request* req, uint64_t* ticket);
/* KDE_E_BUSY while pending.  When done, fills *out (out->g_out/gscale_out, if
 * not NULL, receive n_h values), forgets the ticket and returns KDE_OK; the
 * request's own outcome is out->status.  Unknown tickets give KDE_E_INVAL. */
kde_status kde_poll(kde_ctx* ctx, uint64_t ticket, kde_result* out);
/* As kde_poll, blocking up to timeout_s seconds (< 0: no limit). */
kde_status kde_wait(kde_ctx* ctx, uint64_t ticket, kde_result* out, double timeout_s);
/* Cancels one request: a queued one leaves the queue at once, an admitted one
 * leaves at the end of the scheduler iteration that is running (its slot and
 * budget are released); either way its result, collected by kde_poll or
 * kde_wait, has status KDE_E_CANCELLED.  A request that finishes in the
 * running iteration, or has finished, keeps its result.  KDE_E_INVAL for an
 * unknown (or already collected) ticket. */
kde_status kde_cancel(kde_ctx* ctx, uint64_t ticket);
/* Cancels queued requests (status KDE_E_CANCELLED), finishes admitted ones,
 * stops the scheduler thread.  Results not yet collected stay pollable until
 * the context is destroyed or a new server starts. */
kde_status kde_server_stop(kde_ctx* ctx);

/* Density estimate at query points, eq. (kde-def) with d = 1 and the
 * Gaussian kernel: f_out[k] = (n h)^-1 sum_i phi((points[k] - X_i) / h), for
 * a bandwidth h chosen by the selectors.  Mixed form: FP32 terms in
 * compensated 64-term runs, FP64 across pieces; FP64 form: FP64 terms.
 * points[m] and f_out[m] are host arrays.  KDE_E_INVAL for a bad column,
 * h <= 0 or not finite, m outside [1, KDE_MAX_QUERIES] or a non-finite point. */
kde_status kde_density(kde_ctx* ctx, kde_column x, double h, const double* points, int32_t m, double* f_out);

/* Approximate range aggregates from the estimate (Section 3.2, eq. (count)
 * and eq. (sum)), for ranges [lo[k], hi[k]] of the column's values:
 *   count_out[k] = n * int f = sum_i [Phi(beta_i) - Phi(alpha_i)],
 *   sum_out[k]   = n * int x f = sum_i [X_i (Phi(beta_i) - Phi(alpha_i)) + h (phi(alpha_i) - phi(beta_i))],
 *   avg_out[k]   = sum_out[k] / count_out[k]  (NaN when the count is 0),
 * alpha_i = (lo - X_i)/h, beta_i = (hi - X_i)/h: the Gaussian kernel
 * integrates in closed form, so no numerical quadrature is involved.  FP64,
 * differences of Phi taken between tails (erfc).  Infinite ends are allowed.
 * avg_out may be NULL.  KDE_E_INVAL for a bad column, h <= 0 or not finite,
 * q outside [1, KDE_MAX_QUERIES], a NaN end or lo > hi. */
kde_status kde_range_aggregates(kde_ctx* ctx, kde_column x, double h, const double* lo, const double* hi, int32_t q,
                                double* count_out, double* sum_out, double* avg_out);

/* A matrix of n d-dimensional samples, row-major (sample i occupies
 * data[i*d .. i*d + d)), float32 or float64, host or device memory. */
typedef struct {
  const void* data;
  int64_t n;
  int32_t d;
  kde_dtype dtype;
  int on_device;
} kde_matrix;

/* LSCV_h for d-dimensional samples, Section 4.4.2: the sphered objective
 *   g(h) = h^-d [2 n^-2 sum_{i<j} T~(X_i - X_j) + n^-1 R(K)],
 * T~ = (K*K)~ - 2 K~ of eq. (LSCV_MOD-Kv2)/(LSCV_MOD-KKv) through
 * S(v) = v^T Sigma^-1 v (eq. LSCV_MOD-Pv), Sigma the n-1 sample covariance,
 * R(K) = (4 pi)^(-d/2) |Sigma|^(-1/2) (eq. LSCV_MULTI-rk with H = Sigma); h is
 * in units of Sigma^(1/2).  S(v) is formed per pair from whitened samples
 * (Y = L^-1 (X - mean), Sigma = L L^T) and reused for every h, never stored.
 * h_grid == NULL: n_h points (150 if n_h <= 0) linear over [h0/4, 4 h0],
 * h0 = (4/((d+2) n))^(1/(d+4)).  g_out[n_h]; gscale_out, grid_out may be
 * NULL.  KDE_E_INVAL for a bad matrix (n < 2, d outside [1, KDE_MAX_D], a
 * non-finite value) or grid; KDE_E_DEGENERATE when Sigma is singular (a
 * Cholesky pivot at most 1e-12 of its diagonal entry). */
kde_status kde_lscv_md_curve(kde_ctx* ctx, kde_matrix x, const double* h_grid, int32_t n_h, double* g_out,
                             double* gscale_out, double* grid_out);
/* The grid point minimising the d-dimensional g(h), eq. (LSCV-finalH); ties
 * to the lowest index; k_out may be NULL. */
kde_status kde_bw_lscv_md(kde_ctx* ctx, kde_matrix x, const double* h_grid, int32_t n_h, double* h_out,
                          int32_t* k_out);

/* LSCV_H, Section 4.4.3: the objective at full bandwidth matrices,
 *   g(H) = 2 n^-2 sum_{i<j} [(K*K)_H - 2 K_H](X_i - X_j) + n^-1 R(K),
 * eq. (LSCV_MULTI-gh) with (LSCV_MULTI-KKx), (LSCV_MULTI-Kx), (LSCV_MULTI-rk):
 * (K*K)_H(v) = (4 pi)^(-d/2) |H|^(-1/2) exp(-v^T H^-1 v / 4),
 * K_H(v) = (2 pi)^(-d/2) |H|^(-1/2) exp(-v^T H^-1 v / 2),
 * R(K) = 2^-d pi^(-d/2) |H|^(-1/2); H in the units of the data (H = h^2 for
 * d = 1).  H holds m row-major d x d matrices, only their lower triangles are
 * read.  Each matrix gets a sweep of the pair triangle of its own over the
 * samples whitened for it, Z = L_G^-1 L^-1 (X - mean) with Sigma = L L^T and
 * G = L^-1 H L^-T = L_G L_G^T, so that v^T H^-1 v = |Z_i - Z_j|^2; a matrix's
 * g does not depend on the other matrices of the call.  g_out[m];
 * gscale_out (may be NULL) receives 2 n^-2 (A S1 + 2 B S2) + n^-1 R, the
 * scale of the terms.  A matrix that is not positive definite (a Cholesky
 * pivot at most 1e-12 of its diagonal entry) gets g = +inf and scale 0.  The
 * mixed form rounds Z to FP32 and takes FP32 exponentials; |H| is FP64.
 * KDE_E_INVAL for a bad matrix (n < 2, d outside [1, KDE_MAX_D], a
 * non-finite value), a non-finite entry of H or m outside [1, KDE_MAX_H_EVAL];
 * KDE_E_DEGENERATE when the sample covariance is singular. */
kde_status kde_lscv_H_eval(kde_ctx* ctx, kde_matrix x, const double* H, int32_t m, double* g_out,
                           double* gscale_out);
/* The same evaluation for a caller that evaluates g(H) many times over one
 * sample (its own optimiser over H): kde_lscv_H_prepare stages the samples
 * once (the moments, Sigma and its factor, the sphered working copy and the
 * pass layout of kde_lscv_H_eval) into a device buffer owned by the handle,
 * copying the samples in (host or device; the caller may free them on
 * return); kde_lscv_H_eval_prepared then gives g and its scale at m matrices
 * exactly as kde_lscv_H_eval does on the same sample, bitwise.  The handle
 * keeps its context (and must be released before it) and the precision the
 * context had at prepare: a later change of precision makes the evaluation
 * return KDE_E_INVAL.  Errors as for kde_lscv_H_eval; KDE_E_BUSY while a
 * server runs.  Calls with one handle must not overlap. */
typedef struct kde_lscv_H_prep kde_lscv_H_prep;
kde_status kde_lscv_H_prepare(kde_ctx* ctx, kde_matrix x, kde_lscv_H_prep** out);
kde_status kde_lscv_H_eval_prepared(kde_lscv_H_prep* prep, const double* H, int32_t m, double* g_out,
                                    double* gscale_out);
void kde_lscv_H_release(kde_lscv_H_prep* prep);

typedef struct {
  double g;          /* g(H_out) */
  int32_t evals;     /* evaluations of g */
  int32_t passes;    /* evaluation calls (a batch of matrices each) */
  int32_t converged; /* 1: both tolerances met; 0: stopped at max_evals */
  int32_t pad0;
} kde_lscv_H_info;
/* The LSCV_H bandwidth matrix (Section 4.4.3): Nelder-Mead minimisation of
 * g(H) over H = C C^T, C lower triangular with parameters theta = the lower
 * triangle row by row, log C_aa in place of each diagonal entry, so every
 * trial matrix is positive definite.  Start: the rule-of-thumb matrix of
 * eq. (LSCV-H-start) taken as the squared bandwidth s^2 Sigma,
 * s = (4/(d+2))^(1/(d+4)) n^(-1/(d+4)); initial steps 0.25 on each
 * log-diagonal parameter and 0.25 sqrt(C_aa C_bb) on an off-diagonal one;
 * reflection 1, expansion 2, contractions 1/2, shrink 1/2 towards the best
 * vertex.  Stops when max g - min g over the simplex is at most ftol |min g|
 * and every vertex lies within xtol of the best in every parameter, or after
 * max_evals evaluations.  The p + 1 starting vertices, and the p vertices of
 * a shrink, are evaluated in one call each.  H_out receives the best vertex's
 * matrix (row-major d x d); info may be NULL.  The mixed form's g carries
 * relative noise of about 1e-9 and below between nearby matrices, so an ftol
 * under that can run to max_evals.  Errors as kde_lscv_H_eval, and
 * KDE_E_INVAL for ftol or xtol not > 0 or max_evals < 1. */
kde_status kde_bw_lscv_H(kde_ctx* ctx, kde_matrix x, double ftol, double xtol, int32_t max_evals, double* H_out,
                         kde_lscv_H_info* info);

/* Density estimate with a bandwidth matrix at m query points, eq. (kde-def-H)
 * with K_H of eq. (K_H) and the Gaussian K of eq. (gaussian):
 *   f(p) = n^-1 sum_i (2 pi)^(-d/2) |H|^(-1/2) exp(-(p - X_i)^T H^-1 (p - X_i) / 2),
 * 1 <= d <= KDE_MAX_D; H row-major d x d (lower triangle read), covering the
 * three classes of eq. (3_classes_of_H) (h^2 I, diagonal, full; H = h^2
 * Sigma for the sphered LSCV_h bandwidth).  points: host array, row-major
 * m x d; f_out[m] host.  Samples and points are whitened by L_H^-1
 * (H = L_H L_H^T) in FP64; the squared distance is FP64 in both forms, the
 * mixed form takes its exponential in FP32.  KDE_E_INVAL for a bad matrix
 * (n < 1, d outside [1, KDE_MAX_D], a non-finite value), a non-finite
 * entry of H or point, or m outside [1, KDE_MAX_QUERIES]; KDE_E_DEGENERATE
 * when H is not positive definite (a Cholesky pivot at most 1e-12 of its
 * diagonal entry). */
kde_status kde_density_H(kde_ctx* ctx, kde_matrix x, const double* H, const double* points, int32_t m,
                         double* f_out);

/* Approximate 2-D range aggregates from the estimate of eq. (kde-def-H),
 * eq. (count-sum-2D): for boxes [a, b] x [c, d] (boxes: host array, q rows
 * of a, b, c, d; infinite ends allowed)
 *   count_out[k] = n * int int f,  sumx_out[k] = n * int int x f,
 *   sumy_out[k] = n * int int y f,  avgx_out[k] = sumx / count,
 *   avgy_out[k] = sumy / count (NaN when the count is 0; both may be NULL).
 * Per sample the kernel is a bivariate normal with mean X_i and covariance
 * H, so each term is a rectangle probability (four values of the bivariate
 * normal CDF through Owen's T function, 20-point Gauss-Legendre) and a
 * closed-form first moment; FP64, absolute error about 1e-16 of each
 * sample's unit mass.  x must have d = 2; H row-major 2 x 2, lower triangle
 * read.  KDE_E_INVAL for a bad matrix, a non-finite H, q outside
 * [1, KDE_MAX_QUERIES], a NaN end or an end pair out of order;
 * KDE_E_DEGENERATE when H is not positive definite. */
kde_status kde_range_aggregates_2d(kde_ctx* ctx, kde_matrix x, const double* H, const double* boxes, int32_t q,
                                   double* count_out, double* sumx_out, double* sumy_out, double* avgx_out,
                                   double* avgy_out);

/* LSCV bandwidth by a search instead of a fixed grid: the alternative to the
 * brute-force grid that Section 4.4.2 names (a golden-ratio type search).
 * Each step evaluates g(h) of eq. (LSCV-gh) at `points` bandwidths spaced
 * evenly in log h over the current bracket, ends included, in one pass of
 * the pair kernel (one pair distance for all of them); the bracket becomes
 * the two neighbours of the step's smallest g (ties to the lowest), so it
 * shrinks by 2/(points - 1) in log h per step, until its width hi/lo - 1 is
 * at most rel_tol.  h_out receives the bandwidth with the smallest g of the
 * last step.  On a g with several local minima the first step's spacing
 * decides which one is followed.  info (may be NULL) receives g there, the
 * steps, the bandwidths evaluated and the last bracket.  KDE_E_INVAL unless
 * 0 < h_lo < h_hi (finite), rel_tol > 0 and 4 <= points <= KDE_MAX_NH. */
typedef struct {
  double g;             /* g(h_out) */
  int32_t iterations;   /* search steps (kernel passes) */
  int32_t pad0;
  int64_t evaluated;    /* bandwidths evaluated in all */
  double bracket_lo, bracket_hi;
} kde_lscv_min_info;
kde_status kde_bw_lscv_min(kde_ctx* ctx, kde_column x, double h_lo, double h_hi, double rel_tol, int32_t points,
                           double* h_out, kde_lscv_min_info* info);

/* LSCV bandwidth: the grid point minimising g(h), eq. (LSCV-finalH); ties go
 * to the lowest index.  k_out (may be NULL) receives its index, at_edge (may
 * be NULL) 1 when it is the first or last grid point. */
kde_status kde_bw_lscv(kde_ctx* ctx, kde_column x, const double* h_grid, int32_t n_h, double* h_out,
                       int32_t* k_out, int* at_edge);

#ifdef __cplusplus
}
#endif

#endif /* KDE_BW_H */
