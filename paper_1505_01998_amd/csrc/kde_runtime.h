// kde_runtime.h -- host-side structures shared by the runtime and the server
// of the bandwidth-selection library.  Internal; the ABI is kde_bw.h.
#pragma once

#include <hip/hip_runtime.h>

#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "kde_bw.h"
#include "kde_internal.h"

namespace kde {

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;
};

// Work items of one column for one pass: blocks of the i < j triangle,
// longest first.
struct ColItems {
  std::vector<int> row, jb, je;
  std::vector<double> pairs;
};

struct UnitCost {
  double pairs;  // algorithmic i < j pairs of the unit's item
  double evals;  // pair-term evaluations of the unit
};

// Host plan of one column: its work decomposition (which depends only on n,
// the grid size and the context options, never on other columns) and the
// byte layout of its device block.
struct ColPlan {
  int n = 0;
  int f64 = 0;
  bool plugin = false, lscv = false;
  int stages = 0;  // 0 when no plug-in
  int hc = 16;
  int n_h = 0, n_chunks = 0;
  int grid_kind = 0;
  double grid_lo = 0.0, grid_hi = 0.0;
  std::vector<double> grid_h;  // explicit grid
  ColItems psi_items, lscv_items;
  // tile pruning (mixed form, LSCV): a sorted copy of the column, the first
  // j-tile of every row as "near" items, and per-chunk cut distances
  bool prune = false;
  ColItems near_items;
  size_t off_xs = 0, off_near_part = 0, off_near_sums = 0, off_d2cut = 0;
  // device block layout (byte offsets); raw holds the samples of a host column
  bool want_x64 = false;
  bool raw_in_block = false;
  size_t raw_bytes = 0, off_raw = 0;
  size_t off_y32 = 0, off_mm = 0;
  size_t off_x32 = 0, off_x64 = 0, off_stat = 0, off_nf = 0, off_psi_part = 0, off_psi_sums = 0, off_hin = 0,
         off_h = 0, off_c32 = 0, off_c64 = 0, off_part = 0, off_sums = 0, off_g = 0, off_gs = 0, bytes = 0;
};

// A sort of one column's padded FP32 copy (tile pruning).
struct SortJob {
  const float* in;
  float* out;
  int count;
};

// Everything one pass of the executor launches, in order: moments, the
// plug-in stages, the LSCV passes.  Column ids index `cols`.
struct Upload {
  void* dst;
  const void* src;
  size_t bytes;
};

struct IterPlan {
  std::vector<Upload> uploads;  // host-to-device copies issued before the launches
  std::vector<ColDesc> cols;
  std::vector<int> ids_stats;
  std::vector<int> ids_begin[3], ids_finish[3];
  std::vector<Unit> psi_units[3];
  std::vector<UnitCost> psi_cost[3];
  std::vector<RowDesc> psi_rows[3];
  std::vector<Unit> psi_cond_units[3];  // FP64 re-run (mixed form), of columns finishing the stage
  std::vector<UnitCost> psi_cond_cost[3];
  std::vector<int> ids_plugin_final;
  std::vector<int> ids_lscv_prep;
  std::vector<Unit> lscv_units;
  std::vector<UnitCost> lscv_cost;
  int lscv_groups[kQueueGroups + 1] = {};  // persistent form: group g is lscv_units [lscv_groups[g], [g + 1])
  std::vector<RowDesc> lscv_rows;
  std::vector<int> ids_lscv_final;
  // tile pruning: sorts, near-tile units and rows, cut preparation, pruned units
  std::vector<SortJob> sorts;
  std::vector<Unit> near_units;
  std::vector<UnitCost> near_cost;
  std::vector<RowDesc> near_rows;
  std::vector<int> ids_prune;
  std::vector<Unit> prune_units;
  std::vector<UnitCost> prune_cost;
  int max_stat_blocks = 1;
  void clear();
};

// Byte offsets of one executor pass's arrays in the device blob.
struct PassLayout {
  size_t o_cols = 0, o_stats = 0, o_pf = 0, o_lp = 0, o_lu = 0, o_lr = 0, o_lf = 0, bytes = 0;
  size_t o_nu = 0, o_nr = 0, o_pp = 0, o_pu = 0;  // tile pruning: near units/rows, prune ids, pruned units
  size_t sort_tmp = 0;                            // temporary bytes of the largest sort
  size_t o_ctr = 0;                               // work counters of the persistent launches (ints)
  size_t o_lg = 0;                                // group offsets of the persistent dense LSCV pass
  size_t o_begin[3] = {0, 0, 0}, o_finish[3] = {0, 0, 0}, o_psu[3] = {0, 0, 0}, o_pr[3] = {0, 0, 0},
         o_pc[3] = {0, 0, 0};
};

// Executable graph of a synchronous job (graph option): the job's kernel
// launches, captured once and replayed for later jobs of the same signature
// (request shapes, methods, grids and options).  Only launches are in the
// graph; inputs, the blob and the states are copied around it, so a replay
// sees new samples, grid values and device column addresses.  Jobs run one
// at a time on the context's stream, so graphs of different jobs share the
// context's device buffers.
struct JobGraph {
  std::string sig;
  uint64_t last_use = 0;
  hipGraphExec_t exec = nullptr;
  const void* blocks = nullptr;  // device buffers the graph's kernels address
  const void* st = nullptr;
  const void* blob = nullptr;
  const void* sort_tmp = nullptr;  // tile pruning: the sorts' temporary storage
  std::vector<ColPlan> plans;
  std::vector<int> plan_req;
  std::vector<ColDesc> cols;
  std::vector<char> blob_host;  // packed blob of the captured pass
  PassLayout L;
  void reset();
};

constexpr size_t kMaxGraphs = 8;
// Tile pruning: the skipped share of every pair sum is below this fraction
// of the sum (2^-34).
constexpr double kPruneEps = 5.820766091346741e-11;

// Variant of the LSCV pass chosen by the tile autotuner for one shape.
// Variants of the persistent dense LSCV sweep the autotuner chooses among:
// (bandwidths per block, samples per LDS tile); index 2 is the default.
constexpr int kQueueVariants = 5;
constexpr int kQueueHC[kQueueVariants] = {8, 16, 16, 16, 32};
constexpr int kQueueTJ[kQueueVariants] = {512, 256, 512, 1024, 512};
constexpr int kQueueDefault = 2;

struct TuneChoice {
  int hc = 16;  // bandwidths per block
  int tj = 512;  // samples per LDS tile
  double rate[kQueueVariants] = {0, 0, 0, 0, 0};  // measured evals/s of each variant (0: rejected)
  bool parity[kQueueVariants] = {true, true, true, true, true};  // partial sums bitwise equal to the default's
};

struct Server;
struct ServerDeleter {
  void operator()(Server* s) const;  // kde_server.hip
};
bool server_running(const Server* s);

}  // namespace kde

struct kde_ctx {
  int device = 0;
  kde_prec prec = KDE_PREC_MIXED;
  hipStream_t own = nullptr;
  hipStream_t stream = nullptr;
  std::string err;
  // options
  int opt_hc = 16;
  int64_t opt_seg = -1;            // <0 automatic, 0 whole rows, >0 explicit
  double opt_launch_evals = 4e12;  // pair-term evaluations per launch
  double opt_fp64_kappa = 1e3;
  int opt_mfma = 0;                // LSCV exponent arguments on the matrix cores (FP32, lscv_hc 16)
  double opt_serve_iter_evals = 1e12;  // server: pair-term evaluations per iteration (minimum)
  uint64_t opt_serve_fail_ticket = 0;  // server: the request whose pass is reported failed (0: none)
  double opt_serve_aging_s = 0.0;      // server: aging time constant of the SRPT order (0: plain SRPT)
  double opt_serve_iter_s = 0.0;       // server: target iteration duration (0: size by serve_iter_evals only)
  int opt_autotune = 0;            // synchronous jobs pick the LSCV variant with the tile autotuner
  int opt_graph = 0;               // synchronous jobs replay a captured graph of their launches
  int opt_prune = 0;               // LSCV tile pruning on sorted samples (mixed form, synchronous jobs)
  int opt_tj = 512;                // samples per LDS tile of the persistent dense sweep (256, 512, 1024)
  int opt_persistent = 1;          // dense FP32 LSCV pass as one persistent launch over a device work queue
  // resident blocks of the persistent LSCV kernel per variant (kde::kQueueVariants order; -1: not asked)
  int queue_blocks[5] = {-1, -1, -1, -1, -1};
  kde::DevBuf<char> sort_tmp;      // temporary storage of the column sorts
  kde::DevBuf<char> qbuf;          // query points / ranges, partials and outputs of the consumers
  kde::DevBuf<char> mdbuf;         // d-dimensional LSCV: samples, moments, whitened copy, partials
  std::vector<kde::JobGraph> graphs;  // at most kde::kMaxGraphs, least recently used replaced
  uint64_t graph_clock = 0;
  int64_t graph_captures = 0, graph_replays = 0;
  // prepared LSCV_H samples and resumable jobs created on this context;
  // kde_ctx_destroy releases those still alive
  std::vector<kde_lscv_H_prep*> preps;
  std::vector<kde_job*> jobs;
  // LSCV variant of the current job (from the options, or the autotuner)
  int job_hc = 16;
  int job_tj = 512;  // samples per LDS tile of the persistent dense sweep
  int job_mfma = 0;
  // autotuner: decisions per shape (quarter-octave bucket of n, n_h) and its trial buffer
  std::map<std::pair<int, int>, kde::TuneChoice> tune_cache;
  kde::DevBuf<char> tune_buf;
  // device workspace of synchronous jobs
  kde::DevBuf<char> stage;   // host columns copied in
  kde::DevBuf<char> blocks;  // per-column device blocks, packed
  kde::DevBuf<kde::DevState> st;
  kde::DevBuf<char> blob;    // column table, id lists, units, rows of one executor pass
  // pinned host staging
  kde::DevState* h_st = nullptr;
  size_t h_st_cap = 0;
  double* h_out = nullptr;
  size_t h_out_cap = 0;
  char* h_blob = nullptr;
  size_t h_blob_cap = 0;
  // plan of the current synchronous job (kept alive until its copies finish)
  std::vector<kde::ColPlan> plans;
  std::vector<int> plan_req;  // request index of each planned column
  kde::IterPlan iter;
  // set while a call runs on a fixed workspace (kde_lscv_curve_noalloc): a
  // device or pinned buffer that would have to grow fails instead
  bool no_alloc = false;
  // host staging of those calls (pageable; grown once, then reused)
  std::vector<kde::DevState> na_st;
  std::vector<double> na_out;
  std::vector<char> na_blob;
  // timing
  bool timing = false;
  int64_t t_launches[3] = {0, 0, 0};
  double t_ms[3] = {0, 0, 0};
  double t_evals[3] = {0, 0, 0};
  struct Pending {
    hipEvent_t a, b;
    int family;
    double evals;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> ev_pool;
  // server (null when not serving)
  std::unique_ptr<kde::Server, kde::ServerDeleter> server;
};

namespace kde {

// kernel families of the timing: LSCV pair kernels, psi pair kernels, and the
// d-dimensional pair kernels (LSCV_h, LSCV_H, density with a bandwidth matrix)
constexpr int kFamLscv = 0, kFamPsi = 1, kFamMd = 2;
// While timing is on, bracket the launches between the two calls with events
// on the context's stream (no-ops otherwise); p.family and p.evals name the
// family and the launches' pair-term evaluations.
kde_status timed_begin(kde_ctx* c, kde_ctx::Pending& p);
kde_status timed_end(kde_ctx* c, kde_ctx::Pending& p);

kde_status fail(kde_ctx* c, kde_status st, const std::string& msg);
kde_status status_of(int st);
std::string check_column(const kde_column& x);
std::string check_grid(const kde_grid& g);
// Argument check of one request (column, stages, grid); "" when valid.
std::string check_request(const kde_request& r);
// Bandwidths per block that LSCV work items are sized for, whatever variant runs.
constexpr int kSegRefHC = 16;
// Work items of a column of n samples for items of `seg` samples (0: whole rows).
void make_items(int64_t n, int64_t seg, ColItems& out);
// Item length of a pass whose blocks evaluate `hc` terms per pair.
int64_t pick_seg(const kde_ctx* c, int64_t n, int hc);
// Units a pass may hold before the planner lengthens its items.
constexpr double kMaxUnits = 16777216.0;
// pick_seg, lengthened while items x chunks would exceed kMaxUnits.
int64_t capped_seg(const kde_ctx* c, int64_t n, int hc, double chunks);
// Sets c->job_hc / job_mfma for a synchronous job over these requests: the
// options, or with the autotune option the tuned vector-ALU variant of the
// job's largest LSCV column (tuning that shape first when the job is large).
kde_status select_variant(kde_ctx* c, const kde_request* reqs, int32_t n_req);
// Stages one column on the device (validation, moments, the padded working
// copies) with a rule-of-thumb job and returns the device address of its
// descriptor, valid until the context's next job.  KDE_E_INVAL for a bad or
// non-finite column; a column of zero spread is staged (its DevState says so).
kde_status stage_column(kde_ctx* c, kde_column x, const ColDesc** dcol);
// Times the LSCV variants on a column of n samples and an n_h-point grid (or
// returns the cached decision for that shape).
kde_status tune_shape(kde_ctx* c, int64_t n, int n_h, TuneChoice& out);
// Fills the work decomposition and block layout of one request's column.
std::string plan_column(const kde_ctx* c, const kde_request& r, ColPlan& p);
// Points a descriptor at a column block; raw is the caller's device column
// (ignored when the plan keeps the samples in the block); st is its state.
void bind_column(const ColPlan& p, char* block, const void* raw, DevState* st, ColDesc& d);
// Appends a column's whole work (moments, every plug-in stage, the LSCV pass)
// to an executor plan; host_raw / host grid are uploaded into the block.
// extra_id: with tile pruning, the index of the column's two extra
// descriptors (near tiles, pruned sweep) in the pass's column table, else -1.
void add_full_column(const kde_ctx* c, const ColPlan& p, const ColDesc& d, int id, const void* host_raw,
                     IterPlan& it, int extra_id = -1);
// Tile pruning: the two extra descriptors of a pruned column (near tiles:
// sorted copy and near-tile slab; pruned sweep: sorted copy and main slab),
// and the column's set-up in a pass (sort, near-tile units and rows, cut
// preparation), with the descriptors at it.cols[extra_id], [extra_id + 1].
void prune_descs(const ColPlan& p, const ColDesc& d, ColDesc& nd, ColDesc& sd);
void add_prune_setup(const ColPlan& p, const ColDesc& d, int id, int extra_id, IterPlan& it);
// Pieces used by the server to schedule a column's work over several passes.
void psi_units_of(const ColPlan& p, int id, std::vector<Unit>& u, std::vector<UnitCost>& cost);
void lscv_units_of(const ColPlan& p, int id, std::vector<Unit>& u, std::vector<UnitCost>& cost);
void psi_rows_of(const ColPlan& p, const ColDesc& d, std::vector<RowDesc>& rows);
void lscv_rows_of(const ColPlan& p, const ColDesc& d, std::vector<RowDesc>& rows);
void init_state(const ColPlan& p, double fp64_kappa, DevState& h);
// Resets r (keeping its g/gscale pointers): h's NaN, k_lscv -1, status st.
void init_result(kde_result& r, kde_status st);
// Copies a finished column's scalar results (status, h's, plug-in info) into r.
void fill_result(const ColPlan& p, const DevState& h, kde_result& r);
// Enqueues one executor pass on the context's stream (no synchronisation):
// pack_pass sorts the units and packs the blob in pinned memory,
// upload_pass copies inputs and the blob, launch_pass enqueues the kernels
// (launches only, so it can be captured into a graph).
kde_status pack_pass(kde_ctx* c, IterPlan& it, PassLayout& L);
kde_status upload_pass(kde_ctx* c, const IterPlan& it, const PassLayout& L);
kde_status launch_pass(kde_ctx* c, const IterPlan& it, const PassLayout& L);
kde_status execute(kde_ctx* c, IterPlan& it);
// Blocks the device holds at once of the persistent dense LSCV sweep's
// variant (hc, tj), cached per context (0: no such variant or no answer).
int queue_blocks(kde_ctx* c, int hc, int tj);
// Whether the dense LSCV pass of an executor plan runs as one persistent launch.
bool lscv_queue_form(kde_ctx* c, const IterPlan& it);
// The LSCV curve of one column as kde_lscv_curve computes it (job, copies of
// g, gscale and the grid into the caller's arrays, synchronisation).
kde_status lscv_curve_call(kde_ctx* c, kde_column x, const double* h_grid, int32_t n_h, double* g_out,
                           double* gscale_out, double* grid_out);
// Looks up, once per device, the device address of the fixed scratch of
// kde_lscv_curve_noalloc (the context's device must be current).
void noalloc_setup(kde_ctx* c);
kde_status sync_and_check(kde_ctx* c);
// Folds the timed launches that have completed into the counters (no wait).
kde_status collect_ready_timing(kde_ctx* c);
kde_status ensure_pinned_bytes(kde_ctx* c, char*& p, size_t& cap, size_t bytes);

// Grows a device buffer to hold at least `count` elements (contents are lost).
template <typename T>
kde_status ensure(kde_ctx* c, DevBuf<T>& b, size_t count) {
  if (b.cap >= count) return KDE_OK;
  if (c->no_alloc) return fail(c, KDE_E_NOMEM, "request needs more device workspace than the fixed scratch holds");
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
  const size_t want = count < 256 ? 256 : count;
  hipError_t e = hipMalloc((void**)&b.p, want * sizeof(T));
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(c, KDE_E_NOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
  }
  b.cap = want;
  return KDE_OK;
}

}  // namespace kde

#define KDE_HIP_TRY(ctx, expr)                                                                                \
  do {                                                                                                        \
    hipError_t e_ = (expr);                                                                                   \
    if (e_ != hipSuccess)                                                                                     \
      return ::kde::fail((ctx), KDE_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_));             \
  } while (0)
