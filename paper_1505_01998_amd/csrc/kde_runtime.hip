// kde_runtime.hip -- host runtime and C ABI of the bandwidth-selection library.
//
// Every call is a job over a set of columns (one for the single-column
// selectors, many for kde_batch).  A job is a chain of kernels on one stream:
// moments for all columns (FP64, two passes), the device-side scalar steps of
// the selectors, the pair kernels over work units that mix columns (split into
// launches of bounded work), fixed-order FP64 segmented reductions and the
// finalize kernels; one round of device-to-host copies returns the results.
// No step of the method runs on the host: the host checks arguments and plans
// the work units.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kde_bw.h"
#include "kde_internal.h"

using kde::ColDesc;
using kde::DevState;
using kde::RowDesc;
using kde::Unit;

namespace {

struct Pending {
  hipEvent_t a, b;
  int family;
  double evals;
};

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;
};

// Work items of one column for one pass: blocks of the i < j triangle.
struct ColItems {
  std::vector<int> row, jb, je;
  std::vector<double> pairs;
};

// One column of a job as the host plans it.
struct JobCol {
  int req;            // index of the request it came from
  const void* data;   // caller's samples (host or device)
  int on_device;
  int n;
  int f64;
  bool plugin, lscv;
  int stages;
  kde_grid grid;
  ColDesc d;          // device descriptor (raw pointer filled at run time)
  ColItems lscv_items, psi_items;
};

struct UnitCost {
  double pairs;   // algorithmic i<j pairs of the unit's item
  double evals;   // pair-term evaluations of the unit
};

}  // namespace

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
  // device workspace
  DevBuf<char> stage;
  DevBuf<float> x32;
  DevBuf<double> x64;
  DevBuf<double> part;
  DevBuf<int> part_nf;
  DevBuf<double> stat_part;
  DevBuf<double> psi_sums, lscv_sums;
  DevBuf<double> hin, hdev, c64, g, gs;
  DevBuf<float> c32;
  DevBuf<ColDesc> cols;
  DevBuf<Unit> units;
  DevBuf<RowDesc> rows;
  DevBuf<DevState> st;
  // pinned host staging
  DevState* h_st = nullptr;
  size_t h_st_cap = 0;
  double* h_out = nullptr;
  size_t h_out_cap = 0;
  // host-side plan of the current job (kept alive until the job's copies finish)
  std::vector<JobCol> jcols;
  std::vector<ColDesc> h_cols;
  std::vector<Unit> h_units;       // psi units, then LSCV units
  std::vector<UnitCost> h_cost;
  std::vector<RowDesc> h_rows;     // psi rows, then LSCV rows
  std::vector<double> h_hin;
  size_t n_psi_units = 0, n_lscv_units = 0, n_psi_rows = 0, n_lscv_rows = 0;
  // timing
  bool timing = false;
  int64_t t_launches[2] = {0, 0};
  double t_ms[2] = {0, 0};
  double t_evals[2] = {0, 0};
  std::vector<Pending> pending;
  std::vector<hipEvent_t> ev_pool;
};

namespace {

constexpr int kFamLscv = 0, kFamPsi = 1;

kde_status fail(kde_ctx* c, kde_status st, const std::string& msg) {
  c->err = msg;
  return st;
}

#define HIP_TRY(ctx, expr)                                                                                    \
  do {                                                                                                        \
    hipError_t e_ = (expr);                                                                                   \
    if (e_ != hipSuccess) return fail((ctx), KDE_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
kde_status ensure(kde_ctx* c, DevBuf<T>& b, size_t count) {
  if (b.cap >= count) return KDE_OK;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
  size_t want = std::max<size_t>(count, 256);
  hipError_t e = hipMalloc((void**)&b.p, want * sizeof(T));
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(c, KDE_E_NOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
  }
  b.cap = want;
  return KDE_OK;
}

template <typename T>
kde_status ensure_pinned(kde_ctx* c, T*& p, size_t& cap, size_t count) {
  if (cap >= count) return KDE_OK;
  if (p) (void)hipHostFree(p);
  p = nullptr;
  cap = 0;
  size_t want = std::max<size_t>(count, 64);
  if (hipHostMalloc((void**)&p, want * sizeof(T), hipHostMallocDefault) != hipSuccess) {
    p = nullptr;
    return fail(c, KDE_E_NOMEM, "pinned host allocation failed");
  }
  cap = want;
  return KDE_OK;
}

kde_status status_of(int st) {
  switch (st) {
    case kde::kStOk: return KDE_OK;
    case kde::kStInval: return KDE_E_INVAL;
    case kde::kStDegenerate: return KDE_E_DEGENERATE;
    default: return KDE_E_DEVICE;
  }
}

kde_status map_status(kde_ctx* c, int st) {
  switch (st) {
    case kde::kStOk: return KDE_OK;
    case kde::kStInval: return fail(c, KDE_E_INVAL, "sample column holds a non-finite value");
    case kde::kStDegenerate:
      return fail(c, KDE_E_DEGENERATE,
                  "degenerate sample: zero spread, or a functional estimate with the wrong sign");
    default: return fail(c, KDE_E_DEVICE, "unknown device status");
  }
}

// ---- timing
kde_status timed_begin(kde_ctx* c, Pending& p) {
  if (!c->timing) return KDE_OK;
  for (hipEvent_t* e : {&p.a, &p.b}) {
    if (!c->ev_pool.empty()) {
      *e = c->ev_pool.back();
      c->ev_pool.pop_back();
    } else {
      HIP_TRY(c, hipEventCreate(e));
    }
  }
  HIP_TRY(c, hipEventRecord(p.a, c->stream));
  return KDE_OK;
}

kde_status timed_end(kde_ctx* c, Pending& p) {
  if (!c->timing) return KDE_OK;
  HIP_TRY(c, hipEventRecord(p.b, c->stream));
  c->pending.push_back(p);
  return KDE_OK;
}

// Called after the stream has been synchronised.
kde_status collect_timing(kde_ctx* c) {
  for (Pending& p : c->pending) {
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, p.a, p.b));
    c->t_launches[p.family] += 1;
    c->t_ms[p.family] += ms;
    c->t_evals[p.family] += p.evals;
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->pending.clear();
  return KDE_OK;
}

kde_status sync_and_check(kde_ctx* c) {
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return collect_timing(c);
}

// ---- argument checks
std::string check_column(const kde_column& x) {
  if (!x.data) return "column data is NULL";
  if (x.n < 2) return "a sample column needs n >= 2";
  if (x.n > KDE_MAX_N) return "n exceeds KDE_MAX_N";
  if (x.dtype != KDE_F32 && x.dtype != KDE_F64) return "dtype must be KDE_F32 or KDE_F64";
  return "";
}

std::string check_grid(const kde_grid& g) {
  if (g.n_h < 1 || g.n_h > KDE_MAX_NH) return "n_h out of range";
  if (g.kind == KDE_GRID_EXPLICIT) {
    if (!g.h) return "explicit grid is NULL";
    for (int32_t k = 0; k < g.n_h; ++k) {
      if (!(g.h[k] > 0.0) || !std::isfinite(g.h[k])) return "grid values must be finite and > 0";
      if (k > 0 && !(g.h[k] > g.h[k - 1])) return "grid must be strictly ascending";
    }
  } else if (g.kind == KDE_GRID_LOG_ROT) {
    if (!(g.lo > 0.0) || !(g.hi > g.lo) || !std::isfinite(g.hi)) return "log grid needs 0 < lo < hi";
  } else if (g.kind != KDE_GRID_PAPER) {
    return "unknown grid kind";
  }
  return "";
}

// ---- work items
double item_pairs(int64_t n, int64_t row, int64_t jb, int64_t je) {
  const int64_t i0 = row * kde::kBI;
  const int64_t i1 = std::min<int64_t>(n, i0 + kde::kBI);
  je = std::min<int64_t>(je, n);
  double p = 0.0;
  for (int64_t i = i0; i < i1; ++i) {
    const int64_t b = std::max<int64_t>(jb, i + 1);
    if (je > b) p += (double)(je - b);
  }
  return p;
}

// Items of one column: row r sweeps j in [r*kBI, n) rounded up to kBJ, cut
// into pieces of `seg` samples (0: one piece).  Ordered longest first.
void make_items(int64_t n, int64_t seg, ColItems& out) {
  std::vector<int> row, jb, je;
  std::vector<double> pr;
  const int64_t rows = (n + kde::kBI - 1) / kde::kBI;
  for (int64_t r = 0; r < rows; ++r) {
    const int64_t row0 = r * kde::kBI;
    const int64_t len = ((n - row0) + kde::kBJ - 1) / kde::kBJ * kde::kBJ;
    const int64_t step = seg > 0 ? seg : len;
    for (int64_t b = row0; b < row0 + len; b += step) {
      const int64_t e = std::min(b + step, row0 + len);
      const double p = item_pairs(n, r, b, e);
      if (p <= 0.0) continue;
      row.push_back((int)r);
      jb.push_back((int)b);
      je.push_back((int)e);
      pr.push_back(p);
    }
  }
  std::vector<size_t> order(pr.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return pr[a] > pr[b]; });
  out.row.resize(order.size());
  out.jb.resize(order.size());
  out.je.resize(order.size());
  out.pairs.resize(order.size());
  for (size_t k = 0; k < order.size(); ++k) {
    out.row[k] = row[order[k]];
    out.jb[k] = jb[order[k]];
    out.je[k] = je[order[k]];
    out.pairs[k] = pr[order[k]];
  }
}

// Item length for a pass whose blocks each evaluate `hc` terms per pair.  It
// depends only on n and the context options, never on the rest of a batch.
int64_t pick_seg(const kde_ctx* c, int64_t n, int hc) {
  if (c->opt_seg >= 0) return c->opt_seg == 0 ? 0 : (c->opt_seg + kde::kBJ - 1) / kde::kBJ * kde::kBJ;
  // Aim for ~8192 blocks per launch so each launch fills the chip many times.
  const double per_block_pairs = c->opt_launch_evals / 8192.0 / (double)hc;
  int64_t seg = (int64_t)(per_block_pairs / kde::kBI);
  seg = std::max<int64_t>(kde::kBJ, seg / kde::kBJ * kde::kBJ);
  if (seg >= n) return 0;
  return seg;
}

int lscv_hc(const kde_ctx* c) { return c->prec == KDE_PREC_FP64 ? 8 : c->opt_hc; }

// Plans a job from the requests: columns, offsets, work units and reduction
// rows.  Requests with bad arguments get status INVAL in `st` and no column.
void plan_job(kde_ctx* c, const kde_request* reqs, int32_t n_req, std::vector<kde_status>& st,
              std::vector<std::string>& msg) {
  c->jcols.clear();
  c->h_cols.clear();
  c->h_units.clear();
  c->h_cost.clear();
  c->h_rows.clear();
  c->h_hin.clear();
  const int hc = lscv_hc(c);
  st.assign(n_req, KDE_OK);
  msg.assign(n_req, "");
  int64_t x_off = 0, c_off = 0, part_off = 0;
  for (int32_t k = 0; k < n_req; ++k) {
    const kde_request& r = reqs[k];
    std::string e = check_column(r.x);
    const bool plugin = (r.methods & KDE_METHOD_PLUGIN) != 0;
    const bool lscv = (r.methods & KDE_METHOD_LSCV) != 0;
    if (e.empty() && plugin && r.stages != 2 && r.stages != 3) e = "stages must be 2 or 3";
    if (e.empty() && lscv) e = check_grid(r.grid);
    if (!e.empty()) {
      st[k] = KDE_E_INVAL;
      msg[k] = e;
      continue;
    }
    JobCol jc;
    jc.req = k;
    jc.data = r.x.data;
    jc.on_device = r.x.on_device;
    jc.n = (int)r.x.n;
    jc.f64 = r.x.dtype == KDE_F64;
    jc.plugin = plugin;
    jc.lscv = lscv;
    jc.stages = plugin ? r.stages : 2;
    jc.grid = r.grid;
    std::memset(&jc.d, 0, sizeof(jc.d));
    jc.d.n = jc.n;
    jc.d.raw_f64 = jc.f64;
    jc.d.x_off = x_off;
    x_off += ((int64_t)jc.n + kde::kPad + 63) / 64 * 64;
    if (plugin) {
      make_items(jc.n, pick_seg(c, jc.n, 1), jc.psi_items);
      jc.d.n_items_psi = (int)jc.psi_items.pairs.size();
      jc.d.psi_part_off = part_off;
      part_off += 2 * (int64_t)jc.d.n_items_psi;
    }
    if (lscv) {
      make_items(jc.n, pick_seg(c, jc.n, hc), jc.lscv_items);
      jc.d.n_h = r.grid.n_h;
      jc.d.n_chunks = (r.grid.n_h + hc - 1) / hc;
      jc.d.n_items = (int)jc.lscv_items.pairs.size();
      jc.d.c_off = c_off;
      c_off += (int64_t)jc.d.n_chunks * hc;
      jc.d.part_off = part_off;
      part_off += 2 * (int64_t)r.grid.n_h * jc.d.n_items;
      jc.d.grid_kind = (int)r.grid.kind;
      jc.d.grid_lo = r.grid.lo;
      jc.d.grid_hi = r.grid.hi;
    }
    c->jcols.push_back(std::move(jc));
  }
  const int n_cols = (int)c->jcols.size();
  // explicit grids, at each column's c_off
  c->h_hin.assign((size_t)std::max<int64_t>(c_off, 1), 0.0);
  for (const JobCol& jc : c->jcols)
    if (jc.lscv && jc.grid.kind == KDE_GRID_EXPLICIT)
      std::memcpy(c->h_hin.data() + jc.d.c_off, jc.grid.h, sizeof(double) * jc.grid.n_h);
  struct Tmp {
    Unit u;
    UnitCost cost;
  };
  // psi units of all columns, largest first
  std::vector<Tmp> tmp;
  for (int col = 0; col < n_cols; ++col) {
    const JobCol& jc = c->jcols[col];
    if (!jc.plugin) continue;
    for (size_t it = 0; it < jc.psi_items.pairs.size(); ++it) {
      Tmp t;
      t.u = Unit{col, jc.psi_items.row[it], jc.psi_items.jb[it], jc.psi_items.je[it], (int)it, 0};
      t.cost = UnitCost{jc.psi_items.pairs[it], jc.psi_items.pairs[it]};
      tmp.push_back(t);
    }
  }
  std::stable_sort(tmp.begin(), tmp.end(), [](const Tmp& a, const Tmp& b) { return a.cost.pairs > b.cost.pairs; });
  for (const Tmp& t : tmp) {
    c->h_units.push_back(t.u);
    c->h_cost.push_back(t.cost);
  }
  c->n_psi_units = tmp.size();
  // LSCV units: item-major, chunks inner, largest items first
  tmp.clear();
  for (int col = 0; col < n_cols; ++col) {
    const JobCol& jc = c->jcols[col];
    if (!jc.lscv) continue;
    for (size_t it = 0; it < jc.lscv_items.pairs.size(); ++it)
      for (int ch = 0; ch < jc.d.n_chunks; ++ch) {
        Tmp t;
        t.u = Unit{col, jc.lscv_items.row[it], jc.lscv_items.jb[it], jc.lscv_items.je[it], (int)it, ch};
        const int valid = std::min(hc, jc.d.n_h - ch * hc);
        t.cost = UnitCost{jc.lscv_items.pairs[it], jc.lscv_items.pairs[it] * valid};
        tmp.push_back(t);
      }
  }
  std::stable_sort(tmp.begin(), tmp.end(), [](const Tmp& a, const Tmp& b) { return a.cost.pairs > b.cost.pairs; });
  for (const Tmp& t : tmp) {
    c->h_units.push_back(t.u);
    c->h_cost.push_back(t.cost);
  }
  c->n_lscv_units = tmp.size();
  // reduction rows
  for (int col = 0; col < n_cols; ++col) {
    const JobCol& jc = c->jcols[col];
    if (!jc.plugin) continue;
    for (int w = 0; w < 2; ++w)
      c->h_rows.push_back(RowDesc{jc.d.psi_part_off + (int64_t)w * jc.d.n_items_psi, 2 * (int64_t)col + w,
                                  jc.d.n_items_psi, 0});
  }
  c->n_psi_rows = c->h_rows.size();
  for (int col = 0; col < n_cols; ++col) {
    const JobCol& jc = c->jcols[col];
    if (!jc.lscv) continue;
    for (int r = 0; r < 2 * jc.d.n_h; ++r)
      c->h_rows.push_back(RowDesc{jc.d.part_off + (int64_t)r * jc.d.n_items, 2 * jc.d.c_off + r, jc.d.n_items, 0});
  }
  c->n_lscv_rows = c->h_rows.size() - c->n_psi_rows;
}

int64_t job_part_size(const kde_ctx* c) {
  int64_t m = 0;
  for (const JobCol& jc : c->jcols) {
    if (jc.plugin) m = std::max(m, jc.d.psi_part_off + 2 * (int64_t)jc.d.n_items_psi);
    if (jc.lscv) m = std::max(m, jc.d.part_off + 2 * (int64_t)jc.d.n_h * jc.d.n_items);
  }
  return m;
}

int64_t job_x_size(const kde_ctx* c) {
  int64_t m = 0;
  for (const JobCol& jc : c->jcols) m = std::max(m, jc.d.x_off + (int64_t)jc.n + kde::kPad);
  return m;
}

int64_t job_c_size(const kde_ctx* c, int hc) {
  int64_t m = 0;
  for (const JobCol& jc : c->jcols)
    if (jc.lscv) m = std::max(m, jc.d.c_off + (int64_t)jc.d.n_chunks * hc);
  return m;
}

// Launch ranges over units [u0, u1) of one pass whose summed evaluations stay
// within budget (at least 2048 blocks per launch when the pass has them, so a
// launch fills the chip).  FP64 terms cost about five times the FP32 ones.
template <typename F>
kde_status for_each_launch(kde_ctx* c, size_t first, size_t count, bool f64, F&& launch) {
  const double budget = f64 ? c->opt_launch_evals / 5.0 : c->opt_launch_evals;
  size_t u0 = first;
  const size_t end = first + count;
  while (u0 < end) {
    double acc = c->h_cost[u0].evals;
    size_t u1 = u0 + 1;
    while (u1 < end && (acc + c->h_cost[u1].evals <= budget || u1 - u0 < 2048)) {
      acc += c->h_cost[u1].evals;
      ++u1;
    }
    kde_status s = launch((int)u0, (int)(u1 - u0), acc);
    if (s) return s;
    u0 = u1;
  }
  return KDE_OK;
}

kde_status run_psi_stage(kde_ctx* c, int n_cols, int stage, bool f64, bool conditional) {
  const int r = 8 - 2 * stage;
  kde_status s = for_each_launch(c, 0, c->n_psi_units, f64, [&](int u0, int cnt, double evals) -> kde_status {
    // A conditional pass may exit at once on the device, so it is not timed.
    Pending pd{nullptr, nullptr, kFamPsi, evals};
    kde_status s2 = conditional ? KDE_OK : timed_begin(c, pd);
    if (s2) return s2;
    kde::launch_psi_units(c->stream, r, f64 ? 1 : 0, conditional ? 1 : 0, c->x32.p, c->x64.p, c->cols.p,
                          c->units.p, u0, cnt, c->part.p, c->st.p);
    return conditional ? KDE_OK : timed_end(c, pd);
  });
  if (s) return s;
  kde::launch_reduce_rows(c->stream, c->part.p, c->rows.p, (int)c->n_psi_rows, c->psi_sums.p);
  kde::launch_psi_finish(c->stream, n_cols, c->cols.p, c->st.p, stage, c->psi_sums.p, f64 ? 1 : 0,
                         conditional ? 1 : 0);
  HIP_TRY(c, hipGetLastError());
  return KDE_OK;
}

// Enqueues the whole job planned by plan_job.  Results stay on the device
// except the per-column states, whose copy back is enqueued last.
kde_status run_job(kde_ctx* c) {
  kde_status s;
  const int n_cols = (int)c->jcols.size();
  if (n_cols == 0) return KDE_OK;
  const bool all64 = c->prec == KDE_PREC_FP64;
  const int hc = lscv_hc(c);
  bool any_plugin = false, any_lscv = false;
  int max_stages = 2;
  for (const JobCol& jc : c->jcols) {
    any_plugin |= jc.plugin;
    any_lscv |= jc.lscv;
    if (jc.plugin) max_stages = std::max(max_stages, jc.stages);
  }
  const bool want_x64 = all64 || (any_plugin && c->opt_fp64_kappa > 0.0);
  // stage host columns on the device
  size_t stage_bytes = 0;
  for (const JobCol& jc : c->jcols)
    if (!jc.on_device) stage_bytes += ((size_t)jc.n * (jc.f64 ? 8 : 4) + 255) / 256 * 256;
  if ((s = ensure(c, c->stage, std::max<size_t>(stage_bytes, 1)))) return s;
  size_t so = 0;
  for (JobCol& jc : c->jcols) {
    if (jc.on_device) {
      jc.d.raw = jc.data;
    } else {
      const size_t bytes = (size_t)jc.n * (jc.f64 ? 8 : 4);
      HIP_TRY(c, hipMemcpyAsync(c->stage.p + so, jc.data, bytes, hipMemcpyHostToDevice, c->stream));
      jc.d.raw = c->stage.p + so;
      so += (bytes + 255) / 256 * 256;
    }
  }
  c->h_cols.resize(n_cols);
  for (int k = 0; k < n_cols; ++k) c->h_cols[k] = c->jcols[k].d;
  // buffers
  const int64_t xs = job_x_size(c), cs = std::max<int64_t>(job_c_size(c, hc), 1);
  if ((s = ensure(c, c->x32, (size_t)xs))) return s;
  if (want_x64 && (s = ensure(c, c->x64, (size_t)xs))) return s;
  if ((s = ensure(c, c->stat_part, (size_t)n_cols * kde::kStatBlocks))) return s;
  if ((s = ensure(c, c->part_nf, (size_t)n_cols * kde::kStatBlocks))) return s;
  if ((s = ensure(c, c->part, (size_t)std::max<int64_t>(job_part_size(c), 1)))) return s;
  if ((s = ensure(c, c->psi_sums, (size_t)2 * n_cols))) return s;
  if ((s = ensure(c, c->lscv_sums, (size_t)2 * cs))) return s;
  for (auto* b : {&c->hin, &c->hdev, &c->c64, &c->g, &c->gs})
    if ((s = ensure(c, *b, (size_t)cs))) return s;
  if ((s = ensure(c, c->c32, (size_t)cs))) return s;
  if ((s = ensure(c, c->cols, (size_t)n_cols))) return s;
  if ((s = ensure(c, c->units, std::max<size_t>(c->h_units.size(), 1)))) return s;
  if ((s = ensure(c, c->rows, std::max<size_t>(c->h_rows.size(), 1)))) return s;
  if ((s = ensure(c, c->st, (size_t)n_cols))) return s;
  if ((s = ensure_pinned(c, c->h_st, c->h_st_cap, (size_t)n_cols))) return s;
  // initial per-column state
  for (int k = 0; k < n_cols; ++k) {
    DevState& h = c->h_st[k];
    std::memset(&h, 0, sizeof(h));
    const double nan = std::nan("");
    h.stages = c->jcols[k].plugin ? c->jcols[k].stages : 0;
    for (int q = 0; q < 3; ++q) {
      h.g[q] = h.psi[q] = h.kappa[q] = nan;
      h.prec_used[q] = -1;
    }
    h.h_plugin = h.h_best = h.margin = nan;
    h.k_best = -1;
    h.fp64_kappa = c->opt_fp64_kappa;
  }
  HIP_TRY(c, hipMemcpyAsync(c->st.p, c->h_st, sizeof(DevState) * n_cols, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->cols.p, c->h_cols.data(), sizeof(ColDesc) * n_cols, hipMemcpyHostToDevice,
                            c->stream));
  if (!c->h_units.empty())
    HIP_TRY(c, hipMemcpyAsync(c->units.p, c->h_units.data(), sizeof(Unit) * c->h_units.size(),
                              hipMemcpyHostToDevice, c->stream));
  if (!c->h_rows.empty())
    HIP_TRY(c, hipMemcpyAsync(c->rows.p, c->h_rows.data(), sizeof(RowDesc) * c->h_rows.size(),
                              hipMemcpyHostToDevice, c->stream));
  // moments of every column
  int max_blocks = 1;
  for (const JobCol& jc : c->jcols)
    max_blocks = std::max(max_blocks, std::min(kde::kStatBlocks, (jc.n + 2047) / 2048));
  kde::launch_stats(c->stream, n_cols, max_blocks, c->cols.p, c->stat_part.p, c->part_nf.p, c->x32.p,
                    want_x64 ? c->x64.p : nullptr, c->st.p);
  HIP_TRY(c, hipGetLastError());
  // plug-in stages (columns without the plug-in have no psi units; their
  // scalar steps run harmlessly and are not reported)
  if (any_plugin) {
    for (int stage = (max_stages == 3 ? 0 : 1); stage < 3; ++stage) {
      kde::launch_psi_begin(c->stream, n_cols, c->st.p, stage);
      if ((s = run_psi_stage(c, n_cols, stage, all64, false))) return s;
      if (!all64 && c->opt_fp64_kappa > 0.0 && (s = run_psi_stage(c, n_cols, stage, true, true))) return s;
    }
    kde::launch_plugin_final(c->stream, n_cols, c->st.p);
  }
  // LSCV
  if (any_lscv) {
    HIP_TRY(c, hipMemcpyAsync(c->hin.p, c->h_hin.data(), sizeof(double) * c->h_hin.size(), hipMemcpyHostToDevice,
                              c->stream));
    kde::launch_lscv_prep(c->stream, n_cols, hc, c->cols.p, c->hin.p, c->st.p, c->hdev.p, c->c32.p, c->c64.p);
    s = for_each_launch(c, c->n_psi_units, c->n_lscv_units, all64,
                        [&](int u0, int cnt, double evals) -> kde_status {
                          Pending pd{nullptr, nullptr, kFamLscv, evals};
                          kde_status s2 = timed_begin(c, pd);
                          if (s2) return s2;
                          kde::launch_lscv_units(c->stream, hc, all64 ? 1 : 0, c->x32.p, c->x64.p, c->cols.p,
                                                 c->units.p, u0, cnt, c->c32.p, c->c64.p, c->part.p, c->st.p);
                          return timed_end(c, pd);
                        });
    if (s) return s;
    kde::launch_reduce_rows(c->stream, c->part.p, c->rows.p + c->n_psi_rows, (int)c->n_lscv_rows, c->lscv_sums.p);
    kde::launch_lscv_finalize(c->stream, n_cols, c->cols.p, c->lscv_sums.p, c->hdev.p, c->st.p, c->g.p, c->gs.p);
  }
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipMemcpyAsync(c->h_st, c->st.p, sizeof(DevState) * n_cols, hipMemcpyDeviceToHost, c->stream));
  return KDE_OK;
}

// Single-column helpers ------------------------------------------------------
kde_status run_single(kde_ctx* c, const kde_request& r) {
  std::vector<kde_status> st;
  std::vector<std::string> msg;
  plan_job(c, &r, 1, st, msg);
  if (st[0] != KDE_OK) return fail(c, st[0], msg[0]);
  return run_job(c);
}

kde_request make_req(kde_column x, unsigned methods, int stages, const double* h_grid, int32_t n_h) {
  kde_request r;
  std::memset(&r, 0, sizeof(r));
  r.x = x;
  r.methods = methods;
  r.stages = stages;
  if (h_grid) {
    r.grid.kind = KDE_GRID_EXPLICIT;
    r.grid.h = h_grid;
    r.grid.n_h = n_h;
  } else {
    r.grid.kind = KDE_GRID_PAPER;
    r.grid.n_h = n_h <= 0 ? 150 : n_h;
  }
  return r;
}

void fill_plugin_info(const DevState& h, int stages, kde_plugin_info* info) {
  info->sigma = h.sigma;
  info->h_rot = h.h_rot;
  info->stages = stages;
  for (int k = 0; k < 3; ++k) {
    info->g[k] = h.g[k];
    info->psi[k] = h.psi[k];
    info->kappa[k] = h.kappa[k];
    info->precision_used[k] = h.prec_used[k];
  }
  info->h = h.h_plugin;
}

}  // namespace

// ======================================================================== C ABI
extern "C" {

kde_status kde_ctx_create(int device, kde_prec prec, kde_ctx** out) {
  if (!out) return KDE_E_INVAL;
  *out = nullptr;
  if (prec != KDE_PREC_MIXED && prec != KDE_PREC_FP64) return KDE_E_INVAL;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return KDE_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return KDE_E_DEVICE;
  kde_ctx* c = new (std::nothrow) kde_ctx();
  if (!c) return KDE_E_NOMEM;
  c->device = device;
  c->prec = prec;
  if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return KDE_E_DEVICE;
  }
  c->stream = c->own;
  *out = c;
  return KDE_OK;
}

void kde_ctx_destroy(kde_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  (void)hipFree(c->stage.p);
  (void)hipFree(c->x32.p);
  (void)hipFree(c->x64.p);
  (void)hipFree(c->part.p);
  (void)hipFree(c->part_nf.p);
  (void)hipFree(c->stat_part.p);
  (void)hipFree(c->psi_sums.p);
  (void)hipFree(c->lscv_sums.p);
  (void)hipFree(c->hin.p);
  (void)hipFree(c->hdev.p);
  (void)hipFree(c->c64.p);
  (void)hipFree(c->c32.p);
  (void)hipFree(c->g.p);
  (void)hipFree(c->gs.p);
  (void)hipFree(c->cols.p);
  (void)hipFree(c->units.p);
  (void)hipFree(c->rows.p);
  (void)hipFree(c->st.p);
  if (c->h_st) (void)hipHostFree(c->h_st);
  if (c->h_out) (void)hipHostFree(c->h_out);
  for (Pending& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->own) (void)hipStreamDestroy(c->own);
  delete c;
}

const char* kde_last_error(const kde_ctx* c) {
  if (!c) return "NULL context";
  return c->err.c_str();
}

kde_status kde_ctx_set_stream(kde_ctx* c, void* hip_stream) {
  if (!c) return KDE_E_INVAL;
  c->stream = hip_stream ? (hipStream_t)hip_stream : c->own;
  return KDE_OK;
}

kde_status kde_ctx_set_precision(kde_ctx* c, kde_prec prec) {
  if (!c) return KDE_E_INVAL;
  if (prec != KDE_PREC_MIXED && prec != KDE_PREC_FP64) return fail(c, KDE_E_INVAL, "unknown precision");
  c->prec = prec;
  return KDE_OK;
}

kde_status kde_ctx_set_option(kde_ctx* c, const char* key, int64_t value) {
  if (!c || !key) return KDE_E_INVAL;
  const std::string k(key);
  if (k == "lscv_hc") {
    if (value < 0) value = 16;
    if (value != 8 && value != 16 && value != 32) return fail(c, KDE_E_INVAL, "lscv_hc must be 8, 16 or 32");
    c->opt_hc = (int)value;
  } else if (k == "seg") {
    c->opt_seg = value < 0 ? -1 : value;
  } else if (k == "launch_evals") {
    c->opt_launch_evals = value <= 0 ? 4e12 : (double)value;
  } else if (k == "fp64_kappa") {
    c->opt_fp64_kappa = value < 0 ? 1e3 : (double)value;
  } else {
    return fail(c, KDE_E_INVAL, "unknown option " + k);
  }
  return KDE_OK;
}

kde_status kde_ctx_set_timing(kde_ctx* c, int enable) {
  if (!c) return KDE_E_INVAL;
  c->timing = enable != 0;
  for (int f = 0; f < 2; ++f) {
    c->t_launches[f] = 0;
    c->t_ms[f] = 0.0;
    c->t_evals[f] = 0.0;
  }
  return KDE_OK;
}

kde_status kde_ctx_kernel_time(kde_ctx* c, const char* family, int64_t* launches, double* total_ms, double* evals) {
  if (!c || !family) return KDE_E_INVAL;
  int f;
  if (!std::strcmp(family, "lscv_pairs"))
    f = kFamLscv;
  else if (!std::strcmp(family, "psi_pairs"))
    f = kFamPsi;
  else
    return fail(c, KDE_E_INVAL, "unknown kernel family");
  if (launches) *launches = c->t_launches[f];
  if (total_ms) *total_ms = c->t_ms[f];
  if (evals) *evals = c->t_evals[f];
  return KDE_OK;
}

kde_status kde_bw_rot(kde_ctx* c, kde_column x, double* h_out) {
  if (!c || !h_out) return KDE_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  if ((s = run_single(c, make_req(x, KDE_METHOD_ROT, 2, nullptr, 0)))) return s;
  if ((s = sync_and_check(c))) return s;
  if ((s = map_status(c, c->h_st[0].status))) return s;
  *h_out = c->h_st[0].h_rot;
  return KDE_OK;
}

kde_status kde_bw_plugin(kde_ctx* c, kde_column x, int stages, double* h_out, kde_plugin_info* info) {
  if (!c || !h_out) return KDE_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  if ((s = run_single(c, make_req(x, KDE_METHOD_PLUGIN, stages, nullptr, 0)))) return s;
  if ((s = sync_and_check(c))) return s;
  const DevState& h = c->h_st[0];
  if (info) fill_plugin_info(h, stages, info);
  if ((s = map_status(c, h.status))) return s;
  if ((s = map_status(c, h.pstatus))) return s;
  *h_out = h.h_plugin;
  return KDE_OK;
}

kde_status kde_lscv_curve(kde_ctx* c, kde_column x, const double* h_grid, int32_t n_h, double* g_out,
                          double* gscale_out, double* grid_out) {
  if (!c || !g_out) return KDE_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  if (!h_grid && n_h <= 0) n_h = 150;
  if ((s = run_single(c, make_req(x, KDE_METHOD_LSCV, 2, h_grid, n_h)))) return s;
  if ((s = ensure_pinned(c, c->h_out, c->h_out_cap, (size_t)3 * n_h))) return s;
  const int64_t o = c->jcols[0].d.c_off;
  HIP_TRY(c, hipMemcpyAsync(c->h_out, c->g.p + o, sizeof(double) * n_h, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->h_out + n_h, c->gs.p + o, sizeof(double) * n_h, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->h_out + 2 * (size_t)n_h, c->hdev.p + o, sizeof(double) * n_h, hipMemcpyDeviceToHost,
                            c->stream));
  if ((s = sync_and_check(c))) return s;
  if ((s = map_status(c, c->h_st[0].status))) return s;
  std::memcpy(g_out, c->h_out, sizeof(double) * n_h);
  if (gscale_out) std::memcpy(gscale_out, c->h_out + n_h, sizeof(double) * n_h);
  if (grid_out) std::memcpy(grid_out, c->h_out + 2 * (size_t)n_h, sizeof(double) * n_h);
  return KDE_OK;
}

kde_status kde_lscv_sums(kde_ctx* c, kde_column x, const double* h_grid, int32_t n_h, double* s1_out,
                         double* s2_out) {
  if (!c || !h_grid || !s1_out || !s2_out) return KDE_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  if ((s = run_single(c, make_req(x, KDE_METHOD_LSCV, 2, h_grid, n_h)))) return s;
  if ((s = ensure_pinned(c, c->h_out, c->h_out_cap, (size_t)2 * n_h))) return s;
  HIP_TRY(c, hipMemcpyAsync(c->h_out, c->lscv_sums.p + 2 * c->jcols[0].d.c_off, sizeof(double) * 2 * n_h,
                            hipMemcpyDeviceToHost, c->stream));
  if ((s = sync_and_check(c))) return s;
  if ((s = map_status(c, c->h_st[0].status))) return s;
  for (int32_t k = 0; k < n_h; ++k) {
    s1_out[k] = c->h_out[2 * k];
    s2_out[k] = c->h_out[2 * k + 1];
  }
  return KDE_OK;
}

kde_status kde_lscv_item_sums(kde_ctx* c, kde_column x, const double* h_grid, int32_t n_h, const int32_t* sel,
                              int32_t n_sel, int32_t* n_items_out, int32_t* ranges_out, double* sums_out) {
  if (!c || !h_grid || !n_items_out || n_sel < 0) return KDE_E_INVAL;
  if (n_sel > 0 && (!sel || !ranges_out || !sums_out)) return fail(c, KDE_E_INVAL, "NULL selection buffers");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  if ((s = run_single(c, make_req(x, KDE_METHOD_LSCV, 2, h_grid, n_h)))) return s;
  const JobCol& jc = c->jcols[0];
  const int32_t n_items = jc.d.n_items;
  std::vector<int32_t> idx((size_t)n_sel);
  for (int32_t k = 0; k < n_sel; ++k) {
    idx[k] = sel[k] < 0 ? n_items + sel[k] : sel[k];
    if (idx[k] < 0 || idx[k] >= n_items) {
      (void)hipStreamSynchronize(c->stream);
      return fail(c, KDE_E_INVAL, "item index out of range");
    }
  }
  if ((s = ensure_pinned(c, c->h_out, c->h_out_cap, (size_t)2 * n_h * (n_sel > 0 ? n_sel : 1)))) return s;
  // the column's partials are laid out [2*n_h][n_items]: one strided column per selected item
  for (int32_t k = 0; k < n_sel; ++k)
    HIP_TRY(c, hipMemcpy2DAsync(c->h_out + (size_t)k * 2 * n_h, sizeof(double), c->part.p + jc.d.part_off + idx[k],
                                sizeof(double) * (size_t)n_items, sizeof(double), (size_t)2 * n_h,
                                hipMemcpyDeviceToHost, c->stream));
  if ((s = sync_and_check(c))) return s;
  if ((s = map_status(c, c->h_st[0].status))) return s;
  *n_items_out = n_items;
  for (int32_t k = 0; k < n_sel; ++k) {
    ranges_out[3 * k] = jc.lscv_items.row[idx[k]] * kde::kBI;
    ranges_out[3 * k + 1] = jc.lscv_items.jb[idx[k]];
    ranges_out[3 * k + 2] = jc.lscv_items.je[idx[k]];
    std::memcpy(sums_out + (size_t)k * 2 * n_h, c->h_out + (size_t)k * 2 * n_h, sizeof(double) * 2 * n_h);
  }
  return KDE_OK;
}

kde_status kde_bw_lscv(kde_ctx* c, kde_column x, const double* h_grid, int32_t n_h, double* h_out, int32_t* k_out,
                       int* at_edge) {
  if (!c || !h_out) return KDE_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  if (!h_grid && n_h <= 0) n_h = 150;
  if ((s = run_single(c, make_req(x, KDE_METHOD_LSCV, 2, h_grid, n_h)))) return s;
  if ((s = sync_and_check(c))) return s;
  if ((s = map_status(c, c->h_st[0].status))) return s;
  *h_out = c->h_st[0].h_best;
  if (k_out) *k_out = c->h_st[0].k_best;
  if (at_edge) *at_edge = c->h_st[0].at_edge;
  return KDE_OK;
}

kde_status kde_batch(kde_ctx* c, const kde_request* reqs, int32_t n_req, kde_result* out) {
  if (!c || n_req < 0 || (n_req > 0 && (!reqs || !out))) return KDE_E_INVAL;
  if (n_req > KDE_MAX_BATCH) return fail(c, KDE_E_INVAL, "more than KDE_MAX_BATCH requests");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  std::vector<kde_status> st;
  std::vector<std::string> msg;
  plan_job(c, reqs, n_req, st, msg);
  kde_status s;
  if ((s = run_job(c))) return s;
  // g / gscale of LSCV requests into pinned staging, then to the caller
  size_t total = 0;
  for (const JobCol& jc : c->jcols)
    if (jc.lscv) total += 2 * (size_t)jc.d.n_h;
  if ((s = ensure_pinned(c, c->h_out, c->h_out_cap, std::max<size_t>(total, 1)))) return s;
  size_t o = 0;
  std::vector<size_t> at(c->jcols.size(), 0);
  for (size_t k = 0; k < c->jcols.size(); ++k) {
    const JobCol& jc = c->jcols[k];
    if (!jc.lscv) continue;
    at[k] = o;
    HIP_TRY(c, hipMemcpyAsync(c->h_out + o, c->g.p + jc.d.c_off, sizeof(double) * jc.d.n_h, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->h_out + o + jc.d.n_h, c->gs.p + jc.d.c_off, sizeof(double) * jc.d.n_h,
                              hipMemcpyDeviceToHost, c->stream));
    o += 2 * (size_t)jc.d.n_h;
  }
  if ((s = sync_and_check(c))) return s;
  const double nan = std::nan("");
  for (int32_t k = 0; k < n_req; ++k) {
    kde_result& r = out[k];
    double* g_keep = r.g_out;
    double* gs_keep = r.gscale_out;
    std::memset(&r, 0, sizeof(r));
    r.g_out = g_keep;
    r.gscale_out = gs_keep;
    r.status = st[k];
    r.sigma = r.h_rot = r.h_plugin = r.h_lscv = nan;
    r.k_lscv = -1;
  }
  for (size_t k = 0; k < c->jcols.size(); ++k) {
    const JobCol& jc = c->jcols[k];
    const DevState& h = c->h_st[k];
    kde_result& r = out[jc.req];
    r.status = status_of(h.status);
    if (r.status == KDE_OK && jc.plugin) r.status = status_of(h.pstatus);
    r.sigma = h.sigma;
    r.h_rot = h.h_rot;
    if (jc.plugin) {
      fill_plugin_info(h, jc.stages, &r.plugin);
      r.h_plugin = h.h_plugin;
    }
    if (jc.lscv) {
      r.h_lscv = h.h_best;
      r.k_lscv = h.k_best;
      r.at_edge = h.at_edge;
      if (r.g_out) std::memcpy(r.g_out, c->h_out + at[k], sizeof(double) * jc.d.n_h);
      if (r.gscale_out) std::memcpy(r.gscale_out, c->h_out + at[k] + jc.d.n_h, sizeof(double) * jc.d.n_h);
    }
  }
  return KDE_OK;
}

}  // extern "C"
