// kde_runtime.hip -- host runtime and C ABI of the bandwidth-selection library.
//
// Every call is a job over a set of columns: one for the single-column
// selectors, many for kde_batch, the resident requests of a server iteration.
// Each column gets a device block (working copies of its samples, partial
// sums, grid, results) described by a ColDesc of absolute pointers, and its
// own work decomposition, which depends only on its n, its grid size and the
// context options.  The executor enqueues one pass: moments, the plug-in
// stages, the LSCV pass, each as launches whose work units mix the columns
// (largest first, split into launches of bounded work), then fixed-order
// FP64 segmented reductions and the finalize kernels.  No step of the method
// runs on the host: the host checks arguments and plans the work units.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kde_bw.h"
#include "kde_internal.h"
#include "kde_runtime.h"

using kde::ColDesc;
using kde::ColItems;
using kde::ColPlan;
using kde::DevState;
using kde::IterPlan;
using kde::RowDesc;
using kde::Unit;
using kde::UnitCost;

namespace kde {

kde_status fail(kde_ctx* c, kde_status st, const std::string& msg) {
  c->err = msg;
  return st;
}

kde_status status_of(int st) {
  switch (st) {
    case kStOk: return KDE_OK;
    case kStInval: return KDE_E_INVAL;
    case kStDegenerate: return KDE_E_DEGENERATE;
    default: return KDE_E_DEVICE;
  }
}

kde_status ensure_pinned_bytes(kde_ctx* c, char*& p, size_t& cap, size_t bytes) {
  if (cap >= bytes) return KDE_OK;
  if (c->no_alloc) return fail(c, KDE_E_NOMEM, "request needs more host staging than the call's fixed buffers hold");
  if (p) (void)hipHostFree(p);
  p = nullptr;
  cap = 0;
  const size_t want = std::max<size_t>(bytes, 4096);
  if (hipHostMalloc((void**)&p, want, hipHostMallocDefault) != hipSuccess) {
    p = nullptr;
    return fail(c, KDE_E_NOMEM, "pinned host allocation failed");
  }
  cap = want;
  return KDE_OK;
}

void IterPlan::clear() {
  uploads.clear();
  cols.clear();
  ids_stats.clear();
  for (int s = 0; s < 3; ++s) {
    ids_begin[s].clear();
    ids_finish[s].clear();
    psi_units[s].clear();
    psi_cost[s].clear();
    psi_rows[s].clear();
    psi_cond_units[s].clear();
    psi_cond_cost[s].clear();
  }
  ids_plugin_final.clear();
  ids_lscv_prep.clear();
  lscv_units.clear();
  lscv_cost.clear();
  lscv_rows.clear();
  ids_lscv_final.clear();
  sorts.clear();
  near_units.clear();
  near_cost.clear();
  near_rows.clear();
  ids_prune.clear();
  prune_units.clear();
  prune_cost.clear();
  max_stat_blocks = 1;
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
// Pairs i < j with i in the row's 256 samples, j in [jb, je), both < n:
// sum over i of max(0, je - max(jb, i + 1)) in closed form (rows i < jb
// contribute je - jb each, rows i >= jb the arithmetic series je - 1 - i).
double item_pairs(int64_t n, int64_t row, int64_t jb, int64_t je) {
  const int64_t i0 = row * kBI;
  const int64_t i1 = std::min<int64_t>(n, i0 + kBI);
  je = std::min<int64_t>(je, n);
  int64_t p = 0;
  const int64_t flat_end = std::min(i1, jb);  // i in [i0, flat_end): j from jb
  if (flat_end > i0 && je > jb) p += (flat_end - i0) * (je - jb);
  const int64_t a = std::max(i0, jb), b = std::min(i1, je - 1);  // i in [a, b): j from i + 1
  if (b > a) p += (b - a) * ((je - 1 - a) + (je - b)) / 2;
  return (double)p;
}

// Items of one column: row r sweeps j in [r*kBI, n) rounded up to kBJ, cut
// into pieces of `seg` samples (0: one piece).  Ordered longest first.
void make_items(int64_t n, int64_t seg, ColItems& out) {
  std::vector<int> row, jb, je;
  std::vector<double> pr;
  const int64_t rows = (n + kBI - 1) / kBI;
  for (int64_t r = 0; r < rows; ++r) {
    const int64_t row0 = r * kBI;
    const int64_t len = ((n - row0) + kBJ - 1) / kBJ * kBJ;
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

// Item length for a pass whose blocks each evaluate `hc` terms per pair.
// The LSCV pass sizes its items for kSegRefHC bandwidths per block whatever
// variant runs, so the items, and with them every sum's order, do not depend
// on the variant.
int64_t pick_seg(const kde_ctx* c, int64_t n, int hc) {
  if (c->opt_seg >= 0) return c->opt_seg == 0 ? 0 : (c->opt_seg + kBJ - 1) / kBJ * kBJ;
  // Aim for ~32768 blocks per launch: about 32 rounds of the ~1024 blocks the
  // chip holds at once, so the partly filled last round of each launch (the
  // launches of a pass run back to back, not overlapped) costs ~1-2%.
  const double per_block_pairs = c->opt_launch_evals / 32768.0 / (double)hc;
  int64_t seg = (int64_t)(per_block_pairs / kBI);
  seg = std::max<int64_t>(kBJ, seg / kBJ * kBJ);
  if (seg >= n) return 0;
  return seg;
}

// Item length of a pass with `chunks` units per item: pick_seg's length,
// doubled while the pass would hold more than kMaxUnits units, which bounds
// the planner's host memory (24 bytes a unit) for very large columns; at the
// sizes of the workloads (n <= 2e6) the cap is far away.
int64_t capped_seg(const kde_ctx* c, int64_t n, int hc, double chunks) {
  int64_t seg = pick_seg(c, n, hc);
  if (c->opt_seg >= 0 || seg == 0) return seg;
  const double rows = (double)((n + kBI - 1) / kBI);
  const double row_samples = 0.5 * (double)n * (double)n / kBI;  // sum of the rows' j-spans
  while (seg < n && (row_samples / (double)seg + rows) * chunks > kMaxUnits) seg *= 2;
  return seg >= n ? 0 : seg;
}

namespace {

size_t take(size_t& at, size_t bytes) {
  const size_t o = at;
  at += (bytes + 255) / 256 * 256;
  return o;
}

}  // namespace

std::string check_request(const kde_request& r) {
  std::string e = check_column(r.x);
  if (e.empty() && (r.methods & KDE_METHOD_PLUGIN) && r.stages != 2 && r.stages != 3) e = "stages must be 2 or 3";
  if (e.empty() && (r.methods & KDE_METHOD_LSCV)) e = check_grid(r.grid);
  return e;
}

std::string plan_column(const kde_ctx* c, const kde_request& r, ColPlan& p) {
  std::string e = check_request(r);
  p = ColPlan();
  p.plugin = (r.methods & KDE_METHOD_PLUGIN) != 0;
  p.lscv = (r.methods & KDE_METHOD_LSCV) != 0;
  if (!e.empty()) return e;
  const bool all64 = c->prec == KDE_PREC_FP64;
  p.n = (int)r.x.n;
  p.f64 = r.x.dtype == KDE_F64;
  p.stages = p.plugin ? r.stages : 0;
  p.hc = all64 ? 8 : c->job_hc;
  // psi items are cut like one LSCV chunk's (about 7.6e6 pairs a block at
  // the default launch size): a stage's pass then spans ~30 rounds of the
  // blocks the chip holds, so its partly filled last round costs little
  if (p.plugin) make_items(p.n, capped_seg(c, p.n, kSegRefHC, 1.0), p.psi_items);
  if (p.lscv) {
    p.n_h = r.grid.n_h;
    p.n_chunks = (p.n_h + p.hc - 1) / p.hc;
    p.grid_kind = (int)r.grid.kind;
    p.grid_lo = r.grid.lo;
    p.grid_hi = r.grid.hi;
    if (r.grid.kind == KDE_GRID_EXPLICIT) p.grid_h.assign(r.grid.h, r.grid.h + p.n_h);
    make_items(p.n, capped_seg(c, p.n, kSegRefHC, (double)((p.n_h + kSegRefHC - 1) / kSegRefHC)), p.lscv_items);
    p.prune = c->opt_prune && !all64;
    if (p.prune) {
      // the first j-tile of every row: j in [row0, row0 + kBJ)
      const int rows = (p.n + kBI - 1) / kBI;
      for (int r = 0; r < rows; ++r) {
        p.near_items.row.push_back(r);
        p.near_items.jb.push_back(r * kBI);
        p.near_items.je.push_back(r * kBI + kBJ);
        p.near_items.pairs.push_back(item_pairs(p.n, r, (int64_t)r * kBI, (int64_t)r * kBI + kBJ));
      }
    }
  }
  p.want_x64 = all64 || (p.plugin && c->opt_fp64_kappa > 0.0);
  p.raw_in_block = !r.x.on_device;
  p.raw_bytes = (size_t)p.n * (p.f64 ? 8 : 4);
  size_t at = 0;
  const size_t xn = (size_t)p.n + kPad;
  if (p.raw_in_block) p.off_raw = take(at, p.raw_bytes);
  p.off_x32 = take(at, 4 * xn);
  if (p.want_x64) p.off_x64 = take(at, 8 * xn);
  p.off_stat = take(at, 8 * kStatBlocks);
  p.off_mm = take(at, 8 * kStatBlocks);
  p.off_nf = take(at, 4 * kStatBlocks);
  if (p.plugin) {
    if (!all64) p.off_y32 = take(at, 4 * xn);
    p.off_psi_part = take(at, 16 * p.psi_items.pairs.size());
    p.off_psi_sums = take(at, 16);
  }
  if (p.lscv) {
    const size_t m = (size_t)p.n_chunks * p.hc;
    p.off_hin = take(at, 8 * (size_t)p.n_h);
    p.off_h = take(at, 8 * m);
    p.off_c32 = take(at, 4 * m);
    p.off_c64 = take(at, 8 * m);
    p.off_part = take(at, 16 * (size_t)p.n_h * p.lscv_items.pairs.size());
    p.off_sums = take(at, 16 * (size_t)p.n_h);
    p.off_g = take(at, 8 * (size_t)p.n_h);
    p.off_gs = take(at, 8 * (size_t)p.n_h);
    if (p.prune) {
      p.off_xs = take(at, 4 * xn);
      p.off_near_part = take(at, 16 * (size_t)p.n_h * p.near_items.pairs.size());
      p.off_near_sums = take(at, 16 * (size_t)p.n_h);
      p.off_d2cut = take(at, 4 * (size_t)p.n_chunks);
    }
  }
  p.bytes = at;
  return "";
}

void bind_column(const ColPlan& p, char* b, const void* raw, DevState* st, ColDesc& d) {
  std::memset(&d, 0, sizeof(d));
  d.raw = p.raw_in_block ? (const void*)(b + p.off_raw) : raw;
  d.x32 = (float*)(b + p.off_x32);
  d.x64 = p.want_x64 ? (double*)(b + p.off_x64) : nullptr;
  d.stat = (double*)(b + p.off_stat);
  d.stat_mm = (float*)(b + p.off_mm);
  d.stat_nf = (int*)(b + p.off_nf);
  if (p.plugin) {
    d.y32 = p.off_y32 ? (float*)(b + p.off_y32) : nullptr;
    d.psi_part = (double*)(b + p.off_psi_part);
    d.psi_sums = (double*)(b + p.off_psi_sums);
  }
  if (p.lscv) {
    d.h_in = (const double*)(b + p.off_hin);
    d.h = (double*)(b + p.off_h);
    d.c32 = (float*)(b + p.off_c32);
    d.c64 = (double*)(b + p.off_c64);
    d.part = (double*)(b + p.off_part);
    d.sums = (double*)(b + p.off_sums);
    d.g = (double*)(b + p.off_g);
    d.gs = (double*)(b + p.off_gs);
    if (p.prune) {
      d.near_sums = (double*)(b + p.off_near_sums);
      d.d2cut = (float*)(b + p.off_d2cut);
    }
  }
  d.st = st;
  d.n = p.n;
  d.raw_f64 = p.f64;
  d.n_h = p.lscv ? p.n_h : 0;
  d.n_chunks = p.n_chunks;
  d.n_items = (int)p.lscv_items.pairs.size();
  d.n_items_psi = (int)p.psi_items.pairs.size();
  d.grid_kind = p.grid_kind;
  d.grid_lo = p.grid_lo;
  d.grid_hi = p.grid_hi;
}

void init_state(const ColPlan& p, double fp64_kappa, DevState& h) {
  std::memset(&h, 0, sizeof(h));
  const double nan = std::nan("");
  h.stages = p.stages;
  for (int q = 0; q < 3; ++q) {
    h.g[q] = h.psi[q] = h.kappa[q] = nan;
    h.prec_used[q] = -1;
  }
  h.h_plugin = h.h_best = h.margin = nan;
  h.k_best = -1;
  h.fp64_kappa = fp64_kappa;
}

void psi_units_of(const ColPlan& p, int id, std::vector<Unit>& u, std::vector<UnitCost>& cost) {
  for (size_t it = 0; it < p.psi_items.pairs.size(); ++it) {
    u.push_back(Unit{id, p.psi_items.row[it], p.psi_items.jb[it], p.psi_items.je[it], (int)it, 0});
    cost.push_back(UnitCost{p.psi_items.pairs[it], p.psi_items.pairs[it]});
  }
}

void lscv_units_of(const ColPlan& p, int id, std::vector<Unit>& u, std::vector<UnitCost>& cost) {
  for (size_t it = 0; it < p.lscv_items.pairs.size(); ++it)
    for (int ch = 0; ch < p.n_chunks; ++ch) {
      u.push_back(Unit{id, p.lscv_items.row[it], p.lscv_items.jb[it], p.lscv_items.je[it], (int)it, ch});
      const int valid = std::min(p.hc, p.n_h - ch * p.hc);
      cost.push_back(UnitCost{p.lscv_items.pairs[it], p.lscv_items.pairs[it] * valid});
    }
}

void psi_rows_of(const ColPlan& p, const ColDesc& d, std::vector<RowDesc>& rows) {
  const int m = (int)p.psi_items.pairs.size();
  for (int w = 0; w < 2; ++w) rows.push_back(RowDesc{d.psi_part + (size_t)w * m, d.psi_sums + w, m, 0});
}

void lscv_rows_of(const ColPlan& p, const ColDesc& d, std::vector<RowDesc>& rows) {
  const int m = (int)p.lscv_items.pairs.size();
  for (int r = 0; r < 2 * p.n_h; ++r) rows.push_back(RowDesc{d.part + (size_t)r * m, d.sums + r, m, 0});
}

void prune_descs(const ColPlan& p, const ColDesc& d, ColDesc& nd, ColDesc& sd) {
  nd = d;
  sd = d;
  float* xs = (float*)((char*)d.x32 - p.off_x32 + p.off_xs);
  nd.x32 = sd.x32 = xs;
  nd.part = (double*)((char*)d.x32 - p.off_x32 + p.off_near_part);
  nd.n_items = (int)p.near_items.pairs.size();
}

void add_prune_setup(const ColPlan& p, const ColDesc& d, int id, int extra_id, IterPlan& it) {
  ColDesc nd, sd;
  prune_descs(p, d, nd, sd);
  if ((int)it.cols.size() < extra_id + 2) it.cols.resize(extra_id + 2);
  it.cols[extra_id] = nd;
  it.cols[extra_id + 1] = sd;
  it.sorts.push_back(SortJob{d.x32, sd.x32, p.n + kPad});
  const int m = (int)p.near_items.pairs.size();
  for (int r = 0; r < m; ++r)
    for (int ch = 0; ch < p.n_chunks; ++ch) {
      it.near_units.push_back(Unit{extra_id, p.near_items.row[r], p.near_items.jb[r], p.near_items.je[r], r, ch});
      const int valid = std::min(p.hc, p.n_h - ch * p.hc);
      it.near_cost.push_back(UnitCost{p.near_items.pairs[r], p.near_items.pairs[r] * valid});
    }
  for (int r = 0; r < 2 * p.n_h; ++r)
    it.near_rows.push_back(RowDesc{nd.part + (size_t)r * m, d.near_sums + r, m, 0});
  it.ids_prune.push_back(id);
}

void add_full_column(const kde_ctx* c, const ColPlan& p, const ColDesc& d, int id, const void* host_raw,
                     IterPlan& it, int extra_id) {
  if ((int)it.cols.size() <= id) it.cols.resize(id + 1);
  it.cols[id] = d;
  if (p.raw_in_block) it.uploads.push_back(Upload{(void*)d.raw, host_raw, p.raw_bytes});
  it.ids_stats.push_back(id);
  it.max_stat_blocks = std::max(it.max_stat_blocks, std::min(kStatBlocks, (p.n + 2047) / 2048));
  const bool cond = c->prec != KDE_PREC_FP64 && c->opt_fp64_kappa > 0.0;
  if (p.plugin) {
    for (int s = (p.stages == 3 ? 0 : 1); s < 3; ++s) {
      it.ids_begin[s].push_back(id);
      psi_units_of(p, id, it.psi_units[s], it.psi_cost[s]);
      psi_rows_of(p, d, it.psi_rows[s]);
      it.ids_finish[s].push_back(id);
      if (cond) psi_units_of(p, id, it.psi_cond_units[s], it.psi_cond_cost[s]);
    }
    it.ids_plugin_final.push_back(id);
  }
  if (p.lscv) {
    if (p.grid_kind == KDE_GRID_EXPLICIT)
      it.uploads.push_back(Upload{(void*)d.h_in, p.grid_h.data(), sizeof(double) * p.n_h});
    it.ids_lscv_prep.push_back(id);
    if (p.prune && extra_id >= 0) {
      add_prune_setup(p, d, id, extra_id, it);
      lscv_units_of(p, extra_id + 1, it.prune_units, it.prune_cost);
    } else {
      lscv_units_of(p, id, it.lscv_units, it.lscv_cost);
    }
    lscv_rows_of(p, d, it.lscv_rows);
    it.ids_lscv_final.push_back(id);
  }
}

// ---- timing
kde_status timed_begin(kde_ctx* c, kde_ctx::Pending& p) {
  if (!c->timing) return KDE_OK;
  for (hipEvent_t* e : {&p.a, &p.b}) {
    if (!c->ev_pool.empty()) {
      *e = c->ev_pool.back();
      c->ev_pool.pop_back();
    } else {
      KDE_HIP_TRY(c, hipEventCreate(e));
    }
  }
  KDE_HIP_TRY(c, hipEventRecord(p.a, c->stream));
  return KDE_OK;
}

kde_status timed_end(kde_ctx* c, kde_ctx::Pending& p) {
  if (!c->timing) return KDE_OK;
  KDE_HIP_TRY(c, hipEventRecord(p.b, c->stream));
  c->pending.push_back(p);
  return KDE_OK;
}

namespace {

kde_status collect_timing(kde_ctx* c) {
  for (kde_ctx::Pending& p : c->pending) {
    float ms = 0.f;
    KDE_HIP_TRY(c, hipEventElapsedTime(&ms, p.a, p.b));
    c->t_launches[p.family] += 1;
    c->t_ms[p.family] += ms;
    c->t_evals[p.family] += p.evals;
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->pending.clear();
  return KDE_OK;
}

// Sorts units largest first (the order blocks are dispatched in); results do
// not depend on it, since every unit writes its own partial-sum slot.
// scatter: units of equal planned size are put in a fixed pseudo-random
// order instead of (item, chunk) order.  With tile pruning their real cost
// depends strongly on the chunk (small bandwidths skip most tiles), and
// consecutive blocks are dealt round-robin to the chip's eight dies, so in
// (item, chunk) order each die would always get the same chunks.
void sort_units(std::vector<Unit>& u, std::vector<UnitCost>& cost, bool scatter = false) {
  std::vector<size_t> o(u.size());
  for (size_t k = 0; k < o.size(); ++k) o[k] = k;
  std::vector<uint32_t> key(scatter ? u.size() : 0);
  for (size_t k = 0; k < key.size(); ++k) {
    uint32_t h = (uint32_t)u[k].item * 0x9E3779B1u ^ (uint32_t)u[k].chunk * 0x85EBCA77u ^ (uint32_t)u[k].col;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    key[k] = h;
  }
  std::stable_sort(o.begin(), o.end(), [&](size_t a, size_t b) {
    if (cost[a].pairs != cost[b].pairs) return cost[a].pairs > cost[b].pairs;
    return scatter && key[a] < key[b];
  });
  std::vector<Unit> u2(u.size());
  std::vector<UnitCost> c2(u.size());
  for (size_t k = 0; k < o.size(); ++k) {
    u2[k] = u[o[k]];
    c2[k] = cost[o[k]];
  }
  u.swap(u2);
  cost.swap(c2);
}

// Groups of the persistent dense sweep: the largest-first list is split,
// keeping that order inside each group, into kQueueGroups stretches of about
// equal work in (column, j) position, so that the blocks starting on one die
// read the sample tiles of one stretch of the column.  Positions are bucketed
// (4096 buckets over the columns laid end to end) and the buckets cut where
// the running work passes each equal share: O(units), no second sort.
void group_units(std::vector<Unit>& u, std::vector<UnitCost>& cost, const std::vector<ColDesc>& cols,
                 int (&begin)[kQueueGroups + 1]) {
  constexpr int kBuckets = 4096;
  std::vector<double> col_off(cols.size() + 1, 0.0);
  for (size_t c = 0; c < cols.size(); ++c) col_off[c + 1] = col_off[c] + (double)std::max(cols[c].n, 1);
  const double total_pos = std::max(col_off.back(), 1.0);
  auto bucket = [&](const Unit& x) {
    const double pos = col_off[x.col] + (double)x.j_begin;
    return std::min(kBuckets - 1, (int)(pos / total_pos * kBuckets));
  };
  std::vector<double> work(kBuckets, 0.0);
  double total = 0.0;
  for (size_t k = 0; k < u.size(); ++k) {
    work[bucket(u[k])] += cost[k].evals;
    total += cost[k].evals;
  }
  std::vector<int> group_of(kBuckets, kQueueGroups - 1);
  double run = 0.0;
  int g = 0;
  for (int b = 0; b < kBuckets; ++b) {
    group_of[b] = g;
    run += work[b];
    while (g < kQueueGroups - 1 && run >= total * (double)(g + 1) / kQueueGroups) ++g;
  }
  std::vector<int> count(kQueueGroups, 0);
  for (const Unit& x : u) ++count[group_of[bucket(x)]];
  begin[0] = 0;
  for (int q = 0; q < kQueueGroups; ++q) begin[q + 1] = begin[q] + count[q];
  std::vector<int> at(begin, begin + kQueueGroups);
  std::vector<Unit> u2(u.size());
  std::vector<UnitCost> c2(u.size());
  for (size_t k = 0; k < u.size(); ++k) {
    const int q = group_of[bucket(u[k])];
    u2[at[q]] = u[k];
    c2[at[q]] = cost[k];
    ++at[q];
  }
  u.swap(u2);
  cost.swap(c2);
}

// Launch ranges over units [0, n) whose summed evaluations stay within
// budget, with at least 2048 blocks per launch when the list has them, so a
// launch fills the chip.  FP64 terms cost about five times the FP32 ones.
template <typename F>
kde_status for_each_launch(const kde_ctx* c, const std::vector<UnitCost>& cost, bool f64, F&& launch) {
  const double budget = f64 ? c->opt_launch_evals / 5.0 : c->opt_launch_evals;
  size_t u0 = 0;
  const size_t end = cost.size();
  while (u0 < end) {
    double acc = cost[u0].evals;
    size_t u1 = u0 + 1;
    while (u1 < end && (acc + cost[u1].evals <= budget || u1 - u0 < 2048)) {
      acc += cost[u1].evals;
      ++u1;
    }
    kde_status s = launch((int)u0, (int)(u1 - u0), acc);
    if (s) return s;
    u0 = u1;
  }
  return KDE_OK;
}

// Packs the host arrays of a pass into one pinned blob and copies it to the
// device in one transfer; returns device addresses of each array.
struct Blob {
  std::vector<std::pair<const void*, size_t>> parts;
  std::vector<size_t> offs;
  size_t bytes = 0;
  size_t add(const void* p, size_t n) {
    const size_t o = bytes;
    parts.push_back({p, n});
    offs.push_back(o);
    bytes += (n + 255) / 256 * 256;
    return o;
  }
};

}  // namespace

// Blocks of the persistent LSCV kernel that the device holds at once, asked
// once per variant (0: unavailable, use sliced launches).
int queue_blocks(kde_ctx* c, int hc, int tj) {
  for (int v = 0; v < kQueueVariants; ++v)
    if (kQueueHC[v] == hc && kQueueTJ[v] == tj) {
      if (c->queue_blocks[v] < 0) c->queue_blocks[v] = kde::lscv_queue_blocks(hc, tj);
      return c->queue_blocks[v];
    }
  return 0;
}

// The dense LSCV pass of `it` runs as one persistent launch (mixed form, the
// vector-ALU sweep, option persistent, a variant the device can hold).
bool lscv_queue_form(kde_ctx* c, const IterPlan& it) {
  return c->prec != KDE_PREC_FP64 && !c->job_mfma && c->opt_persistent && !it.lscv_units.empty() &&
         queue_blocks(c, c->job_hc, c->job_tj) > 0;
}

kde_status collect_ready_timing(kde_ctx* c) {
  std::vector<kde_ctx::Pending> later;
  for (kde_ctx::Pending& p : c->pending) {
    if (hipEventQuery(p.b) != hipSuccess) {
      later.push_back(p);
      continue;
    }
    float ms = 0.f;
    KDE_HIP_TRY(c, hipEventElapsedTime(&ms, p.a, p.b));
    c->t_launches[p.family] += 1;
    c->t_ms[p.family] += ms;
    c->t_evals[p.family] += p.evals;
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->pending.swap(later);
  return KDE_OK;
}

kde_status sync_and_check(kde_ctx* c) {
  KDE_HIP_TRY(c, hipGetLastError());
  KDE_HIP_TRY(c, hipStreamSynchronize(c->stream));
  return collect_timing(c);
}

kde_status pack_pass(kde_ctx* c, IterPlan& it, PassLayout& L) {
  kde_status s;
  for (int q = 0; q < 3; ++q) {
    sort_units(it.psi_units[q], it.psi_cost[q]);
    sort_units(it.psi_cond_units[q], it.psi_cond_cost[q]);
  }
  sort_units(it.lscv_units, it.lscv_cost);
  if (lscv_queue_form(c, it)) {
    group_units(it.lscv_units, it.lscv_cost, it.cols, it.lscv_groups);
  } else {
    for (int q = 0; q <= kQueueGroups; ++q) it.lscv_groups[q] = q == 0 ? 0 : (int)it.lscv_units.size();
  }
  sort_units(it.near_units, it.near_cost);
  sort_units(it.prune_units, it.prune_cost, true);
  // one blob: column table, id lists, units, rows
  Blob b;
  auto vbytes = [](const auto& v) { return v.size() * sizeof(v[0]); };
  L.o_cols = b.add(it.cols.data(), vbytes(it.cols));
  L.o_stats = b.add(it.ids_stats.data(), vbytes(it.ids_stats));
  for (int q = 0; q < 3; ++q) {
    L.o_begin[q] = b.add(it.ids_begin[q].data(), vbytes(it.ids_begin[q]));
    L.o_finish[q] = b.add(it.ids_finish[q].data(), vbytes(it.ids_finish[q]));
    L.o_psu[q] = b.add(it.psi_units[q].data(), vbytes(it.psi_units[q]));
    L.o_pr[q] = b.add(it.psi_rows[q].data(), vbytes(it.psi_rows[q]));
    L.o_pc[q] = b.add(it.psi_cond_units[q].data(), vbytes(it.psi_cond_units[q]));
  }
  L.o_pf = b.add(it.ids_plugin_final.data(), vbytes(it.ids_plugin_final));
  L.o_lp = b.add(it.ids_lscv_prep.data(), vbytes(it.ids_lscv_prep));
  L.o_lu = b.add(it.lscv_units.data(), vbytes(it.lscv_units));
  L.o_lr = b.add(it.lscv_rows.data(), vbytes(it.lscv_rows));
  L.o_lf = b.add(it.ids_lscv_final.data(), vbytes(it.ids_lscv_final));
  L.o_nu = b.add(it.near_units.data(), vbytes(it.near_units));
  L.o_nr = b.add(it.near_rows.data(), vbytes(it.near_rows));
  L.o_pp = b.add(it.ids_prune.data(), vbytes(it.ids_prune));
  L.o_pu = b.add(it.prune_units.data(), vbytes(it.prune_units));
  static const int kZeroCounters[64] = {};
  L.o_ctr = b.add(kZeroCounters, sizeof(kZeroCounters));
  L.o_lg = b.add(it.lscv_groups, sizeof(it.lscv_groups));
  L.bytes = b.bytes;
  L.sort_tmp = 0;
  for (const SortJob& j : it.sorts) {
    const size_t t = kde::sort_temp_bytes(j.count);
    if (t == 0) return fail(c, KDE_E_DEVICE, "sort temporary size query failed");
    L.sort_tmp = std::max(L.sort_tmp, t);
  }
  // a device buffer that must grow may still be read by work in flight on the
  // stream (the server enqueues an iteration before the previous one ends):
  // wait for the stream before replacing it
  if ((L.sort_tmp > c->sort_tmp.cap && c->sort_tmp.p) || (b.bytes + 256 > c->blob.cap && c->blob.p))
    KDE_HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (L.sort_tmp && (s = ensure(c, c->sort_tmp, L.sort_tmp))) return s;
  if ((s = ensure_pinned_bytes(c, c->h_blob, c->h_blob_cap, b.bytes + 256))) return s;
  if ((s = ensure(c, c->blob, b.bytes + 256))) return s;
  for (size_t k = 0; k < b.parts.size(); ++k)
    if (b.parts[k].second) std::memcpy(c->h_blob + b.offs[k], b.parts[k].first, b.parts[k].second);
  return KDE_OK;
}

kde_status upload_pass(kde_ctx* c, const IterPlan& it, const PassLayout& L) {
  for (const kde::Upload& u : it.uploads)
    if (u.bytes) KDE_HIP_TRY(c, hipMemcpyAsync(u.dst, u.src, u.bytes, hipMemcpyHostToDevice, c->stream));
  KDE_HIP_TRY(c, hipMemcpyAsync(c->blob.p, c->h_blob, L.bytes, hipMemcpyHostToDevice, c->stream));
  return KDE_OK;
}

kde_status launch_pass(kde_ctx* c, const IterPlan& it, const PassLayout& L) {
  kde_status s;
  const bool all64 = c->prec == KDE_PREC_FP64;
  char* d = c->blob.p;
  const ColDesc* cols = (const ColDesc*)(d + L.o_cols);
  auto ids = [&](size_t o) { return (const int*)(d + o); };
  hipStream_t st = c->stream;
  // moments
  kde::launch_stats(st, cols, ids(L.o_stats), (int)it.ids_stats.size(), it.max_stat_blocks);
  // plug-in stages
  for (int q = 0; q < 3; ++q) {
    if (it.ids_begin[q].empty() && it.psi_units[q].empty() && it.ids_finish[q].empty()) continue;
    const int r = 8 - 2 * q;
    kde::launch_psi_begin(st, cols, ids(L.o_begin[q]), (int)it.ids_begin[q].size(), q, all64 ? 1 : 0);
    const Unit* pu = (const Unit*)(d + L.o_psu[q]);
    s = for_each_launch(c, it.psi_cost[q], all64, [&](int u0, int cnt, double evals) -> kde_status {
      kde_ctx::Pending pd{nullptr, nullptr, kde::kFamPsi, evals};
      kde_status s2 = timed_begin(c, pd);
      if (s2) return s2;
      kde::launch_psi_units(st, r, all64 ? 1 : 0, 0, cols, pu, u0, cnt);
      return timed_end(c, pd);
    });
    if (s) return s;
    kde::launch_reduce_rows(st, (const RowDesc*)(d + L.o_pr[q]), (int)it.psi_rows[q].size());
    kde::launch_psi_finish(st, cols, ids(L.o_finish[q]), (int)it.ids_finish[q].size(), q, all64 ? 1 : 0, 0);
    if (!all64 && !it.psi_cond_units[q].empty()) {
      // FP64 re-run of the columns whose stage is badly conditioned; blocks of
      // other columns exit at once, so these launches are not timed.
      const Unit* pc = (const Unit*)(d + L.o_pc[q]);
      s = for_each_launch(c, it.psi_cond_cost[q], true, [&](int u0, int cnt, double) -> kde_status {
        kde::launch_psi_units(st, r, 1, 1, cols, pc, u0, cnt);
        return KDE_OK;
      });
      if (s) return s;
      kde::launch_reduce_rows(st, (const RowDesc*)(d + L.o_pr[q]), (int)it.psi_rows[q].size());
      kde::launch_psi_finish(st, cols, ids(L.o_finish[q]), (int)it.ids_finish[q].size(), q, 1, 1);
    }
  }
  kde::launch_plugin_final(st, cols, ids(L.o_pf), (int)it.ids_plugin_final.size());
  // LSCV
  const int hc = all64 ? 8 : c->job_hc;
  kde::launch_lscv_prep(st, cols, ids(L.o_lp), (int)it.ids_lscv_prep.size(), hc);
  // tile pruning: sort, near-tile lower bounds and cut distances of the
  // columns whose LSCV work starts in this pass, then the pruned units (a
  // served column's pruned units may span several passes)
  for (const SortJob& j : it.sorts)
    KDE_HIP_TRY(c, kde::sort_keys(c->sort_tmp.p, L.sort_tmp, j.in, j.out, j.count, st));
  if (!it.near_units.empty()) {
    const Unit* nu = (const Unit*)(d + L.o_nu);
    s = for_each_launch(c, it.near_cost, false, [&](int u0, int cnt, double) -> kde_status {
      kde::launch_lscv_units(st, hc, 0, 0, 0, cols, nu, u0, cnt);
      return KDE_OK;
    });
    if (s) return s;
    kde::launch_reduce_rows(st, (const RowDesc*)(d + L.o_nr), (int)it.near_rows.size());
    kde::launch_lscv_prune_prep(st, cols, ids(L.o_pp), (int)it.ids_prune.size(), hc, kPruneEps);
  }
  if (!it.prune_units.empty()) {
    const Unit* pru = (const Unit*)(d + L.o_pu);
    s = for_each_launch(c, it.prune_cost, false, [&](int u0, int cnt, double evals) -> kde_status {
      kde_ctx::Pending pd{nullptr, nullptr, kde::kFamLscv, evals};
      kde_status s2 = timed_begin(c, pd);
      if (s2) return s2;
      kde::launch_lscv_units(st, hc, 0, 0, 1, cols, pru, u0, cnt);
      return timed_end(c, pd);
    });
    if (s) return s;
  }
  const Unit* lu = (const Unit*)(d + L.o_lu);
  if (lscv_queue_form(c, it)) {
    // the whole dense pass in one persistent launch over device work queues
    double evals = 0.0;
    for (const UnitCost& u : it.lscv_cost) evals += u.evals;
    int* ctr = (int*)(d + L.o_ctr);
    kde::launch_zero_ints(st, ctr, kde::kQueueGroups);
    kde_ctx::Pending pd{nullptr, nullptr, kde::kFamLscv, evals};
    if ((s = timed_begin(c, pd))) return s;
    kde::launch_lscv_units_queue(st, hc, c->job_tj, cols, lu, (int)it.lscv_units.size(), (const int*)(d + L.o_lg), ctr,
                                 kde::queue_blocks(c, hc, c->job_tj));
    if ((s = timed_end(c, pd))) return s;
  } else {
    s = for_each_launch(c, it.lscv_cost, all64, [&](int u0, int cnt, double evals) -> kde_status {
      kde_ctx::Pending pd{nullptr, nullptr, kde::kFamLscv, evals};
      kde_status s2 = timed_begin(c, pd);
      if (s2) return s2;
      kde::launch_lscv_units(st, hc, all64 ? 1 : 0, c->job_mfma, 0, cols, lu, u0, cnt);
      return timed_end(c, pd);
    });
    if (s) return s;
  }
  kde::launch_reduce_rows(st, (const RowDesc*)(d + L.o_lr), (int)it.lscv_rows.size());
  kde::launch_lscv_finalize(st, cols, ids(L.o_lf), (int)it.ids_lscv_final.size(), all64 ? 1 : 0);
  KDE_HIP_TRY(c, hipGetLastError());
  return KDE_OK;
}

kde_status execute(kde_ctx* c, IterPlan& it) {
  PassLayout L;
  kde_status s;
  if ((s = pack_pass(c, it, L))) return s;
  if ((s = upload_pass(c, it, L))) return s;
  return launch_pass(c, it, L);
}

void JobGraph::reset() {
  if (exec) (void)hipGraphExecDestroy(exec);
  exec = nullptr;
  last_use = 0;
  sig.clear();
  plans.clear();
  plan_req.clear();
  cols.clear();
  blob_host.clear();
}

}  // namespace kde

namespace {

using kde::fail;

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

kde_status busy(kde_ctx* c) {
  return fail(c, KDE_E_BUSY, "a server is running on this context; use kde_submit/kde_poll/kde_wait");
}

bool serving(const kde_ctx* c) { return c->server && kde::server_running(c->server.get()); }

// ---- graph replay of repeated jobs
// Everything a job's kernel launches depend on besides the device buffers:
// the options, and per request its validity, shape, methods and grid kind.
std::string job_signature(const kde_ctx* c, const kde_request* reqs, int32_t n_req,
                          const std::vector<kde_status>& st) {
  std::string sig;
  auto put = [&](const auto& v) { sig.append(reinterpret_cast<const char*>(&v), sizeof(v)); };
  put(n_req);
  put(c->prec);
  put(c->job_hc);
  put(c->job_tj);
  put(c->job_mfma);
  put(c->opt_seg);
  put(c->opt_launch_evals);
  put(c->opt_fp64_kappa);
  put(c->opt_prune);
  put(c->opt_persistent);
  for (int32_t k = 0; k < n_req; ++k) {
    const kde_request& r = reqs[k];
    const int ok = st[k] == KDE_OK;
    put(ok);
    if (!ok) continue;
    put(r.x.n);
    put(r.x.dtype);
    put(r.x.on_device);
    put(r.methods);
    if (r.methods & KDE_METHOD_PLUGIN) put(r.stages);
    if (r.methods & KDE_METHOD_LSCV) {
      put(r.grid.kind);
      put(r.grid.n_h);
      if (r.grid.kind == KDE_GRID_LOG_ROT) {
        put(r.grid.lo);
        put(r.grid.hi);
      }
    }
  }
  return sig;
}

// Replays the cached graph for a job of the same signature: new samples,
// grids and device column addresses go in through the copies around it.
kde_status replay_job(kde_ctx* c, kde::JobGraph& g, const kde_request* reqs) {
  g.last_use = ++c->graph_clock;
  kde_status s;
  c->plans = g.plans;
  c->plan_req = g.plan_req;
  c->iter.clear();
  c->iter.cols = g.cols;
  const int n_cols = (int)c->plans.size();
  char* hs = reinterpret_cast<char*>(c->h_st);
  if ((s = kde::ensure_pinned_bytes(c, hs, c->h_st_cap, sizeof(DevState) * n_cols))) return s;
  c->h_st = reinterpret_cast<DevState*>(hs);
  if ((s = kde::ensure_pinned_bytes(c, c->h_blob, c->h_blob_cap, g.blob_host.size()))) return s;
  std::memcpy(c->h_blob, g.blob_host.data(), g.blob_host.size());
  for (int k = 0; k < n_cols; ++k) {
    kde::ColPlan& p = c->plans[k];
    const kde_request& r = reqs[c->plan_req[k]];
    ColDesc& d = c->iter.cols[k];
    if (p.raw_in_block)
      KDE_HIP_TRY(c, hipMemcpyAsync((void*)d.raw, r.x.data, p.raw_bytes, hipMemcpyHostToDevice, c->stream));
    else
      d.raw = r.x.data;
    if (p.lscv && p.grid_kind == KDE_GRID_EXPLICIT) {
      p.grid_h.assign(r.grid.h, r.grid.h + p.n_h);
      KDE_HIP_TRY(c, hipMemcpyAsync((void*)d.h_in, p.grid_h.data(), sizeof(double) * p.n_h, hipMemcpyHostToDevice,
                                    c->stream));
    }
    kde::init_state(p, c->opt_fp64_kappa, c->h_st[k]);
  }
  std::memcpy(c->h_blob + g.L.o_cols, c->iter.cols.data(), sizeof(ColDesc) * n_cols);
  KDE_HIP_TRY(c, hipMemcpyAsync(c->st.p, c->h_st, sizeof(DevState) * n_cols, hipMemcpyHostToDevice, c->stream));
  KDE_HIP_TRY(c, hipMemcpyAsync(c->blob.p, c->h_blob, g.L.bytes, hipMemcpyHostToDevice, c->stream));
  KDE_HIP_TRY(c, hipGraphLaunch(g.exec, c->stream));
  KDE_HIP_TRY(c, hipMemcpyAsync(c->h_st, c->st.p, sizeof(DevState) * n_cols, hipMemcpyDeviceToHost, c->stream));
  ++c->graph_replays;
  return KDE_OK;
}

// Enqueues a planned pass with its launches captured into a graph, keeps the
// graph for later jobs of the same signature and launches it.
kde_status capture_job(kde_ctx* c, std::string sig) {
  kde_status s;
  if (c->graphs.size() < kde::kMaxGraphs) c->graphs.emplace_back();
  kde::JobGraph* lru = &c->graphs[0];
  for (kde::JobGraph& x : c->graphs)
    if (x.last_use < lru->last_use) lru = &x;
  kde::JobGraph& g = *lru;
  g.reset();
  g.last_use = ++c->graph_clock;
  kde::PassLayout L;
  if ((s = kde::pack_pass(c, c->iter, L))) return s;
  if ((s = kde::upload_pass(c, c->iter, L))) return s;
  KDE_HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  const kde_status ls = kde::launch_pass(c, c->iter, L);
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(c->stream, &graph);
  if (ls || ee != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    if (ls) return ls;
    return fail(c, KDE_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ee));
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return fail(c, KDE_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
  g.exec = exec;
  g.sig = std::move(sig);
  g.blocks = c->blocks.p;
  g.st = c->st.p;
  g.blob = c->blob.p;
  g.sort_tmp = c->sort_tmp.p;
  g.plans = c->plans;
  g.plan_req = c->plan_req;
  g.cols = c->iter.cols;
  g.blob_host.assign(c->h_blob, c->h_blob + L.bytes);
  g.L = L;
  KDE_HIP_TRY(c, hipGraphLaunch(exec, c->stream));
  ++c->graph_captures;
  return KDE_OK;
}

// Plans and enqueues a synchronous job over n_req requests; per-request
// argument errors land in st/msg.  The states' copy back is enqueued last.
// With the graph option (and timing off, on a non-null stream) the job's
// launches come from a graph: replayed when a kept graph has the job's
// signature and the device buffers did not move, captured otherwise.
kde_status run_requests(kde_ctx* c, const kde_request* reqs, int32_t n_req, std::vector<kde_status>& st,
                        std::vector<std::string>& msg) {
  kde_status s;
  st.assign(n_req, KDE_OK);
  msg.assign(n_req, "");
  if ((s = kde::select_variant(c, reqs, n_req))) return s;
  const bool use_graph = c->opt_graph && !c->timing && c->stream != nullptr;
  std::string sig;
  if (use_graph) {
    for (int32_t k = 0; k < n_req; ++k) {
      msg[k] = kde::check_request(reqs[k]);
      if (!msg[k].empty()) st[k] = KDE_E_INVAL;
    }
    sig = job_signature(c, reqs, n_req, st);
    for (kde::JobGraph& g : c->graphs)
      if (g.exec && g.sig == sig && g.blocks == c->blocks.p && g.st == c->st.p && g.blob == c->blob.p &&
          g.sort_tmp == c->sort_tmp.p && !g.plans.empty())
        return replay_job(c, g, reqs);
  }
  c->plans.clear();
  c->plan_req.clear();
  for (int32_t k = 0; k < n_req; ++k) {
    kde::ColPlan p;
    std::string e = kde::plan_column(c, reqs[k], p);
    if (!e.empty()) {
      st[k] = KDE_E_INVAL;
      msg[k] = e;
      continue;
    }
    c->plans.push_back(std::move(p));
    c->plan_req.push_back(k);
  }
  const int n_cols = (int)c->plans.size();
  if (n_cols == 0) return KDE_OK;
  size_t total = 0;
  std::vector<size_t> at(n_cols);
  for (int k = 0; k < n_cols; ++k) {
    at[k] = total;
    total += (c->plans[k].bytes + 255) / 256 * 256;
  }
  if ((s = kde::ensure(c, c->blocks, total))) return s;
  if ((s = kde::ensure(c, c->st, (size_t)n_cols))) return s;
  char* hs = reinterpret_cast<char*>(c->h_st);
  if ((s = kde::ensure_pinned_bytes(c, hs, c->h_st_cap, sizeof(DevState) * n_cols))) return s;
  c->h_st = reinterpret_cast<DevState*>(hs);
  kde::IterPlan& it = c->iter;
  it.clear();
  int extra = n_cols;  // tile pruning: two more descriptors per pruned column
  for (int k = 0; k < n_cols; ++k) {
    const kde::ColPlan& p = c->plans[k];
    const kde_request& r = reqs[c->plan_req[k]];
    ColDesc d;
    kde::bind_column(p, c->blocks.p + at[k], r.x.data, c->st.p + k, d);
    kde::add_full_column(c, p, d, k, r.x.data, it, p.prune ? extra : -1);
    if (p.prune) extra += 2;
    kde::init_state(p, c->opt_fp64_kappa, c->h_st[k]);
  }
  KDE_HIP_TRY(c, hipMemcpyAsync(c->st.p, c->h_st, sizeof(DevState) * n_cols, hipMemcpyHostToDevice, c->stream));
  if (use_graph)
    s = capture_job(c, std::move(sig));
  else
    s = kde::execute(c, it);
  if (s) return s;
  KDE_HIP_TRY(c, hipMemcpyAsync(c->h_st, c->st.p, sizeof(DevState) * n_cols, hipMemcpyDeviceToHost, c->stream));
  return KDE_OK;
}

kde_status run_single(kde_ctx* c, const kde_request& r) {
  std::vector<kde_status> st;
  std::vector<std::string> msg;
  kde_status s = run_requests(c, &r, 1, st, msg);
  if (s) return s;
  if (st[0] != KDE_OK) return fail(c, st[0], msg[0]);
  return KDE_OK;
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

}  // namespace

kde_status kde::stage_column(kde_ctx* c, kde_column x, const kde::ColDesc** dcol) {
  kde_status s;
  if ((s = run_single(c, make_req(x, KDE_METHOD_ROT, 2, nullptr, 0)))) return s;
  if ((s = kde::sync_and_check(c))) return s;
  if (c->h_st[0].status == kde::kStInval) return kde::fail(c, KDE_E_INVAL, "sample column holds a non-finite value");
  *dcol = reinterpret_cast<const kde::ColDesc*>(c->blob.p);  // the pass's column table starts the blob
  return KDE_OK;
}

namespace {

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

kde_status ensure_out(kde_ctx* c, size_t doubles) {
  char* p = reinterpret_cast<char*>(c->h_out);
  size_t cap = c->h_out_cap * sizeof(double);
  kde_status s = kde::ensure_pinned_bytes(c, p, cap, doubles * sizeof(double));
  c->h_out = reinterpret_cast<double*>(p);
  c->h_out_cap = cap / sizeof(double);
  return s;
}

}  // namespace

// exported for the server (kde_server.hip)
namespace kde {
void init_result(kde_result& r, kde_status st) {
  double* g_keep = r.g_out;
  double* gs_keep = r.gscale_out;
  std::memset(&r, 0, sizeof(r));
  r.g_out = g_keep;
  r.gscale_out = gs_keep;
  r.status = st;
  const double nan = std::nan("");
  r.sigma = r.h_rot = r.h_plugin = r.h_lscv = nan;
  r.k_lscv = -1;
}

void fill_result(const ColPlan& p, const DevState& h, kde_result& r) {
  r.status = status_of(h.status);
  if (r.status == KDE_OK && p.plugin) r.status = status_of(h.pstatus);
  r.sigma = h.sigma;
  r.h_rot = h.h_rot;
  if (p.plugin) {
    fill_plugin_info(h, p.stages, &r.plugin);
    r.h_plugin = h.h_plugin;
  }
  if (p.lscv) {
    r.h_lscv = h.h_best;
    r.k_lscv = h.k_best;
    r.at_edge = h.at_edge;
    r.lscv_evals_dense = 0.5 * (double)p.n * (double)(p.n - 1) * (double)p.n_h;
    r.lscv_evals = r.lscv_evals_dense - h.pruned_evals;
  }
}
}  // namespace kde

kde_status kde::lscv_curve_call(kde_ctx* c, kde_column x, const double* h_grid, int32_t n_h, double* g_out,
                                double* gscale_out, double* grid_out) {
  kde_status s;
  if (!h_grid && n_h <= 0) n_h = 150;
  if ((s = run_single(c, make_req(x, KDE_METHOD_LSCV, 2, h_grid, n_h)))) return s;
  if ((s = ensure_out(c, (size_t)3 * n_h))) return s;
  const ColDesc& d = c->iter.cols[0];
  KDE_HIP_TRY(c, hipMemcpyAsync(c->h_out, d.g, sizeof(double) * n_h, hipMemcpyDeviceToHost, c->stream));
  KDE_HIP_TRY(c, hipMemcpyAsync(c->h_out + n_h, d.gs, sizeof(double) * n_h, hipMemcpyDeviceToHost, c->stream));
  KDE_HIP_TRY(c, hipMemcpyAsync(c->h_out + 2 * (size_t)n_h, d.h, sizeof(double) * n_h, hipMemcpyDeviceToHost,
                                c->stream));
  if ((s = kde::sync_and_check(c))) return s;
  if ((s = map_status(c, c->h_st[0].status))) return s;
  std::memcpy(g_out, c->h_out, sizeof(double) * n_h);
  if (gscale_out) std::memcpy(gscale_out, c->h_out + n_h, sizeof(double) * n_h);
  if (grid_out) std::memcpy(grid_out, c->h_out + 2 * (size_t)n_h, sizeof(double) * n_h);
  return KDE_OK;
}

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
  kde::noalloc_setup(c);
  *out = c;
  return KDE_OK;
}

kde_status kde_server_stop(kde_ctx* c);

void kde_ctx_destroy(kde_ctx* c) {
  if (!c) return;
  if (c->server) (void)kde_server_stop(c);
  c->server.reset();
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  // handles created on the context and not yet released
  while (!c->preps.empty()) kde_lscv_H_release(c->preps.back());
  while (!c->jobs.empty()) kde_job_destroy(c->jobs.back());
  (void)hipFree(c->stage.p);
  (void)hipFree(c->blocks.p);
  (void)hipFree(c->st.p);
  (void)hipFree(c->blob.p);
  (void)hipFree(c->tune_buf.p);
  (void)hipFree(c->sort_tmp.p);
  (void)hipFree(c->qbuf.p);
  (void)hipFree(c->mdbuf.p);
  for (kde::JobGraph& g : c->graphs) g.reset();
  if (c->h_st) (void)hipHostFree(c->h_st);
  if (c->h_out) (void)hipHostFree(c->h_out);
  if (c->h_blob) (void)hipHostFree(c->h_blob);
  for (kde_ctx::Pending& p : c->pending) {
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
  if (serving(c)) return busy(c);
  c->stream = hip_stream ? (hipStream_t)hip_stream : c->own;
  return KDE_OK;
}

kde_status kde_ctx_set_precision(kde_ctx* c, kde_prec prec) {
  if (!c) return KDE_E_INVAL;
  if (serving(c)) return busy(c);
  if (prec != KDE_PREC_MIXED && prec != KDE_PREC_FP64) return fail(c, KDE_E_INVAL, "unknown precision");
  c->prec = prec;
  return KDE_OK;
}

kde_status kde_ctx_set_option(kde_ctx* c, const char* key, int64_t value) {
  if (!c || !key) return KDE_E_INVAL;
  if (serving(c)) return busy(c);
  const std::string k(key);
  if (k == "lscv_hc") {
    if (value < 0) value = 16;
    if (value != 8 && value != 16 && value != 32) return fail(c, KDE_E_INVAL, "lscv_hc must be 8, 16 or 32");
    c->opt_hc = (int)value;
  } else if (k == "seg") {
    c->opt_seg = value < 0 ? -1 : value;
  } else if (k == "launch_evals") {
    c->opt_launch_evals = value <= 0 ? 4e12 : (double)value;
  } else if (k == "lscv_tj") {
    if (value < 0) value = 512;
    if (value != 256 && value != 512 && value != 1024) return fail(c, KDE_E_INVAL, "lscv_tj must be 256, 512 or 1024");
    c->opt_tj = (int)value;
  } else if (k == "fp64_kappa") {
    c->opt_fp64_kappa = value < 0 ? 1e3 : (double)value;
  } else if (k == "lscv_mfma") {
    c->opt_mfma = value < 0 ? 0 : (value != 0);
  } else if (k == "prune") {
    c->opt_prune = value < 0 ? 0 : (value != 0);
  } else if (k == "persistent") {
    c->opt_persistent = value < 0 ? 1 : (value != 0);
  } else if (k == "graph") {
    c->opt_graph = value < 0 ? 0 : (value != 0);
  } else if (k == "autotune") {
    c->opt_autotune = value < 0 ? 0 : (value != 0);
  } else if (k == "serve_iter_evals") {
    c->opt_serve_iter_evals = value <= 0 ? 1e12 : (double)value;
  } else if (k == "serve_iter_ms") {
    c->opt_serve_iter_s = value <= 0 ? 0.0 : (double)value * 1e-3;
  } else if (k == "serve_aging_ms") {
    c->opt_serve_aging_s = value <= 0 ? 0.0 : (double)value * 1e-3;
  } else if (k == "serve_fail_ticket") {
    c->opt_serve_fail_ticket = value <= 0 ? 0 : (uint64_t)value;
  } else {
    return fail(c, KDE_E_INVAL, "unknown option " + k);
  }
  return KDE_OK;
}

kde_status kde_request_footprint(const kde_ctx* c, const kde_request* r, uint64_t* bytes) {
  if (!r || !bytes) return KDE_E_INVAL;
  if (c && serving(c)) return KDE_E_BUSY;
  // the planner reads only the options: a context-free copy of them
  kde_ctx o;
  if (c) {
    o.prec = c->prec;
    o.opt_hc = c->opt_hc;
    o.opt_seg = c->opt_seg;
    o.opt_launch_evals = c->opt_launch_evals;
    o.opt_fp64_kappa = c->opt_fp64_kappa;
    o.opt_prune = c->opt_prune;
  }
  o.job_hc = o.opt_hc;
  kde::ColPlan p;
  if (!kde::plan_column(&o, *r, p).empty()) return KDE_E_INVAL;
  *bytes = (uint64_t)((p.bytes + 255) / 256 * 256);
  return KDE_OK;
}

kde_status kde_plan_items(int64_t n, int32_t n_h, int64_t seg, int32_t cap, int32_t* n_items, int32_t* row_begin,
                          int32_t* j_begin, int32_t* j_end, double* pairs) {
  if (n < 2 || n > KDE_MAX_N || n_h < 0 || n_h > KDE_MAX_NH || cap < 0 || !n_items) return KDE_E_INVAL;
  if (cap > 0 && (!row_begin || !j_begin || !j_end || !pairs)) return KDE_E_INVAL;
  kde_ctx o;
  o.opt_seg = seg < 0 ? -1 : seg;
  kde::ColItems it;
  if (n_h > 0)
    kde::make_items(n, kde::capped_seg(&o, n, kde::kSegRefHC, (double)((n_h + kde::kSegRefHC - 1) / kde::kSegRefHC)),
                    it);
  else
    kde::make_items(n, kde::capped_seg(&o, n, kde::kSegRefHC, 1.0), it);
  const int32_t m = (int32_t)it.pairs.size();
  *n_items = m;
  for (int32_t k = 0; k < std::min(m, cap); ++k) {
    row_begin[k] = it.row[k] * kde::kBI;
    j_begin[k] = it.jb[k];
    j_end[k] = it.je[k];
    pairs[k] = it.pairs[k];
  }
  return KDE_OK;
}

kde_status kde_ctx_graph_stats(kde_ctx* c, int64_t* captures, int64_t* replays) {
  if (!c || !captures || !replays) return KDE_E_INVAL;
  *captures = c->graph_captures;
  *replays = c->graph_replays;
  return KDE_OK;
}

kde_status kde_ctx_set_timing(kde_ctx* c, int enable) {
  if (!c) return KDE_E_INVAL;
  if (serving(c)) return busy(c);
  c->timing = enable != 0;
  for (int f = 0; f < 3; ++f) {
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
    f = kde::kFamLscv;
  else if (!std::strcmp(family, "psi_pairs"))
    f = kde::kFamPsi;
  else if (!std::strcmp(family, "md_pairs"))
    f = kde::kFamMd;
  else
    return fail(c, KDE_E_INVAL, "unknown kernel family");
  if (launches) *launches = c->t_launches[f];
  if (total_ms) *total_ms = c->t_ms[f];
  if (evals) *evals = c->t_evals[f];
  return KDE_OK;
}

kde_status kde_bw_rot(kde_ctx* c, kde_column x, double* h_out) {
  if (!c || !h_out) return KDE_E_INVAL;
  if (serving(c)) return busy(c);
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  if ((s = run_single(c, make_req(x, KDE_METHOD_ROT, 2, nullptr, 0)))) return s;
  if ((s = kde::sync_and_check(c))) return s;
  if ((s = map_status(c, c->h_st[0].status))) return s;
  *h_out = c->h_st[0].h_rot;
  return KDE_OK;
}

kde_status kde_bw_plugin(kde_ctx* c, kde_column x, int stages, double* h_out, kde_plugin_info* info) {
  if (!c || !h_out) return KDE_E_INVAL;
  if (serving(c)) return busy(c);
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  if ((s = run_single(c, make_req(x, KDE_METHOD_PLUGIN, stages, nullptr, 0)))) return s;
  if ((s = kde::sync_and_check(c))) return s;
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
  if (serving(c)) return busy(c);
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  return kde::lscv_curve_call(c, x, h_grid, n_h, g_out, gscale_out, grid_out);
}

kde_status kde_lscv_sums(kde_ctx* c, kde_column x, const double* h_grid, int32_t n_h, double* s1_out,
                         double* s2_out) {
  if (!c || !h_grid || !s1_out || !s2_out) return KDE_E_INVAL;
  if (serving(c)) return busy(c);
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  if ((s = run_single(c, make_req(x, KDE_METHOD_LSCV, 2, h_grid, n_h)))) return s;
  if ((s = ensure_out(c, (size_t)2 * n_h))) return s;
  KDE_HIP_TRY(c, hipMemcpyAsync(c->h_out, c->iter.cols[0].sums, sizeof(double) * 2 * n_h, hipMemcpyDeviceToHost,
                                c->stream));
  if ((s = kde::sync_and_check(c))) return s;
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
  if (serving(c)) return busy(c);
  if (n_sel > 0 && (!sel || !ranges_out || !sums_out)) return fail(c, KDE_E_INVAL, "NULL selection buffers");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  if ((s = run_single(c, make_req(x, KDE_METHOD_LSCV, 2, h_grid, n_h)))) return s;
  const kde::ColPlan& p = c->plans[0];
  const ColDesc& d = c->iter.cols[0];
  const int32_t n_items = d.n_items;
  std::vector<int32_t> idx((size_t)n_sel);
  for (int32_t k = 0; k < n_sel; ++k) {
    idx[k] = sel[k] < 0 ? n_items + sel[k] : sel[k];
    if (idx[k] < 0 || idx[k] >= n_items) {
      (void)hipStreamSynchronize(c->stream);
      return fail(c, KDE_E_INVAL, "item index out of range");
    }
  }
  if ((s = ensure_out(c, (size_t)2 * n_h * (n_sel > 0 ? n_sel : 1)))) return s;
  // the column's partials are laid out [2*n_h][n_items]: one strided column per selected item
  for (int32_t k = 0; k < n_sel; ++k)
    KDE_HIP_TRY(c, hipMemcpy2DAsync(c->h_out + (size_t)k * 2 * n_h, sizeof(double), d.part + idx[k],
                                    sizeof(double) * (size_t)n_items, sizeof(double), (size_t)2 * n_h,
                                    hipMemcpyDeviceToHost, c->stream));
  if ((s = kde::sync_and_check(c))) return s;
  if ((s = map_status(c, c->h_st[0].status))) return s;
  *n_items_out = n_items;
  for (int32_t k = 0; k < n_sel; ++k) {
    ranges_out[3 * k] = p.lscv_items.row[idx[k]] * kde::kBI;
    ranges_out[3 * k + 1] = p.lscv_items.jb[idx[k]];
    ranges_out[3 * k + 2] = p.lscv_items.je[idx[k]];
    std::memcpy(sums_out + (size_t)k * 2 * n_h, c->h_out + (size_t)k * 2 * n_h, sizeof(double) * 2 * n_h);
  }
  return KDE_OK;
}

kde_status kde_bw_lscv(kde_ctx* c, kde_column x, const double* h_grid, int32_t n_h, double* h_out, int32_t* k_out,
                       int* at_edge) {
  if (!c || !h_out) return KDE_E_INVAL;
  if (serving(c)) return busy(c);
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  if (!h_grid && n_h <= 0) n_h = 150;
  if ((s = run_single(c, make_req(x, KDE_METHOD_LSCV, 2, h_grid, n_h)))) return s;
  if ((s = kde::sync_and_check(c))) return s;
  if ((s = map_status(c, c->h_st[0].status))) return s;
  *h_out = c->h_st[0].h_best;
  if (k_out) *k_out = c->h_st[0].k_best;
  if (at_edge) *at_edge = c->h_st[0].at_edge;
  return KDE_OK;
}

kde_status kde_bw_lscv_min(kde_ctx* c, kde_column x, double h_lo, double h_hi, double rel_tol, int32_t points,
                           double* h_out, kde_lscv_min_info* info) {
  if (!c || !h_out) return KDE_E_INVAL;
  if (serving(c)) return busy(c);
  if (!(h_lo > 0.0) || !(h_hi > h_lo) || !std::isfinite(h_hi) || !(rel_tol > 0.0) || points < 4 ||
      points > KDE_MAX_NH)
    return fail(c, KDE_E_INVAL, "need 0 < h_lo < h_hi finite, rel_tol > 0 and 4 <= points <= KDE_MAX_NH");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  std::vector<double> grid((size_t)points), gval((size_t)points);
  double a = h_lo, b = h_hi, best_h = 0.0, best_g = 0.0;
  int it = 0;
  int64_t evaluated = 0;
  for (; it < 200; ++it) {
    // points log-spaced over the bracket, ends included
    for (int32_t j = 0; j < points; ++j) grid[j] = a * std::pow(b / a, (double)j / (double)(points - 1));
    grid[points - 1] = b;
    bool ascending = true;
    for (int32_t j = 1; j < points; ++j) ascending = ascending && grid[j] > grid[j - 1];
    if (!ascending) break;  // the bracket is below the FP64 resolution of h
    if ((s = run_single(c, make_req(x, KDE_METHOD_LSCV, 2, grid.data(), points)))) return s;
    if ((s = ensure_out(c, (size_t)points))) return s;
    KDE_HIP_TRY(c, hipMemcpyAsync(c->h_out, c->iter.cols[0].g, sizeof(double) * points, hipMemcpyDeviceToHost,
                                  c->stream));
    if ((s = kde::sync_and_check(c))) return s;
    if ((s = map_status(c, c->h_st[0].status))) return s;
    std::memcpy(gval.data(), c->h_out, sizeof(double) * points);
    evaluated += points;
    const int k = c->h_st[0].k_best;
    best_h = grid[k];
    best_g = gval[k];
    if (b / a - 1.0 <= rel_tol) {
      ++it;
      break;
    }
    const double na = grid[k > 0 ? k - 1 : 0], nb = grid[k < points - 1 ? k + 1 : points - 1];
    a = na;
    b = nb;
  }
  *h_out = best_h;
  if (info) {
    info->g = best_g;
    info->iterations = it;
    info->evaluated = evaluated;
    info->bracket_lo = a;
    info->bracket_hi = b;
  }
  return KDE_OK;
}

kde_status kde_batch(kde_ctx* c, const kde_request* reqs, int32_t n_req, kde_result* out) {
  if (!c || n_req < 0 || (n_req > 0 && (!reqs || !out))) return KDE_E_INVAL;
  if (serving(c)) return busy(c);
  if (n_req > KDE_MAX_BATCH) return fail(c, KDE_E_INVAL, "more than KDE_MAX_BATCH requests");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  std::vector<kde_status> st;
  std::vector<std::string> msg;
  kde_status s;
  if ((s = run_requests(c, reqs, n_req, st, msg))) return s;
  const int n_cols = (int)c->plans.size();
  // g / gscale of LSCV requests into pinned staging, then to the caller
  size_t total = 0;
  for (const kde::ColPlan& p : c->plans)
    if (p.lscv) total += 2 * (size_t)p.n_h;
  if ((s = ensure_out(c, std::max<size_t>(total, 1)))) return s;
  size_t o = 0;
  std::vector<size_t> at(n_cols, 0);
  for (int k = 0; k < n_cols; ++k) {
    const kde::ColPlan& p = c->plans[k];
    if (!p.lscv) continue;
    const ColDesc& d = c->iter.cols[k];
    at[k] = o;
    KDE_HIP_TRY(c, hipMemcpyAsync(c->h_out + o, d.g, sizeof(double) * p.n_h, hipMemcpyDeviceToHost, c->stream));
    KDE_HIP_TRY(c, hipMemcpyAsync(c->h_out + o + p.n_h, d.gs, sizeof(double) * p.n_h, hipMemcpyDeviceToHost,
                                  c->stream));
    o += 2 * (size_t)p.n_h;
  }
  if ((s = kde::sync_and_check(c))) return s;
  for (int32_t k = 0; k < n_req; ++k) kde::init_result(out[k], st[k]);
  for (int k = 0; k < n_cols; ++k) {
    const kde::ColPlan& p = c->plans[k];
    kde_result& r = out[c->plan_req[k]];
    kde::fill_result(p, c->h_st[k], r);
    if (p.lscv) {
      if (r.g_out) std::memcpy(r.g_out, c->h_out + at[k], sizeof(double) * p.n_h);
      if (r.gscale_out) std::memcpy(r.gscale_out, c->h_out + at[k] + p.n_h, sizeof(double) * p.n_h);
    }
  }
  return KDE_OK;
}

}  // extern "C"
