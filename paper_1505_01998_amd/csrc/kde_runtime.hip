// kde_runtime.hip -- host runtime and C ABI of the bandwidth-selection library.
//
// A call is a chain of kernels on one stream: ingest + moments (FP64, two
// passes), the device-side scalar steps of the selector, the pair kernels
// (split into launches of bounded work), fixed-order FP64 reductions and a
// finalize kernel; one device-to-host copy at the end returns the results.
// No step runs on the host except argument checks and work-list planning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kde_bw.h"
#include "kde_internal.h"

using kde::DevState;
using kde::Item;

namespace {

struct Pending {
  hipEvent_t a, b;
  int family;
  double evals;
};

struct Plan {
  int64_t n = -1;
  int64_t seg = -1;
  std::vector<Item> items;
  std::vector<double> pairs;  // algorithmic i<j pairs of each item
  double total_pairs = 0.0;
  Item* d_items = nullptr;
  size_t cap = 0;
};

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;
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
  int64_t opt_seg = -1;           // <0 automatic, 0 whole rows, >0 explicit
  double opt_launch_evals = 4e12;  // pair-term evaluations per launch
  double opt_fp64_kappa = 1e3;
  // device workspace
  DevBuf<char> stage;
  DevBuf<float> x32;
  DevBuf<double> x64;
  DevBuf<double> part;
  DevBuf<int> part_nf;
  DevBuf<double> stat_part;
  DevBuf<double> sums;
  DevBuf<double> hin, hdev, c64, g, gs;
  DevBuf<float> c32;
  DevState* d_st = nullptr;
  // pinned host staging
  DevState* h_st = nullptr;
  double* h_out = nullptr;
  size_t h_out_cap = 0;
  // work lists (one per segment length in use)
  Plan plans[2];
  int plan_next = 0;
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

#define HIP_TRY(ctx, expr)                                                                         \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
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

kde_status ensure_host_out(kde_ctx* c, size_t count) {
  if (c->h_out_cap >= count) return KDE_OK;
  if (c->h_out) (void)hipHostFree(c->h_out);
  c->h_out = nullptr;
  c->h_out_cap = 0;
  size_t want = std::max<size_t>(count, 4096);
  if (hipHostMalloc((void**)&c->h_out, want * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    c->h_out = nullptr;
    return fail(c, KDE_E_NOMEM, "pinned host allocation failed");
  }
  c->h_out_cap = want;
  return KDE_OK;
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

// ---- column ingest and moments
kde_status check_column(kde_ctx* c, const kde_column& x) {
  if (!x.data) return fail(c, KDE_E_INVAL, "column data is NULL");
  if (x.n < 2) return fail(c, KDE_E_INVAL, "a sample column needs n >= 2");
  if (x.n > KDE_MAX_N) return fail(c, KDE_E_INVAL, "n exceeds KDE_MAX_N");
  if (x.dtype != KDE_F32 && x.dtype != KDE_F64) return fail(c, KDE_E_INVAL, "dtype must be KDE_F32 or KDE_F64");
  return KDE_OK;
}

kde_status init_state(kde_ctx* c, int stages) {
  DevState& h = *c->h_st;
  std::memset(&h, 0, sizeof(h));
  const double nan = std::nan("");
  h.stages = stages;
  for (int k = 0; k < 3; ++k) {
    h.g[k] = h.psi[k] = h.kappa[k] = nan;
    h.prec_used[k] = -1;
  }
  h.h_plugin = h.h_best = h.margin = nan;
  h.k_best = -1;
  h.fp64_kappa = c->opt_fp64_kappa;
  HIP_TRY(c, hipMemcpyAsync(c->d_st, c->h_st, sizeof(DevState), hipMemcpyHostToDevice, c->stream));
  return KDE_OK;
}

// Stages the column on the device and runs the two moment passes; afterwards
// x32 (and x64 when requested) hold the padded sample.  Host copies of the
// state are not refreshed here.
kde_status prepare_column(kde_ctx* c, const kde_column& x, bool want_x64, int stages) {
  kde_status s = check_column(c, x);
  if (s) return s;
  const int n = (int)x.n;
  const int is_f64 = x.dtype == KDE_F64;
  const size_t esz = is_f64 ? 8 : 4;
  const int n_pad = n + kde::kPad;
  if ((s = init_state(c, stages))) return s;
  const void* src = x.data;
  if (!x.on_device) {
    if ((s = ensure(c, c->stage, (size_t)n * esz))) return s;
    HIP_TRY(c, hipMemcpyAsync(c->stage.p, x.data, (size_t)n * esz, hipMemcpyHostToDevice, c->stream));
    src = c->stage.p;
  }
  if ((s = ensure(c, c->x32, (size_t)n_pad))) return s;
  if (want_x64 && (s = ensure(c, c->x64, (size_t)n_pad))) return s;
  const int nblk = std::max(1, std::min(1024, (n + 2047) / 2048));
  if ((s = ensure(c, c->stat_part, (size_t)nblk))) return s;
  if ((s = ensure(c, c->part_nf, (size_t)nblk))) return s;
  kde::launch_stats_sum(c->stream, src, is_f64, n, c->stat_part.p, c->part_nf.p, nblk);
  kde::launch_stats_mean(c->stream, c->stat_part.p, c->part_nf.p, nblk, n, is_f64, c->d_st);
  kde::launch_stats_dev(c->stream, src, is_f64, n, n_pad, c->stat_part.p, c->x32.p, want_x64 ? c->x64.p : nullptr,
                        nblk, c->d_st);
  kde::launch_stats_final(c->stream, c->stat_part.p, nblk, c->d_st);
  HIP_TRY(c, hipGetLastError());
  return KDE_OK;
}

// ---- work lists
double item_pairs(int64_t n, const Item& it) {
  const int64_t i0 = (int64_t)it.row * kde::kBI;
  const int64_t i1 = std::min<int64_t>(n, i0 + kde::kBI);
  const int64_t je = std::min<int64_t>(it.j_end, n);
  double p = 0.0;
  for (int64_t i = i0; i < i1; ++i) {
    const int64_t jb = std::max<int64_t>(it.j_begin, i + 1);
    if (je > jb) p += (double)(je - jb);
  }
  return p;
}

// seg: j-range per item in samples (multiple of kBJ), or 0 for whole rows.
kde_status get_plan(kde_ctx* c, int64_t n, int64_t seg, Plan** out) {
  for (Plan& p : c->plans)
    if (p.n == n && p.seg == seg) {
      *out = &p;
      return KDE_OK;
    }
  Plan& p = c->plans[c->plan_next];
  c->plan_next ^= 1;
  p.n = -1;
  p.items.clear();
  p.pairs.clear();
  p.total_pairs = 0.0;
  const int64_t rows = (n + kde::kBI - 1) / kde::kBI;
  for (int64_t r = 0; r < rows; ++r) {
    const int64_t row0 = r * kde::kBI;
    const int64_t len = ((n - row0) + kde::kBJ - 1) / kde::kBJ * kde::kBJ;
    const int64_t step = seg > 0 ? seg : len;
    for (int64_t jb = row0; jb < row0 + len; jb += step) {
      Item it;
      it.row = (int)r;
      it.j_begin = (int)jb;
      it.j_end = (int)std::min(jb + step, row0 + len);
      it.pad = 0;
      const double pr = item_pairs(n, it);
      if (pr <= 0.0) continue;
      p.items.push_back(it);
      p.pairs.push_back(pr);
      p.total_pairs += pr;
    }
  }
  // longest first: the block scheduler then drains the triangle largest-first
  std::vector<size_t> order(p.items.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return p.pairs[a] > p.pairs[b]; });
  std::vector<Item> items(order.size());
  std::vector<double> pairs(order.size());
  for (size_t k = 0; k < order.size(); ++k) {
    items[k] = p.items[order[k]];
    pairs[k] = p.pairs[order[k]];
  }
  p.items.swap(items);
  p.pairs.swap(pairs);
  if (p.cap < p.items.size()) {
    if (p.d_items) (void)hipFree(p.d_items);
    p.d_items = nullptr;
    p.cap = 0;
    if (hipMalloc((void**)&p.d_items, p.items.size() * sizeof(Item)) != hipSuccess)
      return fail(c, KDE_E_NOMEM, "device allocation of the work list failed");
    p.cap = p.items.size();
  }
  // The stream is idle between calls, so the host vector outlives the copy.
  HIP_TRY(c, hipMemcpyAsync(p.d_items, p.items.data(), p.items.size() * sizeof(Item), hipMemcpyHostToDevice,
                            c->stream));
  p.n = n;
  p.seg = seg;
  *out = &p;
  return KDE_OK;
}

// Item length for a pass whose blocks each evaluate `hc` terms per pair.
int64_t pick_seg(kde_ctx* c, int64_t n, int hc) {
  if (c->opt_seg >= 0) return c->opt_seg == 0 ? 0 : (c->opt_seg + kde::kBJ - 1) / kde::kBJ * kde::kBJ;
  // Aim for ~8192 blocks per launch so each launch fills the chip many times.
  const double per_block_pairs = c->opt_launch_evals / 8192.0 / (double)hc;
  int64_t seg = (int64_t)(per_block_pairs / kde::kBI);
  seg = std::max<int64_t>(kde::kBJ, seg / kde::kBJ * kde::kBJ);
  if (seg >= n) return 0;
  return seg;
}

// Launch ranges over items [i0, i1) whose summed evaluations stay within budget.
// FP64 terms cost about five times the FP32 ones, so their budget is smaller.
template <typename F>
kde_status for_each_launch(kde_ctx* c, const Plan& p, double evals_per_pair, bool f64, F&& launch) {
  const double budget = f64 ? c->opt_launch_evals / 5.0 : c->opt_launch_evals;
  const size_t m = p.items.size();
  size_t i0 = 0;
  while (i0 < m) {
    double acc = p.pairs[i0] * evals_per_pair;
    size_t i1 = i0 + 1;
    while (i1 < m && acc + p.pairs[i1] * evals_per_pair <= budget) {
      acc += p.pairs[i1] * evals_per_pair;
      ++i1;
    }
    kde_status s = launch((int)i0, (int)(i1 - i0), acc);
    if (s) return s;
    i0 = i1;
  }
  return KDE_OK;
}

kde_status read_state(kde_ctx* c) {
  HIP_TRY(c, hipMemcpyAsync(c->h_st, c->d_st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
  return KDE_OK;
}

// ---- plug-in
kde_status run_psi_stage(kde_ctx* c, int n, int stage, bool f64, bool conditional, const Plan& p) {
  const int r = 8 - 2 * stage;
  kde_status s;
  if ((s = ensure(c, c->part, 2 * p.items.size()))) return s;
  s = for_each_launch(c, p, 1.0, f64, [&](int i0, int cnt, double evals) -> kde_status {
    // A conditional pass may exit at once on the device, so it is not timed.
    Pending pd{nullptr, nullptr, kFamPsi, evals};
    kde_status s2 = conditional ? KDE_OK : timed_begin(c, pd);
    if (s2) return s2;
    kde::launch_psi_pairs(c->stream, r, f64 ? 1 : 0, conditional ? 1 : 0, c->x32.p, c->x64.p, n, p.d_items,
                          (int)p.items.size(), i0, cnt, c->part.p, c->d_st);
    return conditional ? KDE_OK : timed_end(c, pd);
  });
  if (s) return s;
  kde::launch_reduce_rows(c->stream, c->part.p, (int)p.items.size(), 2, c->sums.p);
  kde::launch_psi_finish(c->stream, c->d_st, stage, c->sums.p, f64 ? 1 : 0, conditional ? 1 : 0);
  HIP_TRY(c, hipGetLastError());
  return KDE_OK;
}

kde_status run_plugin(kde_ctx* c, const kde_column& x, int stages) {
  if (stages != 2 && stages != 3) return fail(c, KDE_E_INVAL, "stages must be 2 or 3");
  kde_status s;
  if ((s = prepare_column(c, x, true, stages))) return s;
  const int n = (int)x.n;
  if ((s = ensure(c, c->sums, 64))) return s;
  Plan* p = nullptr;
  if ((s = get_plan(c, n, pick_seg(c, n, 1), &p))) return s;
  const bool all64 = c->prec == KDE_PREC_FP64;
  for (int stage = (stages == 3 ? 0 : 1); stage < 3; ++stage) {
    kde::launch_psi_begin(c->stream, c->d_st, stage);
    if ((s = run_psi_stage(c, n, stage, all64, false, *p))) return s;
    if (!all64 && c->opt_fp64_kappa > 0.0 && (s = run_psi_stage(c, n, stage, true, true, *p))) return s;
  }
  kde::launch_plugin_final(c->stream, c->d_st);
  HIP_TRY(c, hipGetLastError());
  return KDE_OK;
}

// ---- LSCV
kde_status check_grid(kde_ctx* c, const double* h, int32_t n_h) {
  if (n_h < 1 || n_h > KDE_MAX_NH) return fail(c, KDE_E_INVAL, "n_h out of range");
  for (int32_t k = 0; k < n_h; ++k) {
    if (!(h[k] > 0.0) || !std::isfinite(h[k])) return fail(c, KDE_E_INVAL, "grid values must be finite and > 0");
    if (k > 0 && !(h[k] > h[k - 1])) return fail(c, KDE_E_INVAL, "grid must be strictly ascending");
  }
  return KDE_OK;
}

// Runs the LSCV pass; results stay on the device (sums, g, gscale, hdev, state).
kde_status run_lscv(kde_ctx* c, const kde_column& x, const double* h_grid, int32_t n_h, Plan** plan_out = nullptr) {
  kde_status s;
  if (h_grid) {
    if ((s = check_grid(c, h_grid, n_h))) return s;
  } else {
    if (n_h <= 0) n_h = 150;
    if (n_h > KDE_MAX_NH) return fail(c, KDE_E_INVAL, "n_h out of range");
  }
  const bool all64 = c->prec == KDE_PREC_FP64;
  if ((s = prepare_column(c, x, all64, 2))) return s;
  const int n = (int)x.n;
  const int hc = all64 ? 8 : c->opt_hc;
  const int n_chunks = (n_h + hc - 1) / hc;
  const int n_h_pad = n_chunks * hc;
  if ((s = ensure(c, c->hin, (size_t)n_h))) return s;
  if ((s = ensure(c, c->hdev, (size_t)n_h))) return s;
  if ((s = ensure(c, c->c32, (size_t)n_h_pad))) return s;
  if ((s = ensure(c, c->c64, (size_t)n_h_pad))) return s;
  if ((s = ensure(c, c->g, (size_t)n_h))) return s;
  if ((s = ensure(c, c->gs, (size_t)n_h))) return s;
  if ((s = ensure(c, c->sums, (size_t)2 * n_h + 64))) return s;
  if (h_grid) HIP_TRY(c, hipMemcpyAsync(c->hin.p, h_grid, sizeof(double) * n_h, hipMemcpyHostToDevice, c->stream));
  kde::launch_lscv_prep(c->stream, h_grid ? c->hin.p : nullptr, n_h, n_h_pad, c->d_st, c->hdev.p, c->c32.p,
                        c->c64.p);
  Plan* p = nullptr;
  if ((s = get_plan(c, n, pick_seg(c, n, hc), &p))) return s;
  const size_t n_items = p->items.size();
  if ((s = ensure(c, c->part, (size_t)2 * n_h * n_items))) return s;
  s = for_each_launch(c, *p, (double)n_h, all64, [&](int i0, int cnt, double evals) -> kde_status {
    Pending pd{nullptr, nullptr, kFamLscv, evals};
    kde_status s2 = timed_begin(c, pd);
    if (s2) return s2;
    kde::launch_lscv_pairs(c->stream, hc, all64 ? 1 : 0, c->x32.p, c->x64.p, n, p->d_items, (int)n_items, n_chunks,
                           c->c32.p, c->c64.p, n_h, i0 * n_chunks, cnt * n_chunks, c->part.p, c->d_st);
    return timed_end(c, pd);
  });
  if (s) return s;
  kde::launch_reduce_rows(c->stream, c->part.p, (int)n_items, 2 * n_h, c->sums.p);
  kde::launch_lscv_finalize(c->stream, c->sums.p, n_h, c->hdev.p, c->d_st, c->g.p, c->gs.p);
  HIP_TRY(c, hipGetLastError());
  if (plan_out) *plan_out = p;
  return KDE_OK;
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
  if (hipMalloc((void**)&c->d_st, sizeof(DevState)) != hipSuccess ||
      hipHostMalloc((void**)&c->h_st, sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
    kde_ctx_destroy(c);
    return KDE_E_NOMEM;
  }
  *out = c;
  return KDE_OK;
}

void kde_ctx_destroy(kde_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto* b : {&c->stage}) (void)hipFree(b->p);
  (void)hipFree(c->x32.p);
  (void)hipFree(c->x64.p);
  (void)hipFree(c->part.p);
  (void)hipFree(c->part_nf.p);
  (void)hipFree(c->stat_part.p);
  (void)hipFree(c->sums.p);
  (void)hipFree(c->hin.p);
  (void)hipFree(c->hdev.p);
  (void)hipFree(c->c64.p);
  (void)hipFree(c->c32.p);
  (void)hipFree(c->g.p);
  (void)hipFree(c->gs.p);
  for (Plan& p : c->plans) (void)hipFree(p.d_items);
  (void)hipFree(c->d_st);
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
  if ((s = prepare_column(c, x, false, 2))) return s;
  if ((s = read_state(c))) return s;
  if ((s = sync_and_check(c))) return s;
  if ((s = map_status(c, c->h_st->status))) return s;
  *h_out = c->h_st->h_rot;
  return KDE_OK;
}

kde_status kde_bw_plugin(kde_ctx* c, kde_column x, int stages, double* h_out, kde_plugin_info* info) {
  if (!c || !h_out) return KDE_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  if ((s = run_plugin(c, x, stages))) return s;
  if ((s = read_state(c))) return s;
  if ((s = sync_and_check(c))) return s;
  const DevState& h = *c->h_st;
  if (info) {
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
  if ((s = map_status(c, h.status))) return s;
  *h_out = h.h_plugin;
  return KDE_OK;
}

kde_status kde_lscv_curve(kde_ctx* c, kde_column x, const double* h_grid, int32_t n_h, double* g_out,
                          double* gscale_out, double* grid_out) {
  if (!c || !g_out) return KDE_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  if (!h_grid && n_h <= 0) n_h = 150;
  if ((s = run_lscv(c, x, h_grid, n_h))) return s;
  if ((s = ensure_host_out(c, (size_t)3 * n_h))) return s;
  HIP_TRY(c, hipMemcpyAsync(c->h_out, c->g.p, sizeof(double) * n_h, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->h_out + n_h, c->gs.p, sizeof(double) * n_h, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->h_out + 2 * (size_t)n_h, c->hdev.p, sizeof(double) * n_h, hipMemcpyDeviceToHost,
                            c->stream));
  if ((s = read_state(c))) return s;
  if ((s = sync_and_check(c))) return s;
  if ((s = map_status(c, c->h_st->status))) return s;
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
  if ((s = run_lscv(c, x, h_grid, n_h))) return s;
  if ((s = ensure_host_out(c, (size_t)2 * n_h))) return s;
  HIP_TRY(c, hipMemcpyAsync(c->h_out, c->sums.p, sizeof(double) * 2 * n_h, hipMemcpyDeviceToHost, c->stream));
  if ((s = read_state(c))) return s;
  if ((s = sync_and_check(c))) return s;
  if ((s = map_status(c, c->h_st->status))) return s;
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
  Plan* p = nullptr;
  if ((s = run_lscv(c, x, h_grid, n_h, &p))) return s;
  const int32_t n_items = (int32_t)p->items.size();
  std::vector<int32_t> idx((size_t)n_sel);
  for (int32_t k = 0; k < n_sel; ++k) {
    idx[k] = sel[k] < 0 ? n_items + sel[k] : sel[k];
    if (idx[k] < 0 || idx[k] >= n_items) {
      (void)hipStreamSynchronize(c->stream);
      return fail(c, KDE_E_INVAL, "item index out of range");
    }
  }
  if ((s = ensure_host_out(c, (size_t)2 * n_h * (n_sel > 0 ? n_sel : 1)))) return s;
  // part is laid out [2*n_h][n_items]: one strided column per selected item
  for (int32_t k = 0; k < n_sel; ++k)
    HIP_TRY(c, hipMemcpy2DAsync(c->h_out + (size_t)k * 2 * n_h, sizeof(double), c->part.p + idx[k],
                                sizeof(double) * (size_t)n_items, sizeof(double), (size_t)2 * n_h,
                                hipMemcpyDeviceToHost, c->stream));
  if ((s = read_state(c))) return s;
  if ((s = sync_and_check(c))) return s;
  if ((s = map_status(c, c->h_st->status))) return s;
  *n_items_out = n_items;
  for (int32_t k = 0; k < n_sel; ++k) {
    const Item& it = p->items[idx[k]];
    ranges_out[3 * k] = it.row * kde::kBI;
    ranges_out[3 * k + 1] = it.j_begin;
    ranges_out[3 * k + 2] = it.j_end;
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
  if ((s = run_lscv(c, x, h_grid, n_h))) return s;
  if ((s = read_state(c))) return s;
  if ((s = sync_and_check(c))) return s;
  if ((s = map_status(c, c->h_st->status))) return s;
  *h_out = c->h_st->h_best;
  if (k_out) *k_out = c->h_st->k_best;
  if (at_edge) *at_edge = c->h_st->at_edge;
  return KDE_OK;
}

}  // extern "C"
