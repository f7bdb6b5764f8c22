// kde_tune.hip -- tile autotuner for the LSCV pair pass.
//
// The dense LSCV pass (Section 4.4.2, every grid h of eq. LSCV-gh from one
// pair distance, Section 4.5) runs as one persistent launch, in one of five
// variants (kQueueHC x kQueueTJ): 8, 16 or 32 bandwidths per block with
// 512-sample LDS tiles, and 16 bandwidths with 256- or 1024-sample tiles.
// The bandwidths per block trade register pressure (waves per SIMD) against
// how far the pair distance is amortised and how much of a padded last chunk
// is wasted; the tile size trades staging and barrier frequency against LDS.
// Work items are sized independently of the variant and every (item, h) sum
// is accumulated in the same order by all of them, so the variant changes
// the speed and never a result.  (The matrix-core form folds shorter runs,
// so its sums differ in rounding; it stays an explicit option and is not a
// candidate.)
//
// The tuner measures each variant's steady-state rate on the persistent
// kernel itself: launches over B and 2B units of a trial column are timed and
// the difference is divided into the extra work, which cancels launch
// overhead and the drain at the end of a launch.  The trial units are the
// rows of a column of L samples (L as long as the column, capped at 8192)
// against the rest of the row, cycled; the samples are spread evenly and the
// grid's exponentials cover the range of a real one (the part draws less
// power on an all-zero column and then runs a few per cent faster).  Before
// a variant may be chosen it must pass a parity gate: its partial sums of
// every trial unit for the first 8 bandwidths must be bitwise those of the
// default variant (16, 512), the property the decomposition guarantees.  The
// rate is scaled by the share of the variant's bandwidth slots that the grid
// fills (a 100-point grid fills 100 of 104 slots at 8 per block, 112 at 16,
// 128 at 32).  Each variant is timed twice (two rounds, the second in reverse
// order) and keeps its better rate; the default is replaced only by a
// variant 3% faster, since single trials vary by a few per cent with the
// part's clock while on real columns the three tile sizes run within 0.2%
// of each other.  Decisions are cached per context by shape (quarter octave
// of n, grid size).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "kde_runtime.h"

namespace kde {

namespace {

constexpr int kTrialUnits = 4096;          // B: about 4096 and 8192 units per variant
constexpr int kTrialMaxJ = 8192;            // trial column length (samples)
constexpr double kTuneMinJobEvals = 1e13;  // jobs smaller than this use the cached or default variant
constexpr double kSwitchGain = 1.03;       // a variant replaces the default only when this much faster
constexpr int kGateH = 8;                  // bandwidths every variant's parity gate compares

std::pair<int, int> shape_key(int64_t n, int n_h) {
  return {(int)std::floor(4.0 * std::log2((double)std::max<int64_t>(n, 2))), n_h};
}

// Pairs i < j of the trial unit for row r of an L-sample column, j in [r*kBI, L).
double trial_pairs(int L, int r) {
  const double i0 = (double)r * kBI, len = (double)L - i0;
  return (double)kBI * len - 0.5 * (double)kBI * ((double)kBI + 1.0);
}

}  // namespace

kde_status tune_shape(kde_ctx* c, int64_t n, int n_h, TuneChoice& out) {
  if (n < 2 || n > KDE_MAX_N || n_h < 1 || n_h > KDE_MAX_NH) return fail(c, KDE_E_INVAL, "bad tuning shape");
  const auto key = shape_key(n, n_h);
  auto hit = c->tune_cache.find(key);
  if (hit != c->tune_cache.end()) {
    out = hit->second;
    return KDE_OK;
  }
  // trial column: L samples (+ padding), R rows; unit k is row k % R against
  // j in [row * kBI, L), so B and 2B units are whole copies of the row cycle
  const int L = (int)std::min<int64_t>(((n + kBJ - 1) / kBJ) * kBJ, kTrialMaxJ);
  const int R = L / kBI;
  const int B = std::max(1, kTrialUnits / R) * R;
  const int B2 = 2 * B;
  const size_t xn = (size_t)L + kPad;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t o = at;
    at += (bytes + 255) / 256 * 256;
    return o;
  };
  const size_t o_x = take(4 * xn), o_c = take(4 * 32), o_part = take(16 * 32 * (size_t)B2),
               o_st = take(sizeof(DevState)), o_col = take(sizeof(ColDesc)), o_units = take(sizeof(Unit) * B2),
               o_ctr = take(sizeof(int) * kQueueGroups), o_gb = take(sizeof(int) * 2 * (kQueueGroups + 1));
  kde_status s;
  if ((s = ensure(c, c->tune_buf, at))) return s;
  char* b = c->tune_buf.p;
  // zero state (status OK); samples spread evenly over [0, 4) with +inf
  // padding and coefficients of 32 bandwidths log-spaced over [0.01, 1]
  KDE_HIP_TRY(c, hipMemsetAsync(b, 0, o_units, c->stream));
  std::vector<Unit> u(B2);
  double extra_pairs = 0.0;  // pairs of the extra B units of the 2B launch
  for (int k = 0; k < B2; ++k) {
    const int r = k % R;
    u[k] = Unit{0, r, r * kBI, L, k, 0};
    if (k >= B) extra_pairs += trial_pairs(L, r);
  }
  {
    std::vector<float> hx(xn), hcf(32);
    for (size_t j = 0; j < xn; ++j) hx[j] = j < (size_t)L ? 4.0f * (float)j / (float)L : HUGE_VALF;
    for (int k = 0; k < 32; ++k) {
      const double h = std::exp(std::log(0.01) + std::log(100.0) * k / 31.0);
      hcf[k] = (float)(-1.4426950408889634 / (4.0 * h * h));
    }
    KDE_HIP_TRY(c, hipMemcpyAsync(b + o_x, hx.data(), 4 * xn, hipMemcpyHostToDevice, c->stream));
    KDE_HIP_TRY(c, hipMemcpyAsync(b + o_c, hcf.data(), 4 * 32, hipMemcpyHostToDevice, c->stream));
    KDE_HIP_TRY(c, hipMemcpyAsync(b + o_units, u.data(), sizeof(Unit) * B2, hipMemcpyHostToDevice, c->stream));
    // one group holding all units: first for the B launches, then for 2B
    std::vector<int> gb(2 * (kQueueGroups + 1));
    for (int q = 0; q <= kQueueGroups; ++q) {
      gb[q] = q == 0 ? 0 : B;
      gb[kQueueGroups + 1 + q] = q == 0 ? 0 : B2;
    }
    KDE_HIP_TRY(c, hipMemcpyAsync(b + o_gb, gb.data(), sizeof(int) * gb.size(), hipMemcpyHostToDevice, c->stream));
    KDE_HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  const ColDesc* cols = (const ColDesc*)(b + o_col);
  const Unit* dev_units = (const Unit*)(b + o_units);
  int* ctr = (int*)(b + o_ctr);
  const int* groups_B = (const int*)(b + o_gb);
  const int* groups_B2 = groups_B + kQueueGroups + 1;
  hipEvent_t ev[3];
  int made = 0;
  hipError_t he = hipSuccess;
  for (; made < 3 && he == hipSuccess; ++made) he = hipEventCreate(&ev[made]);
  if (he != hipSuccess) --made;
  TuneChoice r;
  for (int v = 0; v < kQueueVariants; ++v) {
    r.rate[v] = 0.0;
    r.parity[v] = false;
  }
  std::vector<double> ref, got((size_t)2 * kGateH * B2);
  // Two rounds over the variants, the second in reverse order, each variant
  // keeping its better rate: single trials vary by a few per cent with the
  // part's clock, more than the variants differ.  The default runs first:
  // its partial sums are the gate's reference.
  int order[2 * kQueueVariants];
  order[0] = kQueueDefault;
  for (int v = 0, k = 1; v < kQueueVariants; ++v)
    if (v != kQueueDefault) order[k++] = v;
  for (int q = 0; q < kQueueVariants; ++q) order[kQueueVariants + q] = order[kQueueVariants - 1 - q];
  for (int q = 0; q < 2 * kQueueVariants && he == hipSuccess; ++q) {
    const int v = order[q];
    const int hc = kQueueHC[v], tj = kQueueTJ[v];
    const int blocks = queue_blocks(c, hc, tj);
    if (blocks <= 0) continue;
    ColDesc d;
    std::memset(&d, 0, sizeof(d));
    d.x32 = (float*)(b + o_x);
    d.c32 = (float*)(b + o_c);
    d.part = (double*)(b + o_part);
    d.st = (DevState*)(b + o_st);
    d.n = L;
    d.n_h = hc;
    d.n_items = B2;
    // synchronous, as `d` is reused for the next variant
    he = hipMemcpyAsync(b + o_col, &d, sizeof(d), hipMemcpyHostToDevice, c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    // warm-up, then B units and 2B units back to back (the 2B launch writes
    // every unit's partial slots, which the gate reads)
    if (he == hipSuccess) {
      launch_zero_ints(c->stream, ctr, kQueueGroups);
      launch_lscv_units_queue(c->stream, hc, tj, cols, dev_units, B, groups_B, ctr, blocks);
      launch_zero_ints(c->stream, ctr, kQueueGroups);
      he = hipEventRecord(ev[0], c->stream);
    }
    if (he == hipSuccess) {
      launch_lscv_units_queue(c->stream, hc, tj, cols, dev_units, B, groups_B, ctr, blocks);
      launch_zero_ints(c->stream, ctr, kQueueGroups);
      he = hipEventRecord(ev[1], c->stream);
    }
    if (he == hipSuccess) {
      launch_lscv_units_queue(c->stream, hc, tj, cols, dev_units, B2, groups_B2, ctr, blocks);
      he = hipEventRecord(ev[2], c->stream);
    }
    if (he == hipSuccess) he = hipGetLastError();
    if (he == hipSuccess) he = hipEventSynchronize(ev[2]);
    float t1 = 0.f, t2 = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&t1, ev[0], ev[1]);
    if (he == hipSuccess) he = hipEventElapsedTime(&t2, ev[1], ev[2]);
    if (he == hipSuccess)
      he = hipMemcpy(got.data(), b + o_part, sizeof(double) * got.size(), hipMemcpyDeviceToHost);
    if (he != hipSuccess) break;
    if (q == 0) ref = got;
    const bool same = std::memcmp(got.data(), ref.data(), sizeof(double) * got.size()) == 0;
    r.parity[v] = q < kQueueVariants ? same : (r.parity[v] && same);
    const double fill = (double)n_h / (double)(((n_h + hc - 1) / hc) * hc);
    r.rate[v] = std::max(r.rate[v], (t2 > t1) ? extra_pairs * hc / ((t2 - t1) * 1e-3) * fill : 0.0);
  }
  for (int k = 0; k < made; ++k) (void)hipEventDestroy(ev[k]);
  if (he != hipSuccess) return fail(c, KDE_E_DEVICE, std::string("autotune trial: ") + hipGetErrorString(he));
  int best = kQueueDefault;
  for (int v = 0; v < kQueueVariants; ++v)
    if (r.parity[v] && r.rate[v] > r.rate[best] * kSwitchGain) best = v;
  r.hc = kQueueHC[best];
  r.tj = kQueueTJ[best];
  c->tune_cache[key] = r;
  out = r;
  return KDE_OK;
}

kde_status select_variant(kde_ctx* c, const kde_request* reqs, int32_t n_req) {
  c->job_hc = c->opt_hc;
  c->job_tj = c->opt_tj;
  c->job_mfma = c->opt_mfma;
  if (!c->opt_autotune || c->prec == KDE_PREC_FP64) return KDE_OK;
  // the job's largest LSCV column decides; malformed requests are skipped
  // here and rejected by the planner
  int64_t n_best = 0;
  int nh_best = 0;
  double w_best = 0.0, total = 0.0;
  for (int32_t k = 0; k < n_req; ++k) {
    const kde_request& r = reqs[k];
    if (!(r.methods & KDE_METHOD_LSCV) || r.x.n < 2 || r.x.n > KDE_MAX_N || r.grid.n_h < 1 ||
        r.grid.n_h > KDE_MAX_NH)
      continue;
    const double w = 0.5 * (double)r.x.n * (double)(r.x.n - 1) * r.grid.n_h;
    total += w;
    if (w > w_best) {
      w_best = w;
      n_best = r.x.n;
      nh_best = r.grid.n_h;
    }
  }
  if (n_best == 0) return KDE_OK;
  auto hit = c->tune_cache.find(shape_key(n_best, nh_best));
  TuneChoice t;
  if (hit != c->tune_cache.end()) {
    t = hit->second;
  } else if (total >= kTuneMinJobEvals) {
    kde_status s = tune_shape(c, n_best, nh_best, t);
    if (s) return s;
  } else {
    return KDE_OK;
  }
  c->job_hc = t.hc;
  c->job_tj = t.tj;
  c->job_mfma = 0;
  return KDE_OK;
}

}  // namespace kde

extern "C" kde_status kde_autotune(kde_ctx* c, int64_t n, int32_t n_h, kde_tune_info* out) {
  if (!c) return KDE_E_INVAL;
  if (c->server && kde::server_running(c->server.get()))
    return kde::fail(c, KDE_E_BUSY, "a server is running on this context");
  if (c->prec == KDE_PREC_FP64) return kde::fail(c, KDE_E_INVAL, "the autotuner covers the mixed-precision form");
  if (hipSetDevice(c->device) != hipSuccess) return kde::fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde::TuneChoice t;
  kde_status s = kde::tune_shape(c, n, n_h, t);
  if (s) return s;
  if (out) {
    out->hc = t.hc;
    out->tj = t.tj;
    for (int v = 0; v < kde::kQueueVariants; ++v) {
      out->evals_per_s[v] = t.rate[v];
      out->parity[v] = t.parity[v] ? 1 : 0;
    }
  }
  return KDE_OK;
}

// The sweep's inner loop from one LDS tile (no staging, barriers, masks or
// partial sums): samples spread over [0, 4), coefficients of h log-spaced over
// [0.01, 1], so the exponentials cover the same range as a real grid.  A
// warm-up launch, then launches of kCeilReps and 2 kCeilReps repetitions
// timed by events; the rate is that of the extra kCeilReps repetitions (the
// difference of the two), so the launches' start and drain cancel, as in
// the tile tuner's trials.
extern "C" kde_status kde_lscv_ceiling(kde_ctx* c, int32_t hc, double* evals_per_s) {
  constexpr int kCeilBlocks = 8192, kCeilReps = 64;
  if (!c || !evals_per_s) return KDE_E_INVAL;
  if (hc != 8 && hc != 16 && hc != 32) return kde::fail(c, KDE_E_INVAL, "hc must be 8, 16 or 32");
  if (c->server && kde::server_running(c->server.get()))
    return kde::fail(c, KDE_E_BUSY, "a server is running on this context");
  if (hipSetDevice(c->device) != hipSuccess) return kde::fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  std::vector<float> hx(kde::kBJ), hcf(32);
  for (int j = 0; j < kde::kBJ; ++j) hx[j] = 4.0f * (float)j / (float)kde::kBJ;
  for (int k = 0; k < 32; ++k) {
    const double h = std::exp(std::log(0.01) + std::log(100.0) * k / 31.0);
    hcf[k] = (float)(-1.4426950408889634 / (4.0 * h * h));
  }
  const size_t o_x = 0, o_c = 4 * (size_t)kde::kBJ, o_out = o_c + 4 * 32;
  const size_t bytes = o_out + sizeof(double) * 4 * (size_t)kCeilBlocks;
  kde_status s;
  if ((s = kde::ensure(c, c->tune_buf, bytes))) return s;
  char* b = c->tune_buf.p;
  KDE_HIP_TRY(c, hipMemcpyAsync(b + o_x, hx.data(), 4 * hx.size(), hipMemcpyHostToDevice, c->stream));
  KDE_HIP_TRY(c, hipMemcpyAsync(b + o_c, hcf.data(), 4 * hcf.size(), hipMemcpyHostToDevice, c->stream));
  const float* x = (const float*)(b + o_x);
  const float* cf = (const float*)(b + o_c);
  double* out = (double*)(b + o_out);
  hipEvent_t ev[3];
  int made = 0;
  hipError_t he = hipSuccess;
  for (; made < 3 && he == hipSuccess; ++made) he = hipEventCreate(&ev[made]);
  if (he != hipSuccess) --made;
  float ms1 = 0.f, ms2 = 0.f;
  if (he == hipSuccess) {
    kde::launch_lscv_ceiling(c->stream, hc, x, cf, 1, out, kCeilBlocks);
    he = hipEventRecord(ev[0], c->stream);
  }
  if (he == hipSuccess) {
    kde::launch_lscv_ceiling(c->stream, hc, x, cf, kCeilReps, out, kCeilBlocks);
    he = hipEventRecord(ev[1], c->stream);
  }
  if (he == hipSuccess) {
    kde::launch_lscv_ceiling(c->stream, hc, x, cf, 2 * kCeilReps, out, kCeilBlocks);
    he = hipEventRecord(ev[2], c->stream);
  }
  if (he == hipSuccess) he = hipGetLastError();
  if (he == hipSuccess) he = hipEventSynchronize(ev[2]);
  if (he == hipSuccess) he = hipEventElapsedTime(&ms1, ev[0], ev[1]);
  if (he == hipSuccess) he = hipEventElapsedTime(&ms2, ev[1], ev[2]);
  for (int k = 0; k < made; ++k) (void)hipEventDestroy(ev[k]);
  if (he != hipSuccess) return kde::fail(c, KDE_E_DEVICE, std::string("ceiling trial: ") + hipGetErrorString(he));
  const double evals = (double)kCeilBlocks * kde::kThreads * kCeilReps * kde::kBJ * hc;
  // the extra kCeilReps repetitions of the second launch; the single launch
  // as a fallback should the difference not be positive
  const double dt = ms2 > ms1 ? (double)(ms2 - ms1) : (double)ms1;
  *evals_per_s = dt > 0.0 ? evals / (dt * 1e-3) : 0.0;
  return KDE_OK;
}
