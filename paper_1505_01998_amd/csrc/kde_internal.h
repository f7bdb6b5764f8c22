// kde_internal.h -- types shared by the kernels and the host runtime of the
// bandwidth-selection library.  Not part of the public ABI (see kde_bw.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kde {

// Threads per block of every pair kernel: four 64-wide waves.  Each block
// owns one "row" of kBI consecutive samples i (one per lane).
constexpr int kThreads = 256;
constexpr int kBI = kThreads;
// j-tile staged in LDS per step; item j-ranges are whole multiples of it.
constexpr int kBJ = 512;
// Every column is padded with +inf up to at least n + kPad so that every
// tile read stays in bounds and padded j contribute exactly zero.
constexpr int kPad = kBJ + kBI;
// Blocks per column of the moment passes (a column of n samples uses
// min(kStatBlocks, ceil(n / 2048)) of them).
constexpr int kStatBlocks = 1024;

// Status values written by device code (same numbers as kde_status).
constexpr int kStOk = 0;
constexpr int kStInval = 1;
constexpr int kStDegenerate = 2;

// Grid kinds of an LSCV request (match kde_grid_kind in kde_bw.h).
constexpr int kGridExplicit = 0;
constexpr int kGridPaper = 1;    // linear over sigma * [h0/4, 4 h0]
constexpr int kGridLogRot = 2;   // log-spaced over h_rot * [lo, hi]

// e^x in FP64 for the pair loops (arguments <= 0: x = -D^2 c), by Cody and
// Waite's argument reduction: k = nearest integer to x / ln 2, r = x - k ln 2
// with ln 2 split into a head of 29 significant bits (k * head is exact for
// |k| < 2^24, so x - k * head is exact) and a tail, |r| <= ln(2) / 2; then
// the Taylor series of e^r to degree 13 (truncation below 5e-18 relative)
// and the scaling by 2^k.  About 2 ulp.  Arguments below -1100 (and -inf)
// are raised to -1100, which underflows to exactly 0; no NaN arrives here
// (samples are finite, and masked pairs carry -inf).
__device__ __forceinline__ double exp_cw(double x) {
  constexpr double kInvLn2 = 1.4426950408889634;
  constexpr double kLn2Head = 0x1.62e42ffp-1;         // ln 2 rounded to 29 bits
  constexpr double kLn2Tail = -4.2009150726810846e-11;  // ln 2 - head
  x = fmax(x, -1100.0);
  const double k = rint(x * kInvLn2);
  double r = __builtin_fma(-k, kLn2Head, x);
  r = __builtin_fma(-k, kLn2Tail, r);
  // 1 / j! for j = 13 .. 0
  double p = 1.6059043836821613e-10;
  p = __builtin_fma(p, r, 2.08767569878681e-09);
  p = __builtin_fma(p, r, 2.505210838544172e-08);
  p = __builtin_fma(p, r, 2.755731922398589e-07);
  p = __builtin_fma(p, r, 2.7557319223985893e-06);
  p = __builtin_fma(p, r, 2.48015873015873e-05);
  p = __builtin_fma(p, r, 1.984126984126984e-04);
  p = __builtin_fma(p, r, 1.388888888888889e-03);
  p = __builtin_fma(p, r, 8.333333333333333e-03);
  p = __builtin_fma(p, r, 4.1666666666666664e-02);
  p = __builtin_fma(p, r, 0.16666666666666666);
  p = __builtin_fma(p, r, 0.5);
  p = __builtin_fma(p, r, 1.0);
  p = __builtin_fma(p, r, 1.0);
  return ldexp(p, (int)k);
}

// Device-resident state of one column of a job.  All scalar steps of the
// method run on the device and read/write this struct, so a whole job is a
// chain of kernels on one stream with one copy back at the end.
struct DevState {
  int status;       // column status (invalid sample, zero spread)
  int pstatus;      // plug-in status (a pilot or final radicand not positive)
  int active;       // the current plug-in stage applies to this column
  int need_f64;     // mixed precision: current plug-in stage is re-run in FP64
  int k_best;
  int at_edge;
  int prec_used[3];
  int stages;       // plug-in stages (2 or 3); 0 when the column has no plug-in
  int pad0;
  double n;
  double shift;     // subtracted from float64 samples before rounding to float32
  double mean, var, sigma, h_rot;
  double g[3], psi[3], kappa[3];
  double h_plugin;
  double h_best, margin;
  double fp64_kappa;  // kappa threshold for the FP64 re-run (0 = never)
  float psi_scale;  // FP32 1/g of the current psi pass (the scaled copy is x32 * psi_scale)
  int psi_fast;     // the scaled copy's range keeps every Hermite value finite (no clamp needed)
  double cd[2];     // FP64 pair coefficients: 1/g^2, -1/(2 g^2)
  float xmin, xmax; // range of the FP32 working copy
  double pruned_evals;  // LSCV pair-term evaluations skipped by tile pruning (exact count)
};

// One column of a job: where its data, coefficients, partial sums and state
// live (absolute device addresses, so resident columns of a server and the
// packed columns of a batch are described the same way).
struct ColDesc {
  const void* raw;      // input samples, float32 or float64
  float* x32;           // padded FP32 working copy [n + kPad]
  float* y32;           // psi pass: the working copy times 1/g of the current stage [n + kPad] (may be null)
  double* x64;          // padded FP64 working copy [n + kPad] (may be null)
  double* stat;         // moment partials [kStatBlocks]
  float* stat_mm;       // minimum and maximum partials of the FP32 working copy [2][kStatBlocks]
  int* stat_nf;         // non-finite counts [kStatBlocks]
  double* psi_part;     // psi partials [2][n_items_psi]
  double* psi_sums;     // [2]
  const double* h_in;   // explicit grid [n_h]
  double* h;            // grid used [n_chunks * HC]
  float* c32;           // FP32 exponent coefficients [n_chunks * HC]
  double* c64;          // FP64 exponent coefficients [n_chunks * HC]
  double* part;         // LSCV partials [2 n_h][n_items], row = 2 h + {0, 1}
  double* sums;         // LSCV pair sums [2 n_h]
  double* g;            // g(h) [n_h]
  double* gs;           // gscale(h) [n_h]
  double* near_sums;    // tile pruning: pair sums of each row's first j-tile [2 n_h] (lower bounds)
  float* d2cut;         // tile pruning: squared distance beyond which a tile is skipped, per chunk
  DevState* st;
  int n;
  int raw_f64;
  int n_h;              // LSCV grid points (0: no LSCV for this column)
  int n_chunks;         // ceil(n_h / HC)
  int n_items;          // LSCV work items
  int n_items_psi;      // psi work items
  int grid_kind;        // kGridExplicit / kGridPaper / kGridLogRot
  int pad0;
  double grid_lo, grid_hi;
};

// One block of a pair kernel: the samples i in [row*kBI, row*kBI + kBI) of
// column `col` against j in [j_begin, j_end) (a multiple of kBJ long; a
// column's last item may run past n into the +inf padding).  `item` is the
// item's index within its column, `chunk` the bandwidth chunk (LSCV).
struct Unit {
  int col, row, j_begin, j_end, item, chunk;
};

// One row of a segmented reduction: *dst = sum of src[0 .. n).
struct RowDesc {
  const double* src;
  double* dst;
  int n;
  int pad0;
};

// ---- launchers (kde_kernels.hip); all asynchronous on `s` ----
// Column-level launches act on the columns cols[ids[0 .. n_ids)].
void launch_stats(hipStream_t s, const ColDesc* cols, const int* ids, int n_ids, int max_blocks);
// Pilot bandwidth of the stage and, for the mixed form, the scaled copy
// y32 = x32 / g of every active column.
void launch_psi_begin(hipStream_t s, const ColDesc* cols, const int* ids, int n_ids, int stage, int f64);
void launch_psi_finish(hipStream_t s, const ColDesc* cols, const int* ids, int n_ids, int stage, int was_f64,
                       int conditional);
void launch_plugin_final(hipStream_t s, const ColDesc* cols, const int* ids, int n_ids);
void launch_lscv_prep(hipStream_t s, const ColDesc* cols, const int* ids, int n_ids, int hc);
void launch_lscv_finalize(hipStream_t s, const ColDesc* cols, const int* ids, int n_ids, int f64);
// Pair kernels act on units[u0 .. u0 + n_units).
void launch_psi_units(hipStream_t s, int r, int f64, int conditional, const ColDesc* cols, const Unit* units, int u0,
                      int n_units);
// mfma: use the matrix-core variant (FP32, 16 bandwidths per unit only).
// Tile pruning: per column, the cut distance of every bandwidth chunk from
// the near-tile sums (relative bound eps on every skipped share).
void launch_lscv_prune_prep(hipStream_t s, const ColDesc* cols, const int* ids, int n_ids, int hc, double eps);
// The sweep's inner loop over one LDS tile (x: kBJ samples, c32: hc
// coefficients), reps times per block; out: blocks x 4 doubles.
void launch_lscv_ceiling(hipStream_t s, int hc, const float* x, const float* c32, int reps, double* out, int blocks);
void launch_lscv_units(hipStream_t s, int hc, int f64, int mfma, int prune, const ColDesc* cols, const Unit* units,
                       int u0, int n_units);
void launch_reduce_rows(hipStream_t s, const RowDesc* rows, int n_rows);
// Persistent form of the dense FP32 LSCV sweep: `blocks` blocks take the
// n_units units from kQueueGroups groups, group g being units
// [group_begin[g], group_begin[g + 1]) (device array of kQueueGroups + 1
// ints, group_begin[kQueueGroups] = n_units) with device counter next[g]
// (kQueueGroups ints, all 0 at launch: clear them with launch_zero_ints in
// the same stream).  Variants (hc bandwidths per block, tj samples per LDS
// tile): (8, 512), (16, 256), (16, 512), (16, 1024), (32, 512);
// lscv_queue_variant says whether one exists.  lscv_queue_blocks: the blocks
// the current device holds at once for a variant (0 on failure).
constexpr int kQueueGroups = 8;
void launch_zero_ints(hipStream_t s, int* p, int n);
bool lscv_queue_variant(int hc, int tj);
int lscv_queue_blocks(int hc, int tj);
void launch_lscv_units_queue(hipStream_t s, int hc, int tj, const ColDesc* cols, const Unit* units, int n_units,
                             const int* group_begin, int* next, int blocks);

// ---- ascending sort of FP32 keys (kde_sort.hip): temporary bytes for
// `count` keys (0 on failure), and the sort itself.
size_t sort_temp_bytes(int count);
hipError_t sort_keys(void* tmp, size_t tmp_bytes, const float* in, float* out, int count, hipStream_t s);

}  // namespace kde
