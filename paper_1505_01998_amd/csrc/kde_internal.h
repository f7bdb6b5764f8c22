// kde_internal.h -- types shared by the kernels and the host runtime of the
// bandwidth-selection library.  Not part of the public ABI (see kde_bw.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kde {

// Threads per block of every pair kernel: four 64-wide waves.  Each block
// owns one "row" of BI consecutive samples i (one per lane).
constexpr int kThreads = 256;
constexpr int kBI = kThreads;
// j-tile staged in LDS per step; item j-ranges are whole multiples of it.
constexpr int kBJ = 512;
// Samples are padded with +inf up to at least n + kPad so that every tile
// read stays in bounds and padded j contribute exactly zero.
constexpr int kPad = kBJ + kBI;

// Status values written by device code (same numbers as kde_status).
constexpr int kStOk = 0;
constexpr int kStInval = 1;
constexpr int kStDegenerate = 2;

// Device-resident state of one selector call.  All scalar steps of the
// method run on the device and read/write this struct, so a whole call is a
// chain of kernels on one stream with a single copy back at the end.
struct DevState {
  int status;
  int need_f64;     // mixed precision: current plug-in stage is re-run in FP64
  int k_best;
  int at_edge;
  int prec_used[3];
  int stages;
  double n;
  double shift;     // subtracted from float64 samples before rounding to float32
  double mean, var, sigma, h_rot;
  double g[3], psi[3], kappa[3];
  double h_plugin;
  double h_best, margin;
  double fp64_kappa;  // kappa threshold for the FP64 re-run (0 = never)
  float cf[2];      // FP32 pair coefficients of the current psi pass: 1/g^2, -log2(e)/(2 g^2)
  double cd[2];     // FP64 pair coefficients: 1/g^2, -1/(2 g^2)
};

// One work item of a pair kernel: block row (samples i in [row*kBI, row*kBI+kBI)),
// and the j-range [j_begin, j_end) it sweeps.  j_end - j_begin is a multiple
// of kBJ; the last item of a row may run past n into the +inf padding.
struct Item {
  int row, j_begin, j_end, pad;
};

// ---- launchers (kde_kernels.hip); all asynchronous on `s` ----
void launch_stats_sum(hipStream_t s, const void* x, int is_f64, int n, double* part, int* part_nf, int nblk);
void launch_stats_mean(hipStream_t s, const double* part, const int* part_nf, int nblk, int n, int shift_by_mean,
                       DevState* st);
void launch_stats_dev(hipStream_t s, const void* x, int is_f64, int n, int n_pad, double* part, float* x32,
                      double* x64, int nblk, DevState* st);
void launch_stats_final(hipStream_t s, const double* part, int nblk, DevState* st);

void launch_psi_begin(hipStream_t s, DevState* st, int stage);
void launch_psi_finish(hipStream_t s, DevState* st, int stage, const double* sums, int was_f64, int conditional);
void launch_plugin_final(hipStream_t s, DevState* st);
void launch_psi_pairs(hipStream_t s, int r, int f64, int conditional, const float* x32, const double* x64, int n,
                      const Item* items, int n_items, int bid0, int nblk, double* part, const DevState* st);

void launch_lscv_prep(hipStream_t s, const double* h_in, int n_h, int n_h_pad, DevState* st, double* h_dev,
                      float* c32, double* c64);
void launch_lscv_pairs(hipStream_t s, int hc, int f64, const float* x32, const double* x64, int n,
                       const Item* items, int n_items, int n_chunks, const float* c32, const double* c64, int n_h,
                       int bid0, int nblk, double* part, const DevState* st);
void launch_lscv_finalize(hipStream_t s, const double* sums, int n_h, const double* h_dev, DevState* st,
                          double* g, double* gscale);

void launch_reduce_rows(hipStream_t s, const double* part, int n_cols, int n_rows, double* out);

}  // namespace kde
