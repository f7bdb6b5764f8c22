// kde_md.h -- shared pieces of the d-dimensional paths (LSCV_h, LSCV_H and
// the estimate's consumers): the device state of a sample matrix, FP64
// reduction helpers, and the host launchers of the moment, factor and
// whitening kernels that all three use.
#ifndef KDE_MD_H
#define KDE_MD_H

#include <hip/hip_runtime.h>

#include "kde_runtime.h"

namespace kde {

constexpr int kMdBlocks = 256;  // blocks of the moment passes
constexpr int kMdRun = 64;
constexpr double kPiD = 3.14159265358979323846;
constexpr double kLog2ED = 1.4426950408889634074;

struct MdState {
  int status;
  int d;
  int n;
  int k_best;
  int at_edge;
  int pad0;
  double logdet;
  double h0;
  double h_best;
  double margin;
  double mean[KDE_MAX_D];
  double linv[KDE_MAX_D * KDE_MAX_D];   // L^-1, row-major d x d (stride KDE_MAX_D)
  double sigma[KDE_MAX_D * KDE_MAX_D];  // Sigma, same layout
};

__device__ inline double md_raw(const void* raw, int f64, int64_t idx) {
  return f64 ? reinterpret_cast<const double*>(raw)[idx] : (double)reinterpret_cast<const float*>(raw)[idx];
}

__device__ inline double md_block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ inline double md_wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ inline void md_fold(float& acc, float& comp, float r) {
  const float y = r - comp;
  const float t = acc + y;
  comp = (t - acc) - y;
  acc = t;
}


inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// coordinates per sample as compiled (d rounded up to 2, 3, 4, 8 or 16;
// unused coordinates are 0)
int md_width(int d);
// sums, mean and non-finite count of the samples (raw row-major n x d)
void md_moments(hipStream_t st, const void* raw, bool raw_f64, int n, int d, int nblk, double* ps, int* nf,
                MdState* dst);
// Y[a][i] = sum_b M[a][b] (x_ib - mean_b) for a < D, dimension-major with
// npad samples a dimension (padding: +inf in coordinate 0); M lower
// triangular with row stride KDE_MAX_D; y32 or y64 may be null
void md_whiten(hipStream_t st, const void* raw, bool raw_f64, int n, int D, int npad, const MdState* dst,
               const double* M, float* y32, double* y64);
// moments, covariance, Cholesky factor of Sigma and the sphered samples
void md_stage(hipStream_t st, const void* raw, bool raw_f64, int n, int d, int D, int npad, int nblk, double* ps,
              int* nf, double* pc, MdState* dst, float* y32, double* y64);

}  // namespace kde

#endif  // KDE_MD_H
