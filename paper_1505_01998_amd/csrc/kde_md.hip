// kde_md.hip -- LSCV_h for d-dimensional samples (Section 4.4.2, the sphered
// objective of eq. (LSCV-gh)), d <= 16.
//
// The formula modifications of Section 4.5 write the pair kernels through
// S(v) = v^T Sigma^-1 v, a scalar per pair that does not depend on h.  Here
// S(v) is never stored: the samples are whitened once on the device,
// Y = L^-1 (X - mean) with Sigma = L L^T, so S(X_i - X_j) = |Y_i - Y_j|^2,
// and the pair kernel forms it in registers from the D coordinates of the
// pair and reuses it for a chunk of bandwidths, exactly as the univariate
// kernel reuses the squared difference.  Layout: Y is stored
// dimension-major (D rows of n + padding samples), a block owns a row of 256
// samples i (their D coordinates in registers) and sweeps j-tiles of
// D x 512 coordinates staged in LDS (broadcast reads).  Padding samples hold
// +inf in the first coordinate, so their terms are exactly zero.
//
//   g(h) = h^-d [2 n^-2 (A S1(h) - 2 B S2(h)) + n^-1 A],
//   A = (4 pi)^(-d/2) |Sigma|^(-1/2), B = (2 pi)^(-d/2) |Sigma|^(-1/2),
//   S1(h) = sum_{i<j} exp(-S/(4 h^2)), S2(h) = sum_{i<j} exp(-S/(2 h^2)) = sum e1^2,
// with R(K) = A (eq. LSCV_MULTI-rk with H = Sigma).  Mixed form: FP32 terms in
// compensated 64-term runs, FP64 above the lane; FP64 form: FP64 terms.
// Moments, covariance, Cholesky and whitening are FP64 kernels; Sigma counts
// as singular when a Cholesky pivot is at most 1e-12 of its diagonal entry.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "kde_runtime.h"

namespace kde {

namespace {

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

__device__ __forceinline__ double md_raw(const void* raw, int f64, int64_t idx) {
  return f64 ? reinterpret_cast<const double*>(raw)[idx] : (double)reinterpret_cast<const float*>(raw)[idx];
}

__device__ __forceinline__ double md_block_sum(double v, double* sh) {
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

__device__ __forceinline__ double md_wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ void md_fold(float& acc, float& comp, float r) {
  const float y = r - comp;
  const float t = acc + y;
  comp = (t - acc) - y;
  acc = t;
}

// pass 1: per-block coordinate sums and non-finite counts
__global__ __launch_bounds__(kThreads) void k_md_sum(const void* raw, int f64, int n, int d, int nblk,
                                                     double* part, int* nf) {
  __shared__ double sh[kThreads];
  const int chunk = (n + nblk - 1) / nblk;
  const int b0 = blockIdx.x * chunk, b1 = min(n, b0 + chunk);
  int bad = 0;
  for (int a = 0; a < d; ++a) {
    double s = 0.0;
    for (int i = b0 + threadIdx.x; i < b1; i += kThreads) {
      const double v = md_raw(raw, f64, (int64_t)i * d + a);
      if (!isfinite(v)) ++bad;
      s += isfinite(v) ? v : 0.0;
    }
    s = md_block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x * KDE_MAX_D + a] = s;
  }
  const double nb = md_block_sum((double)bad, sh);
  if (threadIdx.x == 0) nf[blockIdx.x] = (int)nb;
}

__global__ void k_md_mean(const double* part, const int* nf, int nblk, int n, int d, MdState* st) {
  if (threadIdx.x != 0) return;
  st->d = d;
  st->n = n;
  int bad = 0;
  for (int b = 0; b < nblk; ++b) bad += nf[b];
  st->status = bad ? kStInval : kStOk;
  for (int a = 0; a < d; ++a) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[b * KDE_MAX_D + a];
    st->mean[a] = s / (double)n;
  }
}

// pass 2: per-block cross products about the mean (lower triangle a >= b)
__global__ __launch_bounds__(kThreads) void k_md_cov(const void* raw, int f64, int n, int d, int nblk,
                                                     const MdState* st, double* part) {
  __shared__ double sh[kThreads];
  if (st->status != kStOk) return;
  const int chunk = (n + nblk - 1) / nblk;
  const int b0 = blockIdx.x * chunk, b1 = min(n, b0 + chunk);
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b) {
      double s = 0.0;
      for (int i = b0 + threadIdx.x; i < b1; i += kThreads)
        s += (md_raw(raw, f64, (int64_t)i * d + a) - st->mean[a]) * (md_raw(raw, f64, (int64_t)i * d + b) - st->mean[b]);
      s = md_block_sum(s, sh);
      if (threadIdx.x == 0) part[blockIdx.x * KDE_MAX_D * KDE_MAX_D + a * KDE_MAX_D + b] = s;
    }
}

// one thread: Sigma, its Cholesky factor, log|Sigma| and L^-1
__global__ void k_md_factor(const double* part, int nblk, MdState* st) {
  if (threadIdx.x != 0 || st->status != kStOk) return;
  const int d = st->d;
  double S[KDE_MAX_D][KDE_MAX_D], L[KDE_MAX_D][KDE_MAX_D];
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b) {
      double s = 0.0;
      for (int k = 0; k < nblk; ++k) s += part[k * KDE_MAX_D * KDE_MAX_D + a * KDE_MAX_D + b];
      S[a][b] = S[b][a] = s / (double)(st->n - 1);
      st->sigma[a * KDE_MAX_D + b] = st->sigma[b * KDE_MAX_D + a] = S[a][b];
    }
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) L[a][b] = 0.0;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b) {
      double s = S[a][b];
      for (int k = 0; k < b; ++k) s -= L[a][k] * L[b][k];
      if (a == b) {
        if (!(s > 1e-12 * S[a][a]) || !isfinite(s)) {
          st->status = kStDegenerate;
          return;
        }
        L[a][a] = sqrt(s);
      } else {
        L[a][b] = s / L[b][b];
      }
    }
  double ld = 0.0;
  for (int a = 0; a < d; ++a) ld += 2.0 * log(L[a][a]);
  st->logdet = ld;
  for (int cidx = 0; cidx < d; ++cidx)
    for (int a = 0; a < d; ++a) {
      double s = (a == cidx) ? 1.0 : 0.0;
      for (int k = 0; k < a; ++k) s -= L[a][k] * st->linv[k * KDE_MAX_D + cidx];
      st->linv[a * KDE_MAX_D + cidx] = s / L[a][a];
    }
  st->h0 = pow(4.0 / ((d + 2.0) * (double)st->n), 1.0 / (d + 4.0));
}

// Y[a][i] = sum_b M[a][b] (x_ib - mean_b), a < D (coordinates a >= d are 0),
// M lower triangular with row stride KDE_MAX_D (L^-1 for the sphered
// samples); padding: +inf in coordinate 0, 0 elsewhere
__global__ __launch_bounds__(kThreads) void k_md_whiten(const void* raw, int f64, int n, int D, int npad,
                                                        const MdState* st, const double* M, float* y32,
                                                        double* y64) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= npad) return;
  const int d = st->d;
  const bool ok = st->status == kStOk;
  double v[KDE_MAX_D];
  for (int a = 0; a < d; ++a) v[a] = (i < n && ok) ? md_raw(raw, f64, (int64_t)i * d + a) - st->mean[a] : 0.0;
  for (int a = 0; a < D; ++a) {
    double w;
    if (i >= n) {
      w = a == 0 ? (double)__builtin_inff() : 0.0;
    } else if (a < d) {
      w = 0.0;
      for (int b = 0; b <= a; ++b) w += M[a * KDE_MAX_D + b] * v[b];
    } else {
      w = 0.0;
    }
    if (y32) y32[(int64_t)a * npad + i] = (float)w;
    if (y64) y64[(int64_t)a * npad + i] = w;
  }
}

// grid (explicit or the default linear grid over [h0/4, 4 h0]) and exponent coefficients
__global__ __launch_bounds__(kThreads) void k_md_prep(const MdState* st, const double* h_in, int n_h, int m,
                                                      double* h, float* c32, double* c64) {
  for (int k = threadIdx.x; k < m; k += kThreads) {
    if (k < n_h) {
      double hv;
      if (h_in) {
        hv = h_in[k];
      } else {
        const double t = n_h == 1 ? 0.0 : (double)k / (double)(n_h - 1);
        hv = st->h0 * 0.25 + (st->h0 * 4.0 - st->h0 * 0.25) * t;
      }
      h[k] = hv;
      const double q = 1.0 / (4.0 * hv * hv);
      c32[k] = (float)(-kLog2ED * q);
      c64[k] = -q;
    } else {
      h[k] = 0.0;
      c32[k] = -1.0f;
      c64[k] = -1.0;
    }
  }
}

template <int D, int HC, bool MASK>
__device__ __forceinline__ void md_run(const float (*tile)[kBJ], int jl, int jg, const float (&yi)[D], int i,
                                       const float (&ck)[HC], float (&a1)[HC], float (&c1)[HC], float (&a2)[HC],
                                       float (&c2)[HC]) {
  float r1[HC], r2[HC];
#pragma unroll
  for (int k = 0; k < HC; ++k) r1[k] = r2[k] = 0.f;
#pragma unroll 2
  for (int q = 0; q < kMdRun; ++q) {
    float s = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const float dd = yi[a] - tile[a][jl + q];
      s = __builtin_fmaf(dd, dd, s);
    }
    if (MASK) s = (jg + q > i) ? s : __builtin_inff();
#pragma unroll
    for (int k = 0; k < HC; ++k) {
      const float e = __builtin_amdgcn_exp2f(s * ck[k]);
      r1[k] += e;
      r2[k] = __builtin_fmaf(e, e, r2[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    md_fold(a1[k], c1[k], r1[k]);
    md_fold(a2[k], c2[k], r2[k]);
  }
}

template <int D, int HC>
__global__ __launch_bounds__(kThreads) void k_md_units_f32(const float* __restrict__ y, int npad,
                                                           const MdState* __restrict__ st,
                                                           const float* __restrict__ c32,
                                                           const Unit* __restrict__ units, int u0,
                                                           double* __restrict__ part, int n_items, int n_h) {
  if (st->status != kStOk) return;
  const Unit u = units[u0 + blockIdx.x];
  const int n = st->n;
  __shared__ float tile[D][kBJ];
  __shared__ double red[4][2 * HC];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = u.row * kBI;
  const int i = row0 + tid;
  float yi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) yi[a] = (i < n) ? y[(int64_t)a * npad + i] : 0.f;
  const int wave_i0 = row0 + wave * 64;
  float ck[HC], a1[HC], c1[HC], a2[HC], c2[HC];
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    ck[k] = c32[u.chunk * HC + k];
    a1[k] = c1[k] = a2[k] = c2[k] = 0.f;
  }
  for (int t0 = u.j_begin; t0 < u.j_end; t0 += kBJ) {
    __syncthreads();
    for (int a = 0; a < D; ++a)
      for (int q = tid; q < kBJ; q += kThreads) tile[a][q] = y[(int64_t)a * npad + t0 + q];
    __syncthreads();
    int js = max(t0, wave_i0);
    const int te = t0 + kBJ;
    if (js < te) {
      if (js == wave_i0) {
        md_run<D, HC, true>(tile, js - t0, js, yi, i, ck, a1, c1, a2, c2);
        js += kMdRun;
      }
      for (; js < te; js += kMdRun) md_run<D, HC, false>(tile, js - t0, js, yi, i, ck, a1, c1, a2, c2);
    }
  }
  const bool valid = i < n;
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    const double v1 = md_wave_sum(valid ? (double)a1[k] - (double)c1[k] : 0.0);
    const double v2 = md_wave_sum(valid ? (double)a2[k] - (double)c2[k] : 0.0);
    if (lane == 0) {
      red[wave][2 * k] = v1;
      red[wave][2 * k + 1] = v2;
    }
  }
  __syncthreads();
  if (tid < 2 * HC) {
    const int hh = u.chunk * HC + (tid >> 1);
    if (hh < n_h) {
      const double v = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
      part[(int64_t)(2 * hh + (tid & 1)) * n_items + u.item] = v;
    }
  }
}

template <int D, int HC>
__global__ __launch_bounds__(kThreads) void k_md_units_f64(const double* __restrict__ y, int npad,
                                                           const MdState* __restrict__ st,
                                                           const double* __restrict__ c64,
                                                           const Unit* __restrict__ units, int u0,
                                                           double* __restrict__ part, int n_items, int n_h) {
  if (st->status != kStOk) return;
  const Unit u = units[u0 + blockIdx.x];
  const int n = st->n;
  constexpr int kT = kBJ / 2;  // 256 j per tile keeps the FP64 tile within 32 KB
  __shared__ double tile[D][kT];
  __shared__ double red[4][2 * HC];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = u.row * kBI;
  const int i = row0 + tid;
  double yi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) yi[a] = (i < n) ? y[(int64_t)a * npad + i] : 0.0;
  double ck[HC], s1[HC], s2[HC];
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    ck[k] = c64[u.chunk * HC + k];
    s1[k] = s2[k] = 0.0;
  }
  for (int t0 = u.j_begin; t0 < u.j_end; t0 += kT) {
    __syncthreads();
    for (int a = 0; a < D; ++a)
      for (int q = tid; q < kT; q += kThreads) tile[a][q] = y[(int64_t)a * npad + t0 + q];
    __syncthreads();
    for (int q = 0; q < kT; ++q) {
      const int j = t0 + q;
      if (j <= i) continue;
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double dd = yi[a] - tile[a][q];
        s = fma(dd, dd, s);
      }
#pragma unroll
      for (int k = 0; k < HC; ++k) {
        const double e = exp(s * ck[k]);
        s1[k] += e;
        s2[k] = fma(e, e, s2[k]);
      }
    }
  }
  const bool valid = i < n;
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    const double v1 = md_wave_sum(valid ? s1[k] : 0.0);
    const double v2 = md_wave_sum(valid ? s2[k] : 0.0);
    if (lane == 0) {
      red[wave][2 * k] = v1;
      red[wave][2 * k + 1] = v2;
    }
  }
  __syncthreads();
  if (tid < 2 * HC) {
    const int hh = u.chunk * HC + (tid >> 1);
    if (hh < n_h) {
      const double v = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
      part[(int64_t)(2 * hh + (tid & 1)) * n_items + u.item] = v;
    }
  }
}

// g(h), gscale(h), argmin (ties to the lowest index), edge flag, margin
__global__ __launch_bounds__(1024) void k_md_finalize(MdState* st, const double* sums, const double* h,
                                                      const float* c32, int f64, int n_h, double* g, double* gs) {
  __shared__ double bv[1024];
  __shared__ int bk[1024];
  const int t = threadIdx.x;
  const bool ok = st->status == kStOk;
  const int d = st->d;
  const double n = (double)st->n;
  const double sq = exp(-0.5 * st->logdet);
  const double A = pow(4.0 * kPiD, -0.5 * d) * sq, B = pow(2.0 * kPiD, -0.5 * d) * sq;
  double best = __builtin_inf();
  int kbest = 0x7fffffff;
  for (int k = t; k < n_h; k += blockDim.x) {
    double hv = h[k];
    if (!f64) {
      // the bandwidth whose FP32 coefficient the pair sums used
      const double cq = (double)c32[k];
      if (cq < 0.0 && isfinite(cq)) hv = sqrt(-kLog2ED / (4.0 * cq));
    }
    const double hd = pow(hv, -(double)d);
    const double s1 = sums[2 * k], s2 = sums[2 * k + 1];
    const double gv = hd * (2.0 / (n * n) * (A * s1 - 2.0 * B * s2) + A / n);
    g[k] = ok ? gv : NAN;
    gs[k] = ok ? hd * (2.0 / (n * n) * (A * s1 + 2.0 * B * s2) + A / n) : NAN;
    if (ok && gv < best) {
      best = gv;
      kbest = k;
    }
  }
  bv[t] = best;
  bk[t] = kbest;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s && (bv[t + s] < bv[t] || (bv[t + s] == bv[t] && bk[t + s] < bk[t]))) {
      bv[t] = bv[t + s];
      bk[t] = bk[t + s];
    }
    __syncthreads();
  }
  const int kb = bk[0];
  const double vb = bv[0];
  __syncthreads();
  double second = __builtin_inf();
  for (int k = t; k < n_h; k += blockDim.x)
    if (k != kb) second = fmin(second, g[k]);
  bv[t] = second;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) bv[t] = fmin(bv[t], bv[t + s]);
    __syncthreads();
  }
  if (t == 0 && ok) {
    if (kb < n_h) {
      st->k_best = kb;
      st->h_best = h[kb];
      st->at_edge = (kb == 0 || kb == n_h - 1) ? 1 : 0;
      st->margin = n_h > 1 ? bv[0] - vb : 0.0;
    } else {
      st->status = kStDegenerate;
    }
  }
}

// ---- LSCV_H (Section 4.4.3): g(H) at bandwidth matrices H, batched for 1 <= d <= 4.
// In whitened coordinates w = Y_i - Y_j the quadratic form of the pair is
// v^T H^-1 v = w^T P w with P = G^-1, G = L^-1 H L^-T (Sigma = L L^T).  A pair's
// monomials w_a w_b (a <= b < D) are formed once in registers and each matrix
// then costs one dot product with its packed coefficients, one exp2 and two
// accumulations.  The mixed form rounds the coefficients to FP32 and
// evaluates g at the matrix they represent exactly (its determinant taken
// from the rounded coefficients), so each g is a consistent evaluation at a
// matrix within FP32 rounding of H.  Padding samples are masked by index
// (their +inf coordinate would meet cross terms of either sign).
constexpr int kMaxHD = 4;
constexpr int kMaxMono = kMaxHD * (kMaxHD + 1) / 2;

struct HDesc {
  float c32[kMaxMono];   // -log2(e)/4 * P_ab * (a == b ? 1 : 2), a <= b < D, FP32
  int valid;             // H, G (and in the mixed form the rounded P) positive definite
  int pad0;
  double c64[kMaxMono];  // -1/4 * P_ab * (a == b ? 1 : 2), FP64
  double logdet64;       // log |H|
  double logdet32;       // log |H32|, H32 = L P32^-1 L^T the matrix of the FP32 coefficients
};

// Cholesky factor of the d x d symmetric matrix A with the library's pivot
// rule (a pivot at most 1e-12 of its diagonal entry fails) and log|A|.
__device__ bool h_chol(const double (&A)[kMaxHD][kMaxHD], int d, double (&L)[kMaxHD][kMaxHD], double& logdet) {
  for (int a = 0; a < kMaxHD; ++a)
    for (int b = 0; b < kMaxHD; ++b) L[a][b] = 0.0;
  logdet = 0.0;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b) {
      double s = A[a][b];
      for (int k = 0; k < b; ++k) s -= L[a][k] * L[b][k];
      if (a == b) {
        if (!(s > 1e-12 * A[a][a]) || !isfinite(s)) return false;
        L[a][a] = sqrt(s);
        logdet += 2.0 * log(L[a][a]);
      } else {
        L[a][b] = s / L[b][b];
      }
    }
  return true;
}

// one thread per matrix (H row-major d x d, its lower triangle read): G,
// P = G^-1, the packed coefficients over D coordinates and both determinants
__global__ void k_H_prep(const MdState* st, const double* H, int m, int D, int f64, HDesc* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int d = st->d;
  HDesc o;
  for (int q = 0; q < kMaxMono; ++q) {
    o.c32[q] = 0.f;
    o.c64[q] = 0.0;
  }
  o.valid = 0;
  o.pad0 = 0;
  o.logdet64 = o.logdet32 = 0.0;
  double Hs[kMaxHD][kMaxHD], G[kMaxHD][kMaxHD], T[kMaxHD][kMaxHD], L[kMaxHD][kMaxHD];
  const double* Hk = H + (int64_t)k * d * d;
  for (int a = 0; a < kMaxHD; ++a)
    for (int b = 0; b < kMaxHD; ++b) Hs[a][b] = (a < d && b < d) ? Hk[max(a, b) * d + min(a, b)] : 0.0;
  double ldH, ldG;
  bool ok = st->status == kStOk && h_chol(Hs, d, L, ldH);
  if (ok) {
    for (int a = 0; a < d; ++a)  // T = L^-1 H
      for (int b = 0; b < d; ++b) {
        double s = 0.0;
        for (int c = 0; c <= a; ++c) s += st->linv[a * KDE_MAX_D + c] * Hs[c][b];
        T[a][b] = s;
      }
    for (int a = 0; a < d; ++a)  // G = T L^-T (lower triangle, mirrored)
      for (int b = 0; b <= a; ++b) {
        double s = 0.0;
        for (int c = 0; c <= b; ++c) s += T[a][c] * st->linv[b * KDE_MAX_D + c];
        G[a][b] = G[b][a] = s;
      }
    ok = h_chol(G, d, L, ldG);
  }
  if (ok) {
    double Li[kMaxHD][kMaxHD], P[kMaxHD][kMaxHD], P32[kMaxHD][kMaxHD];
    for (int c = 0; c < d; ++c)  // L_G^-1, lower triangular
      for (int a = 0; a < d; ++a) {
        if (a < c) {
          Li[a][c] = 0.0;
          continue;
        }
        double s = (a == c) ? 1.0 : 0.0;
        for (int q = c; q < a; ++q) s -= L[a][q] * Li[q][c];
        Li[a][c] = s / L[a][a];
      }
    for (int a = 0; a < d; ++a)  // P = L_G^-T L_G^-1
      for (int b = 0; b < d; ++b) {
        double s = 0.0;
        for (int q = max(a, b); q < d; ++q) s += Li[q][a] * Li[q][b];
        P[a][b] = s;
      }
    int q = 0;
    for (int a = 0; a < D; ++a)
      for (int b = a; b < D; ++b, ++q) {
        if (b >= d) continue;
        const double w = (a == b) ? 0.25 : 0.5;
        o.c64[q] = -w * P[a][b];
        o.c32[q] = (float)(-kLog2ED * w * P[a][b]);
        P32[a][b] = P32[b][a] = (double)o.c32[q] / (-kLog2ED * w);
      }
    double ldP32;
    const bool ok32 = f64 || h_chol(P32, d, L, ldP32);
    o.logdet64 = st->logdet + ldG;
    o.logdet32 = f64 ? o.logdet64 : st->logdet - ldP32;
    o.valid = ok32 ? 1 : 0;
  }
  out[k] = o;
}

// ---- LSCV_H for 4 < d <= 16: one matrix a sweep.  With G = L_G L_G^T the
// quadratic form is |L_G^-1 w|^2, so the samples are whitened once more,
// Z = M (X - mean) with M = L_G^-1 L^-1 (lower triangular), and the sphered
// pair kernel runs on Z with the single coefficient -1/4 (S2 from e^2).
// Both forms evaluate g at H itself; the mixed form rounds Z to FP32.
__global__ void k_HT_prep(const MdState* st, const double* H, int m, HDesc* out, double* Mout) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int d = st->d;
  double A[KDE_MAX_D][KDE_MAX_D], L[KDE_MAX_D][KDE_MAX_D], T[KDE_MAX_D][KDE_MAX_D];
  double* M = Mout + (int64_t)k * KDE_MAX_D * KDE_MAX_D;
  for (int q = 0; q < KDE_MAX_D * KDE_MAX_D; ++q) M[q] = 0.0;
  HDesc o;
  for (int q = 0; q < kMaxMono; ++q) {
    o.c32[q] = 0.f;
    o.c64[q] = 0.0;
  }
  o.valid = 0;
  o.pad0 = 0;
  o.logdet64 = o.logdet32 = 0.0;
  const double* Hk = H + (int64_t)k * d * d;
  // Cholesky of A with the library's pivot rule; returns log|A| or NaN
  auto chol = [&](double& ld) {
    ld = 0.0;
    for (int a = 0; a < d; ++a)
      for (int b = 0; b <= a; ++b) {
        double s = A[a][b];
        for (int c = 0; c < b; ++c) s -= L[a][c] * L[b][c];
        if (a == b) {
          if (!(s > 1e-12 * A[a][a]) || !isfinite(s)) return false;
          L[a][a] = sqrt(s);
          ld += 2.0 * log(L[a][a]);
        } else {
          L[a][b] = s / L[b][b];
        }
      }
    return true;
  };
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b) A[a][b] = A[b][a] = Hk[a * d + b];
  double ldH, ldG;
  if (st->status != kStOk || !chol(ldH)) {
    out[k] = o;
    return;
  }
  for (int a = 0; a < d; ++a)  // T = L^-1 H
    for (int b = 0; b < d; ++b) {
      double s = 0.0;
      for (int c = 0; c <= a; ++c) s += st->linv[a * KDE_MAX_D + c] * A[c][b];
      T[a][b] = s;
    }
  for (int a = 0; a < d; ++a)  // G = T L^-T into A
    for (int b = 0; b <= a; ++b) {
      double s = 0.0;
      for (int c = 0; c <= b; ++c) s += T[a][c] * st->linv[b * KDE_MAX_D + c];
      A[a][b] = A[b][a] = s;
    }
  if (!chol(ldG)) {
    out[k] = o;
    return;
  }
  for (int c = 0; c < d; ++c)  // T = L_G^-1 (lower)
    for (int a = 0; a < d; ++a) {
      if (a < c) {
        T[a][c] = 0.0;
        continue;
      }
      double s = (a == c) ? 1.0 : 0.0;
      for (int q = c; q < a; ++q) s -= L[a][q] * T[q][c];
      T[a][c] = s / L[a][a];
    }
  for (int a = 0; a < d; ++a)  // M = L_G^-1 L^-1
    for (int b = 0; b <= a; ++b) {
      double s = 0.0;
      for (int c = b; c <= a; ++c) s += T[a][c] * st->linv[c * KDE_MAX_D + b];
      M[a * KDE_MAX_D + b] = s;
    }
  o.logdet64 = o.logdet32 = st->logdet + ldG;
  o.valid = 1;
  out[k] = o;
}

template <int D, int MH, bool MASK>
__device__ __forceinline__ void h_run(const float (*tile)[kBJ], int jl, int jg, int n, const float (&yi)[D], int i,
                                      const float (&ck)[MH][D * (D + 1) / 2], float (&a1)[MH], float (&c1)[MH],
                                      float (&a2)[MH], float (&c2)[MH]) {
  constexpr int NM = D * (D + 1) / 2;
  float r1[MH], r2[MH];
#pragma unroll
  for (int k = 0; k < MH; ++k) r1[k] = r2[k] = 0.f;
#pragma unroll 2
  for (int q = 0; q < kMdRun; ++q) {
    float w[D], mono[NM];
#pragma unroll
    for (int a = 0; a < D; ++a) w[a] = yi[a] - tile[a][jl + q];
    int t = 0;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = a; b < D; ++b) mono[t++] = w[a] * w[b];
    const bool live = !MASK || (jg + q > i && jg + q < n);
#pragma unroll
    for (int k = 0; k < MH; ++k) {
      float s = ck[k][0] * mono[0];
#pragma unroll
      for (int mm = 1; mm < NM; ++mm) s = __builtin_fmaf(ck[k][mm], mono[mm], s);
      s = live ? s : -__builtin_inff();
      const float e = __builtin_amdgcn_exp2f(s);
      r1[k] += e;
      r2[k] = __builtin_fmaf(e, e, r2[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < MH; ++k) {
    md_fold(a1[k], c1[k], r1[k]);
    md_fold(a2[k], c2[k], r2[k]);
  }
}

// block b of a launch: global index u0 + b = chunk * n_items + item; 256
// samples i x the item's j-range x matrices chunk*MH ... chunk*MH + MH - 1;
// part[(2 k + s) * n_items + item], s = 0: S1, 1: S2
template <int D, int MH>
__device__ __forceinline__ void h_store(const double (&v1)[MH], const double (&v2)[MH], const Unit& u, int chunk,
                                        int m, double* part, int n_items, double (*red)[2 * MH]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int k = 0; k < MH; ++k) {
    const double s1 = md_wave_sum(v1[k]);
    const double s2 = md_wave_sum(v2[k]);
    if (lane == 0) {
      red[wave][2 * k] = s1;
      red[wave][2 * k + 1] = s2;
    }
  }
  __syncthreads();
  if (tid < 2 * MH) {
    const int hk = chunk * MH + (tid >> 1);
    if (hk < m) part[(int64_t)(2 * hk + (tid & 1)) * n_items + u.item] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
  }
}

template <int D, int MH>
__global__ __launch_bounds__(kThreads) void k_H_units_f32(const float* __restrict__ y, int npad,
                                                          const MdState* __restrict__ st,
                                                          const HDesc* __restrict__ hd, int m,
                                                          const Unit* __restrict__ units, int u0,
                                                          double* __restrict__ part, int n_items) {
  if (st->status != kStOk) return;
  constexpr int NM = D * (D + 1) / 2;
  const int gidx = u0 + blockIdx.x;
  const int chunk = gidx / n_items;
  const Unit u = units[gidx - chunk * n_items];
  const int n = st->n;
  __shared__ float tile[D][kBJ];
  __shared__ double red[4][2 * MH];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = u.row * kBI;
  const int i = row0 + tid;
  float yi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) yi[a] = (i < n) ? y[(int64_t)a * npad + i] : 0.f;
  const int wave_i0 = row0 + wave * 64;
  float ck[MH][NM], a1[MH], c1[MH], a2[MH], c2[MH];
#pragma unroll
  for (int k = 0; k < MH; ++k) {
    const int hk = chunk * MH + k;
    const bool use = hk < m && hd[hk].valid;
#pragma unroll
    for (int mm = 0; mm < NM; ++mm) ck[k][mm] = use ? hd[hk].c32[mm] : 0.f;
    a1[k] = c1[k] = a2[k] = c2[k] = 0.f;
  }
  for (int t0 = u.j_begin; t0 < u.j_end; t0 += kBJ) {
    __syncthreads();
    for (int a = 0; a < D; ++a)
      for (int q = tid; q < kBJ; q += kThreads) tile[a][q] = y[(int64_t)a * npad + t0 + q];
    __syncthreads();
    int js = max(t0, wave_i0);
    const int te = t0 + kBJ;
    if (te > n) {  // the column's last tile: padding masked by index
      for (; js < te; js += kMdRun) h_run<D, MH, true>(tile, js - t0, js, n, yi, i, ck, a1, c1, a2, c2);
    } else if (js < te) {
      if (js == wave_i0) {
        h_run<D, MH, true>(tile, js - t0, js, n, yi, i, ck, a1, c1, a2, c2);
        js += kMdRun;
      }
      for (; js < te; js += kMdRun) h_run<D, MH, false>(tile, js - t0, js, n, yi, i, ck, a1, c1, a2, c2);
    }
  }
  const bool valid = i < n;
  double v1[MH], v2[MH];
#pragma unroll
  for (int k = 0; k < MH; ++k) {
    v1[k] = valid ? (double)a1[k] - (double)c1[k] : 0.0;
    v2[k] = valid ? (double)a2[k] - (double)c2[k] : 0.0;
  }
  h_store<D, MH>(v1, v2, u, chunk, m, part, n_items, red);
}

template <int D, int MH>
__global__ __launch_bounds__(kThreads) void k_H_units_f64(const double* __restrict__ y, int npad,
                                                          const MdState* __restrict__ st,
                                                          const HDesc* __restrict__ hd, int m,
                                                          const Unit* __restrict__ units, int u0,
                                                          double* __restrict__ part, int n_items) {
  if (st->status != kStOk) return;
  constexpr int NM = D * (D + 1) / 2;
  constexpr int kT = kBJ / 2;
  const int gidx = u0 + blockIdx.x;
  const int chunk = gidx / n_items;
  const Unit u = units[gidx - chunk * n_items];
  const int n = st->n;
  __shared__ double tile[D][kT];
  __shared__ double red[4][2 * MH];
  const int tid = threadIdx.x;
  const int i = u.row * kBI + tid;
  double yi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) yi[a] = (i < n) ? y[(int64_t)a * npad + i] : 0.0;
  double ck[MH][NM], s1[MH], s2[MH];
#pragma unroll
  for (int k = 0; k < MH; ++k) {
    const int hk = chunk * MH + k;
    const bool use = hk < m && hd[hk].valid;
#pragma unroll
    for (int mm = 0; mm < NM; ++mm) ck[k][mm] = use ? hd[hk].c64[mm] : 0.0;
    s1[k] = s2[k] = 0.0;
  }
  for (int t0 = u.j_begin; t0 < u.j_end; t0 += kT) {
    __syncthreads();
    for (int a = 0; a < D; ++a)
      for (int q = tid; q < kT; q += kThreads) tile[a][q] = y[(int64_t)a * npad + t0 + q];
    __syncthreads();
    const int qa = max(0, i + 1 - t0), qb = min(kT, n - t0);
    for (int q = qa; q < qb; ++q) {
      double w[D], mono[NM];
#pragma unroll
      for (int a = 0; a < D; ++a) w[a] = yi[a] - tile[a][q];
      int t = 0;
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) mono[t++] = w[a] * w[b];
#pragma unroll
      for (int k = 0; k < MH; ++k) {
        double sq = 0.0;
#pragma unroll
        for (int mm = 0; mm < NM; ++mm) sq = fma(ck[k][mm], mono[mm], sq);
        const double e = exp(sq);
        s1[k] += e;
        s2[k] = fma(e, e, s2[k]);
      }
    }
  }
  const bool valid = i < n;
  double v1[MH], v2[MH];
#pragma unroll
  for (int k = 0; k < MH; ++k) {
    v1[k] = valid ? s1[k] : 0.0;
    v2[k] = valid ? s2[k] : 0.0;
  }
  h_store<D, MH>(v1, v2, u, chunk, m, part, n_items, red);
}

// g(H) = 2 n^-2 (A S1 - 2 B S2) + n^-1 R with A = (4 pi)^(-d/2) |H|^(-1/2),
// B = (2 pi)^(-d/2) |H|^(-1/2), R = 2^-d pi^(-d/2) |H|^(-1/2) (eq. LSCV_MULTI-gh
// with LSCV_MULTI-Kx, -KKx, -rk), and the scale of its terms
// 2 n^-2 (A S1 + 2 B S2) + n^-1 R; +inf (scale 0) for a matrix that is not
// positive definite, NaN when the samples were rejected
__global__ void k_H_final(const MdState* st, const HDesc* hd, int m, int f64, const double* sums, double* g,
                          double* gs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  if (st->status != kStOk) {
    g[k] = gs[k] = NAN;
    return;
  }
  if (!hd[k].valid) {
    g[k] = __builtin_inf();
    gs[k] = 0.0;
    return;
  }
  const int d = st->d;
  const double n = (double)st->n;
  const double sq = exp(-0.5 * (f64 ? hd[k].logdet64 : hd[k].logdet32));
  const double A = pow(4.0 * kPiD, -0.5 * d) * sq, B = pow(2.0 * kPiD, -0.5 * d) * sq;
  const double R = pow(2.0, -(double)d) * pow(kPiD, -0.5 * d) * sq;
  g[k] = 2.0 / (n * n) * (A * sums[2 * k] - 2.0 * B * sums[2 * k + 1]) + R / n;
  gs[k] = 2.0 / (n * n) * (A * sums[2 * k] + 2.0 * B * sums[2 * k + 1]) + R / n;
}

template <int D, int MH>
void launch_H_units(hipStream_t s, bool f64, const float* y32, const double* y64, int npad, const MdState* st,
                    const HDesc* hd, int m, const Unit* units, int u0, int cnt, double* part, int n_items) {
  if (f64)
    k_H_units_f64<D, MH><<<cnt, kThreads, 0, s>>>(y64, npad, st, hd, m, units, u0, part, n_items);
  else
    k_H_units_f32<D, MH><<<cnt, kThreads, 0, s>>>(y32, npad, st, hd, m, units, u0, part, n_items);
}

void launch_H(hipStream_t s, int D, int MH, bool f64, const float* y32, const double* y64, int npad,
              const MdState* st, const HDesc* hd, int m, const Unit* units, int u0, int cnt, double* part,
              int n_items) {
#define KDE_H_CASE(DD)                                                                                     \
  switch (MH) {                                                                                            \
    case 1: launch_H_units<DD, 1>(s, f64, y32, y64, npad, st, hd, m, units, u0, cnt, part, n_items); return; \
    case 2: launch_H_units<DD, 2>(s, f64, y32, y64, npad, st, hd, m, units, u0, cnt, part, n_items); return; \
    default: launch_H_units<DD, 4>(s, f64, y32, y64, npad, st, hd, m, units, u0, cnt, part, n_items); return; \
  }
  if (D == 2 && MH == 8) {
    launch_H_units<2, 8>(s, f64, y32, y64, npad, st, hd, m, units, u0, cnt, part, n_items);
    return;
  }
  switch (D) {
    case 2: KDE_H_CASE(2);
    case 3: KDE_H_CASE(3);
    default: KDE_H_CASE(4);
  }
#undef KDE_H_CASE
}

template <int D, int HC>
void launch_md_units(hipStream_t s, bool f64, const float* y32, const double* y64, int npad, const MdState* st,
                     const float* c32, const double* c64, const Unit* units, int u0, int cnt, double* part,
                     int n_items, int n_h) {
  if (f64)
    k_md_units_f64<D, HC><<<cnt, kThreads, 0, s>>>(y64, npad, st, c64, units, u0, part, n_items, n_h);
  else
    k_md_units_f32<D, HC><<<cnt, kThreads, 0, s>>>(y32, npad, st, c32, units, u0, part, n_items, n_h);
}

// coordinates per sample as compiled (d rounded up; unused coordinates are 0)
int md_width(int d) { return d <= 2 ? 2 : d <= 3 ? 3 : d <= 4 ? 4 : d <= 8 ? 8 : 16; }
// bandwidths per block: fewer for wide samples (registers)
int md_hc(int D, bool f64) { return f64 ? 4 : (D <= 4 ? 16 : 8); }

void launch_md(hipStream_t s, int D, bool f64, const float* y32, const double* y64, int npad, const MdState* st,
               const float* c32, const double* c64, const Unit* units, int u0, int cnt, double* part, int n_items,
               int n_h) {
#define KDE_MD_CASE(DD, HH)                                                                                  \
  launch_md_units<DD, HH>(s, f64, y32, y64, npad, st, c32, c64, units, u0, cnt, part, n_items, n_h);          \
  return
  if (f64) {
    switch (D) {
      case 2: KDE_MD_CASE(2, 4);
      case 3: KDE_MD_CASE(3, 4);
      case 4: KDE_MD_CASE(4, 4);
      case 8: KDE_MD_CASE(8, 4);
      default: KDE_MD_CASE(16, 4);
    }
  }
  switch (D) {
    case 2: KDE_MD_CASE(2, 16);
    case 3: KDE_MD_CASE(3, 16);
    case 4: KDE_MD_CASE(4, 16);
    case 8: KDE_MD_CASE(8, 8);
    default: KDE_MD_CASE(16, 8);
  }
#undef KDE_MD_CASE
}

// ---- consumers for d-dimensional samples: the density with a bandwidth
// matrix (eq. kde-def-H with K_H of eq. (K_H) and the Gaussian K) at query
// points, d <= 16, and range COUNT/SUM over boxes for d = 2 (eq.
// count-sum-2D).
//
// Density: with H = L_H L_H^T the quadratic form (p - X_i)^T H^-1 (p - X_i)
// is |L_H^-1 (p - mean) - L_H^-1 (X_i - mean)|^2, so samples and query points
// are whitened once by L_H^-1 (FP64, the sample mean subtracted) and a block
// holds 256 query points, one per lane, sweeping a piece of the samples in
// LDS tiles of 256 x D coordinates.  The squared distance is FP64 in both
// forms; the mixed form takes exp2 of its FP32-rounded exponent in FP32,
// 64-term runs folded into a compensated FP32 sum; the FP64 form takes exp
// in FP64.  f(p) = n^-1 (2 pi)^(-d/2) |H|^(-1/2) sum_i exp(-|.|^2 / 2).
//
// Range aggregates, d = 2: per sample the kernel is a bivariate normal with
// mean X_i and covariance H, so over a box the sample contributes its
// rectangle probability P, and E[U 1{box}], E[V 1{box}] of its standardised
// coordinates (U, V), corr rho:
//   COUNT = sum_i P_i,  SUM_x = sum_i (x_i P_i + sqrt(H11) E[U]_i),
//   SUM_y = sum_i (y_i P_i + sqrt(H22) E[V]_i).
// P is four corner values of the bivariate normal CDF, each from Owen's
// T function, Phi2(h, k; rho) = (Phi(h) + Phi(k))/2 - T(h, a_h) - T(k, a_k)
// - beta (Owen 1956), a_h = (k - rho h)/(h s), a_k = (h - rho k)/(k s),
// s = sqrt(1 - rho^2), beta = 1/2 when h k < 0 (or h k = 0 and h + k < 0);
// T(h, a) for |a| <= 1 by 20-point Gauss-Legendre quadrature of its integral
// over [0, min(a, 9/h)], for |a| > 1 through T(h, a) + T(ah, 1/a) =
// (Phi(h) Q(ah) + Phi(ah) Q(h))/2 (Q the upper tail).  The box is first
// reflected so that each interval's midpoint is at most 0 (the corner values
// are then small and carry relative precision).  E[U 1{box}] integrates by
// parts in closed form:
//   phi(al1) G(al1) - phi(be1) G(be1)
//   - rho [phi(be2) (Phi((be1 - rho be2)/s) - Phi((al1 - rho be2)/s))
//          - phi(al2) (Phi((be1 - rho al2)/s) - Phi((al1 - rho al2)/s))],
// G(u) = Phi((be2 - rho u)/s) - Phi((al2 - rho u)/s), and E[V] alike with the
// roles swapped.  All FP64; absolute error about 1e-16 of a sample's mass.

// 20-point Gauss-Legendre rule on [-1, 1]: the positive nodes and their weights
__constant__ double kGL20[10][2] = {
    {0.076526521133497338, 0.15275338713072578}, {0.2277858511416451, 0.14917298647260366},
    {0.37370608871541955, 0.14209610931838187},  {0.51086700195082713, 0.13168863844917653},
    {0.63605368072651502, 0.11819453196151825},  {0.7463319064601508, 0.10193011981724026},
    {0.83911697182221878, 0.083276741576704671}, {0.91223442825132584, 0.062672048334109443},
    {0.96397192727791381, 0.040601429800386217}, {0.99312859918509488, 0.017614007139153273},
};
constexpr double kInvSqrt2D = 0.70710678118654752440;
constexpr double kInvSqrt2PiD = 0.39894228040143267794;

// one thread: Cholesky factor of H (lower triangle read, the pivot rule of the
// library), L_H^-1 into st->linv and log|H| into st->logdet
__global__ void k_dq_factor(MdState* st, const double* H) {
  if (threadIdx.x != 0 || st->status != kStOk) return;
  const int d = st->d;
  double A[KDE_MAX_D][KDE_MAX_D], L[KDE_MAX_D][KDE_MAX_D];
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b) A[a][b] = H[a * d + b];
  double ld = 0.0;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b) {
      double s = A[a][b];
      for (int c = 0; c < b; ++c) s -= L[a][c] * L[b][c];
      if (a == b) {
        if (!(s > 1e-12 * A[a][a]) || !isfinite(s)) {
          st->status = kStDegenerate;
          return;
        }
        L[a][a] = sqrt(s);
        ld += 2.0 * log(L[a][a]);
      } else {
        L[a][b] = s / L[b][b];
      }
    }
  for (int c = 0; c < d; ++c)
    for (int a = 0; a < d; ++a) {
      double s = (a == c) ? 1.0 : 0.0;
      for (int k = c; k < a; ++k) s -= L[a][k] * st->linv[k * KDE_MAX_D + c];
      st->linv[a * KDE_MAX_D + c] = a < c ? 0.0 : s / L[a][a];
    }
  st->logdet = ld;
}

// grid (query blocks, pieces): part[q * pieces + piece] = sum over the piece
template <int D, bool F64>
__global__ __launch_bounds__(kThreads) void k_dq_units(const double* __restrict__ zq, int m, int mpad,
                                                       const double* __restrict__ y, int npad,
                                                       const MdState* __restrict__ st, int piece_len, int pieces,
                                                       double* __restrict__ part) {
  if (st->status != kStOk) return;
  const int n = st->n;
  __shared__ double tile[D][kThreads];
  const int tid = threadIdx.x;
  const int k = blockIdx.x * kThreads + tid;
  double q[D];
#pragma unroll
  for (int a = 0; a < D; ++a) q[a] = (k < m) ? zq[(int64_t)a * mpad + k] : 0.0;
  const int j0 = blockIdx.y * piece_len, j1 = min(n, j0 + piece_len);
  float acc = 0.f, comp = 0.f;
  double s64 = 0.0;
  for (int t0 = j0; t0 < j1; t0 += kThreads) {
    __syncthreads();
#pragma unroll
    for (int a = 0; a < D; ++a) tile[a][tid] = y[(int64_t)a * npad + t0 + tid];
    __syncthreads();
    const int cnt = min(kThreads, j1 - t0);
    for (int u0 = 0; u0 < cnt; u0 += kMdRun) {
      const int u1 = min(cnt, u0 + kMdRun);
      float run = 0.f;
      for (int u = u0; u < u1; ++u) {
        double d2 = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const double t = q[a] - tile[a][u];
          d2 = fma(t, t, d2);
        }
        if (F64)
          s64 += exp(-0.5 * d2);
        else
          run += __builtin_amdgcn_exp2f((float)(-0.5 * kLog2ED * d2));
      }
      if (!F64) md_fold(acc, comp, run);
    }
  }
  if (k < m) part[(int64_t)k * pieces + blockIdx.y] = F64 ? s64 : (double)acc - (double)comp;
}

__global__ __launch_bounds__(kThreads) void k_dq_final(const MdState* st, const double* part, int m, int pieces,
                                                      double* out) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k >= m) return;
  if (st->status != kStOk) {
    out[k] = NAN;
    return;
  }
  double s = 0.0;
  for (int p = 0; p < pieces; ++p) s += part[(int64_t)k * pieces + p];
  out[k] = s * pow(2.0 * kPiD, -0.5 * st->d) * exp(-0.5 * st->logdet) / (double)st->n;
}

__device__ __forceinline__ double q_upper(double z) { return 0.5 * erfc(z * kInvSqrt2D); }
__device__ __forceinline__ double q_cdf(double z) { return 0.5 * erfc(-z * kInvSqrt2D); }
__device__ __forceinline__ double q_pdf(double z) { return isinf(z) ? 0.0 : kInvSqrt2PiD * exp(-0.5 * z * z); }
// Phi(b) - Phi(a), a <= b, between tails
__device__ __forceinline__ double q_diff(double a, double b) {
  if (a >= 0.0) return q_upper(a) - q_upper(b);
  if (b <= 0.0) return q_upper(-b) - q_upper(-a);
  return 1.0 - q_upper(-a) - q_upper(b);
}

// Owen's T(h, a) for h >= 0, 0 < a <= 1: Gauss-Legendre over [0, min(a, 9/h)]
// (beyond 9/h the integrand is below e^-40 of its value at 0)
__device__ double owen_gl(double h, double a) {
  const double lim = h > 0.0 ? fmin(a, 9.0 / h) : a;
  const double half = 0.5 * lim, hh = -0.5 * h * h;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    const double tp = half * (1.0 + kGL20[k][0]), tm = half * (1.0 - kGL20[k][0]);
    const double fp = exp(hh * (1.0 + tp * tp)) / (1.0 + tp * tp);
    const double fm = exp(hh * (1.0 + tm * tm)) / (1.0 + tm * tm);
    s += kGL20[k][1] * (fp + fm);
  }
  return half * s / (2.0 * kPiD);
}

__device__ double owen_t(double h, double a) {
  h = fabs(h);
  if (a == 0.0) return 0.0;
  const double sg = a > 0.0 ? 1.0 : -1.0;
  a = fabs(a);
  if (isinf(a)) return sg * 0.5 * q_upper(h);
  if (a <= 1.0) return sg * owen_gl(h, a);
  const double ah = a * h;
  return sg * (0.5 * (q_cdf(h) * q_upper(ah) + q_cdf(ah) * q_upper(h)) - owen_gl(ah, 1.0 / a));
}

// bivariate standard normal CDF P(U <= h, V <= k), corr r, s = sqrt(1 - r^2)
__device__ double bvn_cdf(double h, double k, double r, double s) {
  if (h == -__builtin_inf() || k == -__builtin_inf()) return 0.0;
  if (h == __builtin_inf()) return q_cdf(k);
  if (k == __builtin_inf()) return q_cdf(h);
  if (h == 0.0 && k == 0.0) return 0.25 + asin(r) / (2.0 * kPiD);
  const double ah = h != 0.0 ? (k - r * h) / (h * s) : copysign(__builtin_inf(), k);
  const double ak = k != 0.0 ? (h - r * k) / (k * s) : copysign(__builtin_inf(), h);
  const double beta = (h * k < 0.0 || (h * k == 0.0 && h + k < 0.0)) ? 0.5 : 0.0;
  return 0.5 * (q_cdf(h) + q_cdf(k)) - owen_t(h, ah) - owen_t(k, ak) - beta;
}

// E[U 1{al1 <= U <= be1, al2 <= V <= be2}] (terms at infinite limits vanish)
__device__ double bvn_first_moment(double al1, double be1, double al2, double be2, double r, double s) {
  double e = 0.0;
  if (!isinf(al1)) e += q_pdf(al1) * q_diff((al2 - r * al1) / s, (be2 - r * al1) / s);
  if (!isinf(be1)) e -= q_pdf(be1) * q_diff((al2 - r * be1) / s, (be2 - r * be1) / s);
  double t = 0.0;
  if (!isinf(be2)) t += q_pdf(be2) * q_diff((al1 - r * be2) / s, (be1 - r * be2) / s);
  if (!isinf(al2)) t -= q_pdf(al2) * q_diff((al1 - r * al2) / s, (be1 - r * al2) / s);
  return e - r * t;
}

// grid (boxes, pieces): one box per block, lanes stride over the piece's samples
__global__ __launch_bounds__(kThreads) void k_r2_units(const void* raw, int fx, const MdState* st, double h11,
                                                       double h21, double h22, const double* __restrict__ boxes,
                                                       int piece_len, int pieces, double* __restrict__ part) {
  __shared__ double sh[kThreads];
  const int bx = blockIdx.x;
  const double lo1 = boxes[4 * bx], hi1 = boxes[4 * bx + 1], lo2 = boxes[4 * bx + 2], hi2 = boxes[4 * bx + 3];
  const double s1 = sqrt(h11), s2 = sqrt(h22), rho = h21 / (s1 * s2), sr = sqrt((1.0 - rho) * (1.0 + rho));
  const int n = st->n;
  const int i0 = blockIdx.y * piece_len, i1 = min(n, i0 + piece_len);
  double cnt = 0.0, sx = 0.0, sy = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
    const double xi = md_raw(raw, fx, 2 * (int64_t)i), yi = md_raw(raw, fx, 2 * (int64_t)i + 1);
    double a1 = (lo1 - xi) / s1, b1 = (hi1 - xi) / s1, a2 = (lo2 - yi) / s2, b2 = (hi2 - yi) / s2;
    // reflect each interval whose midpoint is above 0 (an interval with both
    // ends infinite stays)
    const bool f1 = !(isinf(a1) && isinf(b1)) && a1 + b1 > 0.0;
    const bool f2 = !(isinf(a2) && isinf(b2)) && a2 + b2 > 0.0;
    if (f1) {
      const double t = a1;
      a1 = -b1;
      b1 = -t;
    }
    if (f2) {
      const double t = a2;
      a2 = -b2;
      b2 = -t;
    }
    const double r = (f1 != f2) ? -rho : rho;
    double P = 0.0, eu = 0.0, ev = 0.0;
    if (a1 < b1 && a2 < b2) {
      P = bvn_cdf(b1, b2, r, sr) - bvn_cdf(a1, b2, r, sr) - bvn_cdf(b1, a2, r, sr) + bvn_cdf(a1, a2, r, sr);
      P = fmax(P, 0.0);
      eu = bvn_first_moment(a1, b1, a2, b2, r, sr);
      ev = bvn_first_moment(a2, b2, a1, b1, r, sr);
      if (f1) eu = -eu;
      if (f2) ev = -ev;
    }
    cnt += P;
    sx += xi * P + s1 * eu;
    sy += yi * P + s2 * ev;
  }
  cnt = md_block_sum(cnt, sh);
  sx = md_block_sum(sx, sh);
  sy = md_block_sum(sy, sh);
  if (threadIdx.x == 0) {
    double* o = part + ((int64_t)bx * pieces + blockIdx.y) * 3;
    o[0] = cnt;
    o[1] = sx;
    o[2] = sy;
  }
}

// per box, fixed-order sums over pieces: COUNT, SUM_x, SUM_y, AVG_x, AVG_y
__global__ __launch_bounds__(kThreads) void k_r2_final(const MdState* st, const double* __restrict__ part,
                                                      int pieces, double* __restrict__ out) {
  __shared__ double sh[kThreads];
  const int bx = blockIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  for (int p = threadIdx.x; p < pieces; p += kThreads)
    for (int c = 0; c < 3; ++c) v[c] += part[((int64_t)bx * pieces + p) * 3 + c];
  for (int c = 0; c < 3; ++c) v[c] = md_block_sum(v[c], sh);
  if (threadIdx.x == 0) {
    const bool ok = st->status == kStOk;
    out[5 * bx] = ok ? v[0] : NAN;
    out[5 * bx + 1] = ok ? v[1] : NAN;
    out[5 * bx + 2] = ok ? v[2] : NAN;
    out[5 * bx + 3] = ok && v[0] > 0.0 ? v[1] / v[0] : NAN;
    out[5 * bx + 4] = ok && v[0] > 0.0 ? v[2] / v[0] : NAN;
  }
}

template <int D>
void launch_dq(hipStream_t s, bool f64, dim3 grid, const double* zq, int m, int mpad, const double* y, int npad,
               const MdState* st, int piece_len, int pieces, double* part) {
  if (f64)
    k_dq_units<D, true><<<grid, kThreads, 0, s>>>(zq, m, mpad, y, npad, st, piece_len, pieces, part);
  else
    k_dq_units<D, false><<<grid, kThreads, 0, s>>>(zq, m, mpad, y, npad, st, piece_len, pieces, part);
}

// pieces of the samples so that a launch has about 4096 blocks, each piece at
// least 2048 samples
int dq_pieces(int64_t n, int64_t other_blocks) {
  const int64_t want = std::max<int64_t>(1, 4096 / std::max<int64_t>(1, other_blocks));
  const int64_t most = std::max<int64_t>(1, n / 2048);
  return (int)std::min(want, most);
}

// the sphered pair kernel with a single coefficient (LSCV_H, 4 < d <= 16)
void launch_md_one(hipStream_t s, int D, bool f64, const float* y32, const double* y64, int npad,
                   const MdState* st, const float* c32, const double* c64, const Unit* units, int u0, int cnt,
                   double* part, int n_items) {
  if (D <= 8)
    launch_md_units<8, 1>(s, f64, y32, y64, npad, st, c32, c64, units, u0, cnt, part, n_items, 1);
  else
    launch_md_units<16, 1>(s, f64, y32, y64, npad, st, c32, c64, units, u0, cnt, part, n_items, 1);
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// moments, covariance, Cholesky factor and whitened copy of the samples (the
// copy in the form's precision, dimension-major, npad samples a dimension)
void md_stage(hipStream_t st, const void* raw, bool raw_f64, int n, int d, int D, int npad, int nblk, double* ps,
              int* nf, double* pc, MdState* dst, float* y32, double* y64) {
  const int fx = raw_f64 ? 1 : 0;
  k_md_sum<<<nblk, kThreads, 0, st>>>(raw, fx, n, d, nblk, ps, nf);
  k_md_mean<<<1, 64, 0, st>>>(ps, nf, nblk, n, d, dst);
  k_md_cov<<<nblk, kThreads, 0, st>>>(raw, fx, n, d, nblk, dst, pc);
  k_md_factor<<<1, 64, 0, st>>>(pc, nblk, dst);
  k_md_whiten<<<(npad + kThreads - 1) / kThreads, kThreads, 0, st>>>(raw, fx, n, D, npad, dst, dst->linv, y32,
                                                                     y64);
}

}  // namespace

// Runs the whole d-dimensional LSCV pass; results in c->mdbuf (state, g, gs, h).
static kde_status run_md(kde_ctx* c, const kde_matrix& x, const double* h_grid, int32_t n_h, MdState* h_state,
                         std::vector<double>& g, std::vector<double>& gs, std::vector<double>& hv) {
  if (!x.data || x.n < 2 || x.n > KDE_MAX_N || x.d < 1 || x.d > KDE_MAX_D ||
      (x.dtype != KDE_F32 && x.dtype != KDE_F64))
    return fail(c, KDE_E_INVAL, "need a row-major n x d matrix, 2 <= n <= KDE_MAX_N, 1 <= d <= KDE_MAX_D");
  if (h_grid) {
    if (n_h < 1 || n_h > KDE_MAX_NH) return fail(c, KDE_E_INVAL, "grid size outside [1, KDE_MAX_NH]");
    for (int32_t k = 0; k < n_h; ++k)
      if (!(h_grid[k] > 0.0) || !std::isfinite(h_grid[k]) || (k > 0 && !(h_grid[k] > h_grid[k - 1])))
        return fail(c, KDE_E_INVAL, "grid values must be finite, > 0 and strictly ascending");
  } else {
    if (n_h <= 0) n_h = 150;
    if (n_h > KDE_MAX_NH) return fail(c, KDE_E_INVAL, "grid size above KDE_MAX_NH");
  }
  const bool f64 = c->prec == KDE_PREC_FP64;
  const int n = (int)x.n, d = x.d;
  const int D = md_width(d);
  const int hc = md_hc(D, f64);
  const int chunks = (n_h + hc - 1) / hc;
  const int m = chunks * hc;
  const int npad = n + kPad;
  const int esz = x.dtype == KDE_F64 ? 8 : 4;
  const int nblk = std::min(kMdBlocks, std::max(1, (n + 2047) / 2048));
  // work items as the univariate planner cuts the triangle
  ColItems items;
  make_items(n, capped_seg(c, n, kSegRefHC, (double)chunks), items);
  const int n_items = (int)items.pairs.size();
  std::vector<Unit> units;
  std::vector<double> cost;
  for (int it = 0; it < n_items; ++it)
    for (int ch = 0; ch < chunks; ++ch) {
      units.push_back(Unit{0, items.row[it], items.jb[it], items.je[it], it, ch});
      cost.push_back(items.pairs[it] * std::min(hc, n_h - ch * hc) * (1.0 + 2.0 * D / hc));
    }
  std::vector<RowDesc> rows;
  // device layout
  size_t at = 0;
  auto take = [&](size_t b) {
    const size_t o = at;
    at += al256(b);
    return o;
  };
  const size_t o_raw = x.on_device ? 0 : take((size_t)n * d * esz);
  const size_t o_ps = take(8 * (size_t)kMdBlocks * KDE_MAX_D), o_nf = take(4 * (size_t)kMdBlocks),
               o_pc = take(8 * (size_t)kMdBlocks * KDE_MAX_D * KDE_MAX_D), o_st = take(sizeof(MdState)),
               o_y32 = f64 ? 0 : take(4 * (size_t)D * npad), o_y64 = f64 ? take(8 * (size_t)D * npad) : 0,
               o_hin = take(8 * (size_t)n_h), o_h = take(8 * (size_t)m), o_c32 = take(4 * (size_t)m),
               o_c64 = take(8 * (size_t)m), o_part = take(16 * (size_t)n_h * n_items), o_sums = take(16 * (size_t)n_h),
               o_g = take(8 * (size_t)n_h), o_gs = take(8 * (size_t)n_h), o_units = take(sizeof(Unit) * units.size()),
               o_rows = take(sizeof(RowDesc) * 2 * (size_t)n_h);
  kde_status s;
  if ((s = ensure(c, c->mdbuf, at))) return s;
  char* b = c->mdbuf.p;
  const void* raw = x.on_device ? x.data : (const void*)(b + o_raw);
  double* part = (double*)(b + o_part);
  double* sums = (double*)(b + o_sums);
  for (int r = 0; r < 2 * n_h; ++r) rows.push_back(RowDesc{part + (size_t)r * n_items, sums + r, n_items, 0});
  hipStream_t st = c->stream;
  if (!x.on_device)
    KDE_HIP_TRY(c, hipMemcpyAsync(b + o_raw, x.data, (size_t)n * d * esz, hipMemcpyHostToDevice, st));
  if (h_grid) KDE_HIP_TRY(c, hipMemcpyAsync(b + o_hin, h_grid, 8 * (size_t)n_h, hipMemcpyHostToDevice, st));
  KDE_HIP_TRY(c, hipMemcpyAsync(b + o_units, units.data(), sizeof(Unit) * units.size(), hipMemcpyHostToDevice, st));
  KDE_HIP_TRY(c, hipMemcpyAsync(b + o_rows, rows.data(), sizeof(RowDesc) * rows.size(), hipMemcpyHostToDevice, st));
  MdState* dst = (MdState*)(b + o_st);
  float* y32 = f64 ? nullptr : (float*)(b + o_y32);
  double* y64 = f64 ? (double*)(b + o_y64) : nullptr;
  md_stage(st, raw, x.dtype == KDE_F64, n, d, D, npad, nblk, (double*)(b + o_ps), (int*)(b + o_nf),
           (double*)(b + o_pc), dst, y32, y64);
  k_md_prep<<<1, kThreads, 0, st>>>(dst, h_grid ? (const double*)(b + o_hin) : nullptr, n_h, m, (double*)(b + o_h),
                                     (float*)(b + o_c32), (double*)(b + o_c64));
  // launches of at most launch_evals pair-term evaluations and at least 2048 blocks
  const double budget = f64 ? c->opt_launch_evals / 5.0 : c->opt_launch_evals;
  for (size_t u0 = 0; u0 < units.size();) {
    double acc = cost[u0];
    size_t u1 = u0 + 1;
    while (u1 < units.size() && (acc + cost[u1] <= budget || u1 - u0 < 2048)) acc += cost[u1++];
    launch_md(st, D, f64, y32, y64, npad, dst, (const float*)(b + o_c32), (const double*)(b + o_c64),
              (const Unit*)(b + o_units), (int)u0, (int)(u1 - u0), part, n_items, n_h);
    u0 = u1;
  }
  launch_reduce_rows(st, (const RowDesc*)(b + o_rows), 2 * n_h);
  k_md_finalize<<<1, 1024, 0, st>>>(dst, sums, (const double*)(b + o_h), (const float*)(b + o_c32), f64 ? 1 : 0, n_h,
                                     (double*)(b + o_g), (double*)(b + o_gs));
  g.resize(n_h);
  gs.resize(n_h);
  hv.resize(n_h);
  KDE_HIP_TRY(c, hipMemcpyAsync(h_state, dst, sizeof(MdState), hipMemcpyDeviceToHost, st));
  KDE_HIP_TRY(c, hipMemcpyAsync(g.data(), b + o_g, 8 * (size_t)n_h, hipMemcpyDeviceToHost, st));
  KDE_HIP_TRY(c, hipMemcpyAsync(gs.data(), b + o_gs, 8 * (size_t)n_h, hipMemcpyDeviceToHost, st));
  KDE_HIP_TRY(c, hipMemcpyAsync(hv.data(), b + o_h, 8 * (size_t)n_h, hipMemcpyDeviceToHost, st));
  if ((s = sync_and_check(c))) return s;
  if (h_state->status == kStInval) return fail(c, KDE_E_INVAL, "sample matrix holds a non-finite value");
  if (h_state->status == kStDegenerate)
    return fail(c, KDE_E_DEGENERATE, "sample covariance is singular (collinear or constant samples)");
  return KDE_OK;
}


// ---- LSCV_H on the host side: staging once per call, then passes of at
// most kHPass matrices each (prep, pair units, row reduction, finalize).
namespace {

constexpr int kHPass = 64;

struct HRun {
  kde_ctx* c = nullptr;
  int n = 0, d = 0, D = 0, npad = 0, n_items = 0;
  bool f64 = false;
  bool one = false;           // d > kMaxHD: one matrix a sweep on re-whitened samples
  const void* raw = nullptr;  // the samples on the device
  bool raw_f64 = false;
  std::vector<double> pairs;  // per item
  char* b = nullptr;
  size_t o_st = 0, o_y32 = 0, o_y64 = 0, o_hin = 0, o_hd = 0, o_part = 0, o_sums = 0, o_g = 0, o_gs = 0,
         o_units = 0, o_rows = 0, o_hm = 0, o_coef = 0;
  MdState state{};
  int passes = 0;
  float coef32 = 0.f;  // host sources of the coefficient copies (live until the stage's sync)
  double coef64 = 0.0;
};

// Item length of an LSCV_H pass: about 8192 blocks for a single matrix
// (an explicit "seg" option wins).
int64_t h_seg(const kde_ctx* c, int64_t n) {
  if (c->opt_seg >= 0) return pick_seg(c, n, 1);
  int64_t seg = (int64_t)(0.5 * (double)n * (double)n / 8192.0 / kBI) / kBJ * kBJ;
  seg = std::max<int64_t>(kBJ, seg);
  return seg >= n ? 0 : seg;
}

kde_status h_stage(kde_ctx* c, const kde_matrix& x, HRun& r) {
  if (!x.data || x.n < 2 || x.n > KDE_MAX_N || x.d < 1 || x.d > KDE_MAX_D ||
      (x.dtype != KDE_F32 && x.dtype != KDE_F64))
    return fail(c, KDE_E_INVAL, "need a row-major n x d matrix, 2 <= n <= KDE_MAX_N, 1 <= d <= KDE_MAX_D");
  r.c = c;
  r.f64 = c->prec == KDE_PREC_FP64;
  r.n = (int)x.n;
  r.d = x.d;
  r.D = md_width(r.d);
  r.one = r.d > kMaxHD;
  r.npad = r.n + kPad;
  const int n = r.n, d = r.d, D = r.D;
  const int esz = x.dtype == KDE_F64 ? 8 : 4;
  const int nblk = std::min(kMdBlocks, std::max(1, (n + 2047) / 2048));
  ColItems items;
  make_items(n, h_seg(c, n), items);
  r.n_items = (int)items.pairs.size();
  r.pairs = items.pairs;
  // one unit per item; a pass's block index runs over chunk * n_items + item
  std::vector<Unit> units;
  units.reserve(r.n_items);
  for (int it = 0; it < r.n_items; ++it) units.push_back(Unit{0, items.row[it], items.jb[it], items.je[it], it, 0});
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t o = at;
    at += al256(bytes);
    return o;
  };
  const size_t o_raw = x.on_device ? 0 : take((size_t)n * d * esz);
  const size_t o_ps = take(8 * (size_t)kMdBlocks * KDE_MAX_D), o_nf = take(4 * (size_t)kMdBlocks),
               o_pc = take(8 * (size_t)kMdBlocks * KDE_MAX_D * KDE_MAX_D);
  r.o_st = take(sizeof(MdState));
  r.o_y32 = r.f64 ? 0 : take(4 * (size_t)D * r.npad);
  r.o_y64 = r.f64 ? take(8 * (size_t)D * r.npad) : 0;
  r.o_hin = take(8 * (size_t)kHPass * d * d);
  r.o_hd = take(sizeof(HDesc) * kHPass);
  r.o_part = take(16 * (size_t)kHPass * r.n_items);
  r.o_sums = take(16 * (size_t)kHPass);
  r.o_g = take(8 * (size_t)kHPass);
  r.o_gs = take(8 * (size_t)kHPass);
  r.o_units = take(sizeof(Unit) * units.size());
  r.o_rows = take(sizeof(RowDesc) * 2 * (size_t)kHPass);
  r.o_hm = r.one ? take(8 * (size_t)kHPass * KDE_MAX_D * KDE_MAX_D) : 0;
  r.o_coef = take(16);
  kde_status s;
  if ((s = ensure(c, c->mdbuf, at))) return s;
  char* b = r.b = c->mdbuf.p;
  double* part = (double*)(b + r.o_part);
  double* sums = (double*)(b + r.o_sums);
  std::vector<RowDesc> rows;
  for (int q = 0; q < 2 * kHPass; ++q) rows.push_back(RowDesc{part + (size_t)q * r.n_items, sums + q, r.n_items, 0});
  hipStream_t st = c->stream;
  const void* raw = r.raw = x.on_device ? x.data : (const void*)(b + o_raw);
  r.raw_f64 = x.dtype == KDE_F64;
  if (!x.on_device)
    KDE_HIP_TRY(c, hipMemcpyAsync(b + o_raw, x.data, (size_t)n * d * esz, hipMemcpyHostToDevice, st));
  // the single coefficient of the one-matrix sweep: -log2(e)/4 (FP32), -1/4 (FP64)
  r.coef32 = (float)(-kLog2ED * 0.25);
  r.coef64 = -0.25;
  KDE_HIP_TRY(c, hipMemcpyAsync(b + r.o_coef, &r.coef64, 8, hipMemcpyHostToDevice, st));
  KDE_HIP_TRY(c, hipMemcpyAsync(b + r.o_coef + 8, &r.coef32, 4, hipMemcpyHostToDevice, st));
  KDE_HIP_TRY(c, hipMemcpyAsync(b + r.o_units, units.data(), sizeof(Unit) * units.size(), hipMemcpyHostToDevice, st));
  KDE_HIP_TRY(c, hipMemcpyAsync(b + r.o_rows, rows.data(), sizeof(RowDesc) * rows.size(), hipMemcpyHostToDevice, st));
  MdState* dst = (MdState*)(b + r.o_st);
  md_stage(st, raw, x.dtype == KDE_F64, n, d, D, r.npad, nblk, (double*)(b + o_ps), (int*)(b + o_nf),
           (double*)(b + o_pc), dst, r.f64 ? nullptr : (float*)(b + r.o_y32),
           r.f64 ? (double*)(b + r.o_y64) : nullptr);
  KDE_HIP_TRY(c, hipMemcpyAsync(&r.state, dst, sizeof(MdState), hipMemcpyDeviceToHost, st));
  if ((s = sync_and_check(c))) return s;
  if (r.state.status == kStInval) return fail(c, KDE_E_INVAL, "sample matrix holds a non-finite value");
  if (r.state.status == kStDegenerate)
    return fail(c, KDE_E_DEGENERATE, "sample covariance is singular (collinear or constant samples)");
  return KDE_OK;
}

// g and its scale at m <= kHPass matrices (row-major d x d each)
kde_status h_pass(HRun& r, const double* H, int m, double* g, double* gs) {
  kde_ctx* c = r.c;
  hipStream_t st = c->stream;
  char* b = r.b;
  // matrices a block: as many as the pass has, up to 4 (8 for d <= 2, where
  // the shared per-pair work is a larger share of the cost)
  const int MH = m == 1 ? 1 : m == 2 ? 2 : (r.D == 2 && m >= 8) ? 8 : 4;
  const int chunks = (m + MH - 1) / MH;
  const MdState* dst = (const MdState*)(b + r.o_st);
  const HDesc* hd = (const HDesc*)(b + r.o_hd);
  double* part = (double*)(b + r.o_part);
  KDE_HIP_TRY(c, hipMemcpyAsync(b + r.o_hin, H, 8 * (size_t)m * r.d * r.d, hipMemcpyHostToDevice, st));
  // launches of at most launch_evals pair-term evaluations and at least 2048 blocks
  const double budget = r.f64 ? c->opt_launch_evals / 5.0 : c->opt_launch_evals;
  if (r.one) {
    const double* hm = (const double*)(b + r.o_hm);
    k_HT_prep<<<1, kHPass, 0, st>>>(dst, (const double*)(b + r.o_hin), m, (HDesc*)(b + r.o_hd), (double*)hm);
    float* z32 = r.f64 ? nullptr : (float*)(b + r.o_y32);
    double* z64 = r.f64 ? (double*)(b + r.o_y64) : nullptr;
    for (int k = 0; k < m; ++k) {
      k_md_whiten<<<(r.npad + kThreads - 1) / kThreads, kThreads, 0, st>>>(
          r.raw, r.raw_f64 ? 1 : 0, r.n, r.D, r.npad, dst, hm + (size_t)k * KDE_MAX_D * KDE_MAX_D, z32, z64);
      for (size_t u0 = 0; u0 < (size_t)r.n_items;) {
        double acc = r.pairs[u0];
        size_t u1 = u0 + 1;
        while (u1 < (size_t)r.n_items && (acc + r.pairs[u1] <= budget || u1 - u0 < 2048)) acc += r.pairs[u1++];
        launch_md_one(st, r.D, r.f64, z32, z64, r.npad, dst, (const float*)(b + r.o_coef + 8),
                      (const double*)(b + r.o_coef), (const Unit*)(b + r.o_units), (int)u0, (int)(u1 - u0),
                      part + (size_t)2 * k * r.n_items, r.n_items);
        u0 = u1;
      }
    }
  } else {
    k_H_prep<<<1, kHPass, 0, st>>>(dst, (const double*)(b + r.o_hin), m, r.D, r.f64 ? 1 : 0, (HDesc*)(b + r.o_hd));
  }
  const size_t total = r.one ? 0 : (size_t)chunks * r.n_items;
  for (size_t u0 = 0; u0 < total;) {
    double acc = r.pairs[u0 % r.n_items] * MH;
    size_t u1 = u0 + 1;
    while (u1 < total && (acc + r.pairs[u1 % r.n_items] * MH <= budget || u1 - u0 < 2048))
      acc += r.pairs[u1++ % r.n_items] * MH;
    launch_H(st, r.D, MH, r.f64, (const float*)(b + r.o_y32), (const double*)(b + r.o_y64), r.npad, dst, hd, m,
             (const Unit*)(b + r.o_units), (int)u0, (int)(u1 - u0), part, r.n_items);
    u0 = u1;
  }
  launch_reduce_rows(st, (const RowDesc*)(b + r.o_rows), 2 * m);
  k_H_final<<<1, kHPass, 0, st>>>(dst, hd, m, r.f64 ? 1 : 0, (const double*)(b + r.o_sums), (double*)(b + r.o_g),
                                  (double*)(b + r.o_gs));
  KDE_HIP_TRY(c, hipMemcpyAsync(g, b + r.o_g, 8 * (size_t)m, hipMemcpyDeviceToHost, st));
  KDE_HIP_TRY(c, hipMemcpyAsync(gs, b + r.o_gs, 8 * (size_t)m, hipMemcpyDeviceToHost, st));
  ++r.passes;
  return sync_and_check(c);
}

kde_status h_eval(HRun& r, const double* H, int m, double* g, double* gs) {
  std::vector<double> scratch(kHPass);
  for (int k0 = 0; k0 < m; k0 += kHPass) {
    const int mm = std::min(kHPass, m - k0);
    kde_status s = h_pass(r, H + (size_t)k0 * r.d * r.d, mm, g + k0, gs ? gs + k0 : scratch.data());
    if (s) return s;
  }
  return KDE_OK;
}

// H = C C^T from theta: the lower triangle of C row by row, the logarithm of
// each diagonal entry in place of the entry
void theta_to_H(const double* th, int d, double* H) {
  double C[KDE_MAX_D][KDE_MAX_D] = {};
  int p = 0;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b, ++p) C[a][b] = (a == b) ? std::exp(th[p]) : th[p];
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double s = 0.0;
      for (int k = 0; k < d; ++k) s += C[a][k] * C[b][k];
      H[a * d + b] = s;
    }
}

// Nelder-Mead over theta (Section 4.4.3 names the method).  Start: the
// rule-of-thumb matrix s^2 Sigma, s = (4/(d+2))^(1/(d+4)) n^(-1/(d+4)); initial
// steps 0.25 on the log-diagonal and 0.25 sqrt(C_aa C_bb) off it; reflection
// 1, expansion 2, inside and outside contraction 1/2, shrink 1/2 towards the
// best vertex; stop once max g - min g over the simplex is at most
// ftol |min g| and every vertex lies within xtol of the best in every
// parameter, or after max_evals evaluations.  Vertices are kept ordered by g
// with a stable insertion sort.
kde_status h_search(HRun& r, double ftol, double xtol, int max_evals, double* H_out, kde_lscv_H_info* info) {
  const int d = r.d, p = d * (d + 1) / 2;
  kde_ctx* c = r.c;
  // Cholesky factor of s^2 Sigma
  const double sc = std::pow(4.0 / (d + 2.0), 1.0 / (d + 4.0)) * std::pow((double)r.n, -1.0 / (d + 4.0));
  double S[KDE_MAX_D][KDE_MAX_D], Ls[KDE_MAX_D][KDE_MAX_D] = {};
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) S[a][b] = r.state.sigma[a * KDE_MAX_D + b] * sc * sc;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b) {
      double s = S[a][b];
      for (int k = 0; k < b; ++k) s -= Ls[a][k] * Ls[b][k];
      if (a == b) {
        if (!(s > 1e-12 * S[a][a]) || !std::isfinite(s))
          return fail(c, KDE_E_DEGENERATE, "sample covariance is singular (collinear or constant samples)");
        Ls[a][a] = std::sqrt(s);
      } else {
        Ls[a][b] = s / Ls[b][b];
      }
    }
  std::vector<double> V((size_t)(p + 1) * p), F(p + 1), Hb((size_t)(p + 1) * d * d), gsb(p + 1);
  {
    int q = 0;
    for (int a = 0; a < d; ++a)
      for (int b = 0; b <= a; ++b, ++q) V[q] = (a == b) ? std::log(Ls[a][a]) : Ls[a][b];
    q = 0;
    for (int a = 0; a < d; ++a)
      for (int b = 0; b <= a; ++b, ++q) {
        double* v = &V[(size_t)(q + 1) * p];
        std::copy(V.begin(), V.begin() + p, v);
        v[q] += (a == b) ? 0.25 : 0.25 * std::sqrt(Ls[a][a] * Ls[b][b]);
      }
  }
  int evals = 0;
  auto eval = [&](const double* th, int k, double* f) -> kde_status {
    for (int t = 0; t < k; ++t) theta_to_H(th + (size_t)t * p, d, &Hb[(size_t)t * d * d]);
    kde_status s = h_eval(r, Hb.data(), k, f, gsb.data());
    evals += k;
    return s;
  };
  kde_status s;
  if ((s = eval(V.data(), p + 1, F.data()))) return s;
  std::vector<double> cen(p), xr(p), xe(p), xc(p);
  bool converged = false;
  for (;;) {
    for (int i = 1; i <= p; ++i)
      for (int j = i; j > 0 && F[j] < F[j - 1]; --j) {
        std::swap(F[j], F[j - 1]);
        std::swap_ranges(V.begin() + (size_t)j * p, V.begin() + (size_t)(j + 1) * p, V.begin() + (size_t)(j - 1) * p);
      }
    double spread = 0.0;
    for (int i = 1; i <= p; ++i)
      for (int j = 0; j < p; ++j) spread = std::max(spread, std::fabs(V[(size_t)i * p + j] - V[j]));
    if (F[p] - F[0] <= ftol * std::fabs(F[0]) && spread <= xtol) {
      converged = true;
      break;
    }
    if (evals >= max_evals) break;
    double* worst = &V[(size_t)p * p];
    for (int j = 0; j < p; ++j) {
      double t = 0.0;
      for (int i = 0; i < p; ++i) t += V[(size_t)i * p + j];
      cen[j] = t / (double)p;
    }
    for (int j = 0; j < p; ++j) xr[j] = cen[j] + (cen[j] - worst[j]);
    double fr, fe, fc;
    if ((s = eval(xr.data(), 1, &fr))) return s;
    bool shrink = false;
    if (fr < F[0]) {
      for (int j = 0; j < p; ++j) xe[j] = cen[j] + 2.0 * (cen[j] - worst[j]);
      if ((s = eval(xe.data(), 1, &fe))) return s;
      const bool take_e = fe < fr;
      std::copy_n(take_e ? xe.data() : xr.data(), p, worst);
      F[p] = take_e ? fe : fr;
    } else if (fr < F[p - 1]) {
      std::copy_n(xr.data(), p, worst);
      F[p] = fr;
    } else if (fr < F[p]) {  // outside contraction
      for (int j = 0; j < p; ++j) xc[j] = cen[j] + 0.5 * (xr[j] - cen[j]);
      if ((s = eval(xc.data(), 1, &fc))) return s;
      if (fc <= fr) {
        std::copy_n(xc.data(), p, worst);
        F[p] = fc;
      } else {
        shrink = true;
      }
    } else {  // inside contraction
      for (int j = 0; j < p; ++j) xc[j] = cen[j] + 0.5 * (worst[j] - cen[j]);
      if ((s = eval(xc.data(), 1, &fc))) return s;
      if (fc < F[p]) {
        std::copy_n(xc.data(), p, worst);
        F[p] = fc;
      } else {
        shrink = true;
      }
    }
    if (shrink) {
      for (int i = 1; i <= p; ++i)
        for (int j = 0; j < p; ++j) V[(size_t)i * p + j] = V[j] + 0.5 * (V[(size_t)i * p + j] - V[j]);
      if ((s = eval(&V[p], p, &F[1]))) return s;
    }
  }
  theta_to_H(V.data(), d, H_out);
  if (info) {
    info->g = F[0];
    info->evals = evals;
    info->passes = r.passes;
    info->converged = converged ? 1 : 0;
    info->pad0 = 0;
  }
  return KDE_OK;
}

}  // namespace


// ---- consumers for d-dimensional samples (host side)
namespace {

bool finite_span(const double* v, int64_t k) {
  for (int64_t i = 0; i < k; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

kde_status check_matrix(kde_ctx* c, const kde_matrix& x, int d_lo, int d_hi) {
  if (!x.data || x.n < 1 || x.n > KDE_MAX_N || x.d < d_lo || x.d > d_hi ||
      (x.dtype != KDE_F32 && x.dtype != KDE_F64))
    return fail(c, KDE_E_INVAL, "bad sample matrix (n >= 1, d in range, float32 or float64)");
  return KDE_OK;
}

}  // namespace

static kde_status run_density_H(kde_ctx* c, const kde_matrix& x, const double* H, const double* points, int32_t m,
                                double* f_out) {
  kde_status s;
  if ((s = check_matrix(c, x, 1, KDE_MAX_D))) return s;
  const int n = (int)x.n, d = x.d, D = md_width(d);
  if (m < 1 || m > KDE_MAX_QUERIES) return fail(c, KDE_E_INVAL, "query count outside [1, KDE_MAX_QUERIES]");
  if (!finite_span(H, (int64_t)d * d) || !finite_span(points, (int64_t)m * d))
    return fail(c, KDE_E_INVAL, "bandwidth matrix and query points must be finite");
  const bool f64 = c->prec == KDE_PREC_FP64;
  const int esz = x.dtype == KDE_F64 ? 8 : 4;
  const int npad = n + kPad, mpad = m + kPad;
  const int nblk = std::min(kMdBlocks, std::max(1, (n + 2047) / 2048));
  const int qblocks = (m + kThreads - 1) / kThreads;
  int pieces = dq_pieces(n, qblocks);
  int piece_len = (n + pieces - 1) / pieces;
  piece_len = (piece_len + kThreads - 1) / kThreads * kThreads;
  pieces = (n + piece_len - 1) / piece_len;
  size_t at = 0;
  auto take = [&](size_t b) {
    const size_t o = at;
    at += al256(b);
    return o;
  };
  const size_t o_raw = x.on_device ? 0 : take((size_t)n * d * esz);
  const size_t o_ps = take(8 * (size_t)kMdBlocks * KDE_MAX_D), o_nf = take(4 * (size_t)kMdBlocks),
               o_st = take(sizeof(MdState)), o_H = take(8 * (size_t)d * d), o_y = take(8 * (size_t)D * npad),
               o_qr = take(8 * (size_t)m * d), o_zq = take(8 * (size_t)D * mpad),
               o_part = take(8 * (size_t)m * pieces), o_out = take(8 * (size_t)m);
  if ((s = ensure(c, c->mdbuf, at))) return s;
  char* b = c->mdbuf.p;
  hipStream_t st = c->stream;
  const void* raw = x.on_device ? x.data : (const void*)(b + o_raw);
  if (!x.on_device)
    KDE_HIP_TRY(c, hipMemcpyAsync(b + o_raw, x.data, (size_t)n * d * esz, hipMemcpyHostToDevice, st));
  KDE_HIP_TRY(c, hipMemcpyAsync(b + o_H, H, 8 * (size_t)d * d, hipMemcpyHostToDevice, st));
  KDE_HIP_TRY(c, hipMemcpyAsync(b + o_qr, points, 8 * (size_t)m * d, hipMemcpyHostToDevice, st));
  MdState* dst = (MdState*)(b + o_st);
  const int fx = x.dtype == KDE_F64 ? 1 : 0;
  k_md_sum<<<nblk, kThreads, 0, st>>>(raw, fx, n, d, nblk, (double*)(b + o_ps), (int*)(b + o_nf));
  k_md_mean<<<1, 64, 0, st>>>((const double*)(b + o_ps), (const int*)(b + o_nf), nblk, n, d, dst);
  k_dq_factor<<<1, 64, 0, st>>>(dst, (const double*)(b + o_H));
  double* y = (double*)(b + o_y);
  double* zq = (double*)(b + o_zq);
  k_md_whiten<<<(npad + kThreads - 1) / kThreads, kThreads, 0, st>>>(raw, fx, n, D, npad, dst, dst->linv, nullptr,
                                                                     y);
  k_md_whiten<<<(mpad + kThreads - 1) / kThreads, kThreads, 0, st>>>(b + o_qr, 1, m, D, mpad, dst, dst->linv,
                                                                     nullptr, zq);
  const dim3 grid(qblocks, pieces);
  double* part = (double*)(b + o_part);
  switch (D) {
    case 2: launch_dq<2>(st, f64, grid, zq, m, mpad, y, npad, dst, piece_len, pieces, part); break;
    case 3: launch_dq<3>(st, f64, grid, zq, m, mpad, y, npad, dst, piece_len, pieces, part); break;
    case 4: launch_dq<4>(st, f64, grid, zq, m, mpad, y, npad, dst, piece_len, pieces, part); break;
    case 8: launch_dq<8>(st, f64, grid, zq, m, mpad, y, npad, dst, piece_len, pieces, part); break;
    default: launch_dq<16>(st, f64, grid, zq, m, mpad, y, npad, dst, piece_len, pieces, part); break;
  }
  k_dq_final<<<qblocks, kThreads, 0, st>>>(dst, part, m, pieces, (double*)(b + o_out));
  MdState hs;
  KDE_HIP_TRY(c, hipMemcpyAsync(&hs, dst, sizeof(MdState), hipMemcpyDeviceToHost, st));
  KDE_HIP_TRY(c, hipMemcpyAsync(f_out, b + o_out, 8 * (size_t)m, hipMemcpyDeviceToHost, st));
  if ((s = sync_and_check(c))) return s;
  if (hs.status == kStInval) return fail(c, KDE_E_INVAL, "sample matrix holds a non-finite value");
  if (hs.status == kStDegenerate)
    return fail(c, KDE_E_DEGENERATE, "bandwidth matrix is not positive definite");
  return KDE_OK;
}

static kde_status run_range_2d(kde_ctx* c, const kde_matrix& x, const double* H, const double* boxes, int32_t q,
                               std::vector<double>& out) {
  kde_status s;
  if ((s = check_matrix(c, x, 2, 2))) return s;
  if (q < 1 || q > KDE_MAX_QUERIES) return fail(c, KDE_E_INVAL, "box count outside [1, KDE_MAX_QUERIES]");
  if (!finite_span(H, 4)) return fail(c, KDE_E_INVAL, "bandwidth matrix must be finite");
  for (int32_t k = 0; k < q; ++k) {
    const double* bx = boxes + 4 * (size_t)k;
    if (std::isnan(bx[0]) || std::isnan(bx[1]) || std::isnan(bx[2]) || std::isnan(bx[3]) || !(bx[0] <= bx[1]) ||
        !(bx[2] <= bx[3]))
      return fail(c, KDE_E_INVAL, "every box needs lo <= hi in both coordinates (infinite ends allowed)");
  }
  // positive definite by the library's pivot rule: H11 > 0, H22 - H21^2/H11 > 1e-12 H22
  if (!(H[0] > 0.0) || !(H[3] - H[2] * H[2] / H[0] > 1e-12 * H[3]))
    return fail(c, KDE_E_DEGENERATE, "bandwidth matrix is not positive definite");
  const int n = (int)x.n;
  const int esz = x.dtype == KDE_F64 ? 8 : 4;
  const int nblk = std::min(kMdBlocks, std::max(1, (n + 2047) / 2048));
  int pieces = dq_pieces(n, q);
  const int piece_len = (n + pieces - 1) / pieces;
  pieces = (n + piece_len - 1) / piece_len;
  size_t at = 0;
  auto take = [&](size_t b) {
    const size_t o = at;
    at += al256(b);
    return o;
  };
  const size_t o_raw = x.on_device ? 0 : take((size_t)n * 2 * esz);
  const size_t o_ps = take(8 * (size_t)kMdBlocks * KDE_MAX_D), o_nf = take(4 * (size_t)kMdBlocks),
               o_st = take(sizeof(MdState)), o_bx = take(32 * (size_t)q), o_part = take(24 * (size_t)q * pieces),
               o_out = take(40 * (size_t)q);
  if ((s = ensure(c, c->mdbuf, at))) return s;
  char* b = c->mdbuf.p;
  hipStream_t st = c->stream;
  const void* raw = x.on_device ? x.data : (const void*)(b + o_raw);
  if (!x.on_device)
    KDE_HIP_TRY(c, hipMemcpyAsync(b + o_raw, x.data, (size_t)n * 2 * esz, hipMemcpyHostToDevice, st));
  KDE_HIP_TRY(c, hipMemcpyAsync(b + o_bx, boxes, 32 * (size_t)q, hipMemcpyHostToDevice, st));
  MdState* dst = (MdState*)(b + o_st);
  const int fx = x.dtype == KDE_F64 ? 1 : 0;
  k_md_sum<<<nblk, kThreads, 0, st>>>(raw, fx, n, 2, nblk, (double*)(b + o_ps), (int*)(b + o_nf));
  k_md_mean<<<1, 64, 0, st>>>((const double*)(b + o_ps), (const int*)(b + o_nf), nblk, n, 2, dst);
  k_r2_units<<<dim3(q, pieces), kThreads, 0, st>>>(raw, fx, dst, H[0], H[2], H[3], (const double*)(b + o_bx),
                                                    piece_len, pieces, (double*)(b + o_part));
  k_r2_final<<<q, kThreads, 0, st>>>(dst, (const double*)(b + o_part), pieces, (double*)(b + o_out));
  out.resize(5 * (size_t)q);
  MdState hs;
  KDE_HIP_TRY(c, hipMemcpyAsync(&hs, dst, sizeof(MdState), hipMemcpyDeviceToHost, st));
  KDE_HIP_TRY(c, hipMemcpyAsync(out.data(), b + o_out, 40 * (size_t)q, hipMemcpyDeviceToHost, st));
  if ((s = sync_and_check(c))) return s;
  if (hs.status == kStInval) return fail(c, KDE_E_INVAL, "sample matrix holds a non-finite value");
  return KDE_OK;
}

}  // namespace kde

extern "C" {

kde_status kde_lscv_md_curve(kde_ctx* c, kde_matrix x, const double* h_grid, int32_t n_h, double* g_out,
                             double* gscale_out, double* grid_out) {
  if (!c || !g_out) return KDE_E_INVAL;
  if (c->server && kde::server_running(c->server.get())) return kde::fail(c, KDE_E_BUSY, "a server is running");
  if (hipSetDevice(c->device) != hipSuccess) return kde::fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde::MdState h;
  std::vector<double> g, gs, hv;
  kde_status s = kde::run_md(c, x, h_grid, n_h, &h, g, gs, hv);
  if (s) return s;
  std::memcpy(g_out, g.data(), 8 * g.size());
  if (gscale_out) std::memcpy(gscale_out, gs.data(), 8 * gs.size());
  if (grid_out) std::memcpy(grid_out, hv.data(), 8 * hv.size());
  return KDE_OK;
}

kde_status kde_bw_lscv_md(kde_ctx* c, kde_matrix x, const double* h_grid, int32_t n_h, double* h_out,
                          int32_t* k_out) {
  if (!c || !h_out) return KDE_E_INVAL;
  if (c->server && kde::server_running(c->server.get())) return kde::fail(c, KDE_E_BUSY, "a server is running");
  if (hipSetDevice(c->device) != hipSuccess) return kde::fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde::MdState h;
  std::vector<double> g, gs, hv;
  kde_status s = kde::run_md(c, x, h_grid, n_h, &h, g, gs, hv);
  if (s) return s;
  *h_out = h.h_best;
  if (k_out) *k_out = h.k_best;
  return KDE_OK;
}

kde_status kde_lscv_H_eval(kde_ctx* c, kde_matrix x, const double* H, int32_t m, double* g_out,
                           double* gscale_out) {
  if (!c || !g_out || !H) return KDE_E_INVAL;
  if (c->server && kde::server_running(c->server.get())) return kde::fail(c, KDE_E_BUSY, "a server is running");
  if (m < 1 || m > KDE_MAX_H_EVAL) return kde::fail(c, KDE_E_INVAL, "matrix count outside [1, KDE_MAX_H_EVAL]");
  if (x.d >= 1 && x.d <= KDE_MAX_D)
    for (int64_t q = 0; q < (int64_t)m * x.d * x.d; ++q)
      if (!std::isfinite(H[q])) return kde::fail(c, KDE_E_INVAL, "bandwidth matrix holds a non-finite value");
  if (hipSetDevice(c->device) != hipSuccess) return kde::fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde::HRun r;
  kde_status s = kde::h_stage(c, x, r);
  if (s) return s;
  return kde::h_eval(r, H, m, g_out, gscale_out);
}

kde_status kde_bw_lscv_H(kde_ctx* c, kde_matrix x, double ftol, double xtol, int32_t max_evals, double* H_out,
                         kde_lscv_H_info* info) {
  if (!c || !H_out) return KDE_E_INVAL;
  if (c->server && kde::server_running(c->server.get())) return kde::fail(c, KDE_E_BUSY, "a server is running");
  if (!(ftol > 0.0) || !(xtol > 0.0) || !std::isfinite(ftol) || !std::isfinite(xtol) || max_evals < 1)
    return kde::fail(c, KDE_E_INVAL, "need ftol > 0, xtol > 0 and max_evals >= 1");
  if (hipSetDevice(c->device) != hipSuccess) return kde::fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde::HRun r;
  kde_status s = kde::h_stage(c, x, r);
  if (s) return s;
  return kde::h_search(r, ftol, xtol, max_evals, H_out, info);
}

kde_status kde_density_H(kde_ctx* c, kde_matrix x, const double* H, const double* points, int32_t m,
                         double* f_out) {
  if (!c || !H || !points || !f_out) return KDE_E_INVAL;
  if (c->server && kde::server_running(c->server.get())) return kde::fail(c, KDE_E_BUSY, "a server is running");
  if (hipSetDevice(c->device) != hipSuccess) return kde::fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  return kde::run_density_H(c, x, H, points, m, f_out);
}

kde_status kde_range_aggregates_2d(kde_ctx* c, kde_matrix x, const double* H, const double* boxes, int32_t q,
                                   double* count_out, double* sumx_out, double* sumy_out, double* avgx_out,
                                   double* avgy_out) {
  if (!c || !H || !boxes || !count_out || !sumx_out || !sumy_out) return KDE_E_INVAL;
  if (c->server && kde::server_running(c->server.get())) return kde::fail(c, KDE_E_BUSY, "a server is running");
  if (hipSetDevice(c->device) != hipSuccess) return kde::fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  std::vector<double> out;
  kde_status s = kde::run_range_2d(c, x, H, boxes, q, out);
  if (s) return s;
  for (int32_t k = 0; k < q; ++k) {
    count_out[k] = out[5 * (size_t)k];
    sumx_out[k] = out[5 * (size_t)k + 1];
    sumy_out[k] = out[5 * (size_t)k + 2];
    if (avgx_out) avgx_out[k] = out[5 * (size_t)k + 3];
    if (avgy_out) avgy_out[k] = out[5 * (size_t)k + 4];
  }
  return KDE_OK;
}

}  // extern "C"
