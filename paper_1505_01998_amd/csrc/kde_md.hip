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

#include "kde_md.h"

namespace kde {

namespace {

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

// md_run for wide samples (D = 8, 16): the j coordinates are the same for
// every lane of a wave, so they are read with uniform addresses (scalar loads
// through the scalar cache) instead of from an LDS tile
template <int D, int HC, bool MASK>
__device__ __forceinline__ void md_run_s(const float* __restrict__ y, int npad, int jg, const float (&yi)[D],
                                         int i, const float (&ck)[HC], float (&a1)[HC], float (&c1)[HC],
                                         float (&a2)[HC], float (&c2)[HC]) {
  float r1[HC], r2[HC];
#pragma unroll
  for (int k = 0; k < HC; ++k) r1[k] = r2[k] = 0.f;
#pragma unroll 2
  for (int q = 0; q < kMdRun; ++q) {
    float s = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const float dd = yi[a] - y[(int64_t)a * npad + jg + q];
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
  __shared__ double red[4][2 * HC];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = u.row * kBI;
  const int i = row0 + tid;
  float yi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) yi[a] = (i < n) ? y[(int64_t)a * npad + i] : 0.f;
  const int wave_i0 = __builtin_amdgcn_readfirstlane(row0 + wave * 64);
  float ck[HC], a1[HC], c1[HC], a2[HC], c2[HC];
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    ck[k] = c32[u.chunk * HC + k];
    a1[k] = c1[k] = a2[k] = c2[k] = 0.f;
  }
  if constexpr (D >= 8) {
    // wide samples: D tile reads a pair would limit the sweep; read the j
    // coordinates with uniform addresses instead (no tile, no barrier)
    int js = __builtin_amdgcn_readfirstlane(max(u.j_begin, wave_i0));
    const int je = __builtin_amdgcn_readfirstlane(u.j_end);
    if (js < je && js == wave_i0) {
      md_run_s<D, HC, true>(y, npad, js, yi, i, ck, a1, c1, a2, c2);
      js += kMdRun;
    }
    for (; js < je; js += kMdRun) md_run_s<D, HC, false>(y, npad, js, yi, i, ck, a1, c1, a2, c2);
  } else {
    __shared__ float tile[D][kBJ];
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
        const double e = exp_cw(s * ck[k]);
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

template <int D, int HC>
void launch_md_units(hipStream_t s, bool f64, const float* y32, const double* y64, int npad, const MdState* st,
                     const float* c32, const double* c64, const Unit* units, int u0, int cnt, double* part,
                     int n_items, int n_h) {
  if (f64)
    k_md_units_f64<D, HC><<<cnt, kThreads, 0, s>>>(y64, npad, st, c64, units, u0, part, n_items, n_h);
  else
    k_md_units_f32<D, HC><<<cnt, kThreads, 0, s>>>(y32, npad, st, c32, units, u0, part, n_items, n_h);
}

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


}  // namespace

int md_width(int d) { return d <= 2 ? 2 : d <= 3 ? 3 : d <= 4 ? 4 : d <= 8 ? 8 : 16; }

void md_moments(hipStream_t st, const void* raw, bool raw_f64, int n, int d, int nblk, double* ps, int* nf,
                MdState* dst) {
  k_md_sum<<<nblk, kThreads, 0, st>>>(raw, raw_f64 ? 1 : 0, n, d, nblk, ps, nf);
  k_md_mean<<<1, 64, 0, st>>>(ps, nf, nblk, n, d, dst);
}

void md_whiten(hipStream_t st, const void* raw, bool raw_f64, int n, int D, int npad, const MdState* dst,
               const double* M, float* y32, double* y64) {
  k_md_whiten<<<(npad + kThreads - 1) / kThreads, kThreads, 0, st>>>(raw, raw_f64 ? 1 : 0, n, D, npad, dst, M, y32,
                                                                     y64);
}

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
  std::vector<double> cost, ev;  // planning cost, pair-term evaluations
  for (int it = 0; it < n_items; ++it)
    for (int ch = 0; ch < chunks; ++ch) {
      units.push_back(Unit{0, items.row[it], items.jb[it], items.je[it], it, ch});
      cost.push_back(items.pairs[it] * std::min(hc, n_h - ch * hc) * (1.0 + 2.0 * D / hc));
      ev.push_back(items.pairs[it] * std::min(hc, n_h - ch * hc));
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
    kde_ctx::Pending pd{nullptr, nullptr, kFamMd, 0.0};
    for (size_t u = u0; u < u1; ++u) pd.evals += ev[u];
    if ((s = timed_begin(c, pd))) return s;
    launch_md(st, D, f64, y32, y64, npad, dst, (const float*)(b + o_c32), (const double*)(b + o_c64),
              (const Unit*)(b + o_units), (int)u0, (int)(u1 - u0), part, n_items, n_h);
    if ((s = timed_end(c, pd))) return s;
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


}  // extern "C"
