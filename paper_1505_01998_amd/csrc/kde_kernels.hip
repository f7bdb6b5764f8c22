// kde_kernels.hip -- gfx950 kernels for exact bandwidth-selection pair sums.
//
// Method: Andrzejewski, Gramacki, Gramacki, arXiv 1505.01998, Section 4.4
// (selectors), Section 4.5 (pair distance reused across bandwidths) and
// Section 5.4 (sums of a function of X_i - X_j over the i < j triangle).
//
// Jobs.  Every call works on a set of columns (one for the single-column
// selectors, many for a batch).  Column descriptors (ColDesc) say where each
// column's samples, grid coefficients and partial sums live; every pair
// kernel block decodes one work unit (Unit: column, row of samples i, j-range,
// bandwidth chunk), so units of different columns share a launch.
//
// Pair kernels.  A block of 256 threads (four 64-wide waves) owns a "row" of
// 256 consecutive samples i, one per lane, held in a register for the whole
// block.  The block sweeps a j-range of the triangle in tiles of kBJ samples
// that are staged in LDS with coalesced 16-byte loads; every lane of a wave
// reads the same LDS address (a broadcast), so each wave walks j in lockstep
// against its 64 register-resident i.  Because j is wave-uniform, loop bounds
// are uniform and nothing diverges; the only masking is the 64x64 diagonal
// block of each wave, where pairs with j <= i are given an infinite squared
// distance (exp2(-inf) = 0 exactly).  Padded samples beyond n hold +inf and
// contribute exactly zero the same way; padded lanes (i >= n) are dropped
// when the block's partial sums are formed.
//
// Precision (mixed form).  Pair terms are FP32 (v_exp_f32).  Each lane sums
// 64 consecutive j in plain FP32, then folds that run into an FP64
// accumulator (the LSCV sweep: a conversion and an FP64 add, which issue at
// the unpacked FP32 rate, half the cost of a compensated FP32 fold) or a
// Kahan-compensated FP32 one (the psi pass, two sums per 64 pairs).  Lane
// accumulators are reduced in FP64 across the wave (butterfly shuffles), the
// block (LDS, fixed order) and the work items (a separate row-reduction
// kernel, fixed order), so the result is deterministic and independent of
// scheduling.  The FP64 form
// computes every term and sum in FP64.
#include <hip/hip_runtime.h>
#include <math.h>

#include "kde_internal.h"

namespace kde {

namespace {

constexpr float kInfF = __builtin_inff();
constexpr double kInfD = __builtin_inf();
constexpr double kPi = 3.14159265358979323846;
constexpr double kLog2E = 1.4426950408889634074;
constexpr int kRun = 64;  // j per plain-FP32 run before a compensated fold
// Squared scaled distance beyond which a psi term is zero in FP32; clamping
// keeps the Hermite polynomial finite when the distance is huge or infinite.
constexpr float kWMax = 4096.0f;
// A column whose scaled copy (samples / g) spans at most this range has every
// squared scaled distance below 4e8, where He_8 stays far inside the FP32
// range, so its psi sweep needs no clamp except on masked and padded pairs.
constexpr double kPsiFastRange = 2.0e4;
// exp2 factor of the psi term: e^(-w/2) = exp2(w * kPsiExp2)
constexpr float kPsiExp2 = (float)(-0.5 * 1.4426950408889634074);

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// Block-wide minimum and maximum (every thread receives both).
__device__ __forceinline__ void block_minmax(float& lo, float& hi, float* sh) {
  const int t = threadIdx.x;
  sh[t] = lo;
  sh[kThreads + t] = hi;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (t < s) {
      sh[t] = fminf(sh[t], sh[t + s]);
      sh[kThreads + t] = fmaxf(sh[kThreads + t], sh[kThreads + t + s]);
    }
    __syncthreads();
  }
  lo = sh[0];
  hi = sh[kThreads];
  __syncthreads();
}

// A wave-uniform float kept in a scalar register: the bandwidth coefficients
// of the LSCV sweeps are the same for every lane, and holding them in SGPRs
// instead of VGPRs frees HC vector registers per lane (more waves per SIMD).
__device__ __forceinline__ float uniform_f32(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Kahan fold of a run sum r into (acc, comp); the compensated value is acc - comp.
__device__ __forceinline__ void kahan_add(float& acc, float& comp, float r) {
  const float y = r - comp;
  const float t = acc + y;
  comp = (t - acc) - y;
  acc = t;
}

// Probabilists' Hermite polynomial He_r(u) as a polynomial in w = u^2.
template <int R>
__device__ __forceinline__ float herm_w(float w);
template <>
__device__ __forceinline__ float herm_w<4>(float w) {
  return __builtin_fmaf(w - 6.0f, w, 3.0f);
}
template <>
__device__ __forceinline__ float herm_w<6>(float w) {
  float p = __builtin_fmaf(w - 15.0f, w, 45.0f);
  return __builtin_fmaf(p, w, -15.0f);
}
template <>
__device__ __forceinline__ float herm_w<8>(float w) {
  float p = __builtin_fmaf(w - 28.0f, w, 210.0f);
  p = __builtin_fmaf(p, w, -420.0f);
  return __builtin_fmaf(p, w, 105.0f);
}
template <int R>
__device__ __forceinline__ double herm_w64(double w);
template <>
__device__ __forceinline__ double herm_w64<4>(double w) {
  return __builtin_fma(w - 6.0, w, 3.0);
}
template <>
__device__ __forceinline__ double herm_w64<6>(double w) {
  double p = __builtin_fma(w - 15.0, w, 45.0);
  return __builtin_fma(p, w, -15.0);
}
template <>
__device__ __forceinline__ double herm_w64<8>(double w) {
  double p = __builtin_fma(w - 28.0, w, 210.0);
  p = __builtin_fma(p, w, -420.0);
  return __builtin_fma(p, w, 105.0);
}

// He_r(0) = (-1)^(r/2) (r-1)!! for even r, from the recurrence
// He_{k+1}(0) = -k He_{k-1}(0) with He_0(0) = 1: the kernel-derivative value
// K^(r)(0) = He_r(0) / sqrt(2 pi) (r = 4, 6, 8) and the normal-scale
// functionals below (r = 8, 10).
__device__ __forceinline__ double herm_at0(int r) {
  double h = 1.0;
  for (int k = 1; k < r; k += 2) h *= -(double)k;
  return h;
}

// Normal-scale functional psi_r of N(0, sigma^2): the integral of f^(r) f
// for the normal density is He_r(0) / (2^(r/2+1) sqrt(pi) sigma^(r+1)) (the
// convolution of two N(0, sigma^2) densities is N(0, 2 sigma^2), whose r-th
// derivative at 0 is He_r(0) / (sqrt(2 pi) (sqrt(2) sigma)^(r+1))); r = 8
// gives the printed 105 / (32 sqrt(pi) sigma^9).
__device__ double psi_normal_scale(int r, double sigma) {
  return herm_at0(r) / (ldexp(1.0, r / 2 + 1) * sqrt(kPi) * pow(sigma, (double)(r + 1)));
}

// ------------------------------------------------------------------ statistics
__device__ __forceinline__ double load_raw(const ColDesc& c, int i) {
  return c.raw_f64 ? reinterpret_cast<const double*>(c.raw)[i] : (double)reinterpret_cast<const float*>(c.raw)[i];
}

__device__ __forceinline__ int stat_blocks(int n) { return min(kStatBlocks, (n + 2047) / 2048); }

// Pass 1: per-block FP64 sum of the samples and count of non-finite values.
// Grid (max blocks, columns).
__global__ __launch_bounds__(kThreads) void k_stats_sum(const ColDesc* __restrict__ cols, const int* __restrict__ ids) {
  const ColDesc c = cols[ids[blockIdx.y]];
  const int nblk = stat_blocks(c.n);
  if ((int)blockIdx.x >= nblk) return;
  __shared__ double sh[kThreads];
  __shared__ int nf_sh;
  const int chunk = (c.n + nblk - 1) / nblk;
  const int b0 = blockIdx.x * chunk;
  const int b1 = min(c.n, b0 + chunk);
  if (threadIdx.x == 0) nf_sh = 0;
  __syncthreads();
  double s = 0.0;
  int nf = 0;
  for (int i = b0 + threadIdx.x; i < b1; i += kThreads) {
    const double v = load_raw(c, i);
    if (!isfinite(v)) ++nf; else s += v;
  }
  if (nf) atomicAdd(&nf_sh, nf);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    c.stat[blockIdx.x] = s;
    c.stat_nf[blockIdx.x] = nf_sh;
  }
}

// Mean of each column (block per column); float64 columns are shifted by it.
__global__ __launch_bounds__(kThreads) void k_stats_mean(const ColDesc* __restrict__ cols,
                                                         const int* __restrict__ ids) {
  const ColDesc c = cols[ids[blockIdx.x]];
  const int nblk = stat_blocks(c.n);
  __shared__ double sh[kThreads];
  __shared__ int nf_sh;
  if (threadIdx.x == 0) nf_sh = 0;
  __syncthreads();
  double s = 0.0;
  int nf = 0;
  for (int b = threadIdx.x; b < nblk; b += kThreads) {
    s += c.stat[b];
    nf += c.stat_nf[b];
  }
  if (nf) atomicAdd(&nf_sh, nf);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    DevState& d = *c.st;
    d.n = (double)c.n;
    d.status = nf_sh ? kStInval : kStOk;
    d.mean = s / (double)c.n;
    d.shift = c.raw_f64 ? d.mean : 0.0;
  }
}

// Pass 2: per-block sum of squared deviations; writes the padded FP32 (and
// FP64) working copies of the column.
__global__ __launch_bounds__(kThreads) void k_stats_dev(const ColDesc* __restrict__ cols, const int* __restrict__ ids) {
  const ColDesc c = cols[ids[blockIdx.y]];
  const int nblk = stat_blocks(c.n);
  if ((int)blockIdx.x >= nblk) return;
  __shared__ double sh[kThreads];
  const double mean = c.st->mean, shift = c.st->shift;
  float* y32 = c.x32;
  double* y64 = c.x64;
  const int chunk = (c.n + nblk - 1) / nblk;
  const int b0 = blockIdx.x * chunk;
  const int b1 = min(c.n, b0 + chunk);
  __shared__ float shm[2 * kThreads];
  double s = 0.0;
  float lo = kInfF, hi = -kInfF;
  for (int i = b0 + threadIdx.x; i < b1; i += kThreads) {
    const double v = load_raw(c, i);
    const double d = v - mean;
    s += d * d;
    const float w = (float)(v - shift);
    y32[i] = w;
    lo = fminf(lo, w);
    hi = fmaxf(hi, w);
    if (y64) y64[i] = v;
  }
  for (int i = c.n + blockIdx.x * kThreads + threadIdx.x; i < c.n + kPad; i += nblk * kThreads) {
    y32[i] = kInfF;
    if (y64) y64[i] = kInfD;
  }
  s = block_sum(s, sh);
  block_minmax(lo, hi, shm);
  if (threadIdx.x == 0) {
    c.stat[blockIdx.x] = s;
    c.stat_mm[blockIdx.x] = lo;
    c.stat_mm[kStatBlocks + blockIdx.x] = hi;
  }
}

__global__ __launch_bounds__(kThreads) void k_stats_final(const ColDesc* __restrict__ cols,
                                                          const int* __restrict__ ids) {
  const ColDesc c = cols[ids[blockIdx.x]];
  const int nblk = stat_blocks(c.n);
  __shared__ double sh[kThreads];
  __shared__ float shm[2 * kThreads];
  double s = 0.0;
  float lo = kInfF, hi = -kInfF;
  for (int b = threadIdx.x; b < nblk; b += kThreads) {
    s += c.stat[b];
    lo = fminf(lo, c.stat_mm[b]);
    hi = fmaxf(hi, c.stat_mm[kStatBlocks + b]);
  }
  s = block_sum(s, sh);
  block_minmax(lo, hi, shm);
  if (threadIdx.x == 0) {
    DevState& d = *c.st;
    d.xmin = lo;
    d.xmax = hi;
    const double n = d.n;
    d.var = s / (n - 1.0);
    d.sigma = sqrt(d.var);
    // normal-reference rule: (4/3)^(1/5) sigma n^(-1/5)
    d.h_rot = pow(4.0 / 3.0, 0.2) * pow(n, -0.2) * d.sigma;
    if (d.status == kStOk && !(d.sigma > 0.0 && isfinite(d.sigma))) d.status = kStDegenerate;
  }
}

// ------------------------------------------------------------------ plug-in scalar steps
// One thread per column.  Stage s in {0, 1, 2} estimates psi_r, r = 8 - 2 s.
__global__ void k_psi_begin(const ColDesc* __restrict__ cols, const int* __restrict__ ids, int n_ids, int stage) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_ids) return;
  DevState& d = *cols[ids[k]].st;
  d.active = 0;
  d.need_f64 = 0;
  if (d.status != kStOk || d.pstatus != kStOk || d.stages == 0) return;
  if (stage == 0 && d.stages != 3) return;
  const int r = 8 - 2 * stage;
  double psi_next;
  if (stage == 0) {
    psi_next = psi_normal_scale(10, d.sigma);
  } else if (stage == 1) {
    if (d.stages == 2) d.psi[0] = psi_normal_scale(8, d.sigma);
    psi_next = d.psi[0];
  } else {
    psi_next = d.psi[1];
  }
  // AMSE pilot: g = [-2 K^(r)(0) / (mu_2 psi_{r+2} n)]^(1/(r+3)), mu_2 = 1
  const double k0 = herm_at0(r) / sqrt(2.0 * kPi);
  const double rad = -2.0 * k0 / (psi_next * d.n);
  if (!(rad > 0.0) || !isfinite(rad)) {
    d.pstatus = kStDegenerate;
    return;
  }
  const double g = pow(rad, 1.0 / (double)(r + 3));
  d.active = 1;
  d.g[stage] = g;
  const double ig2 = 1.0 / (g * g);
  d.psi_scale = (float)(1.0 / g);
  d.psi_fast = ((double)d.xmax - (double)d.xmin) * (double)d.psi_scale <= kPsiFastRange ? 1 : 0;
  d.cd[0] = ig2;
  d.cd[1] = -0.5 * ig2;
}

// Scaled copy of the mixed form's psi pass: y = x32 * (1/g) in FP32 (padding
// stays +inf).  Grid (blocks, columns); inactive columns are skipped.
__global__ __launch_bounds__(kThreads) void k_psi_scale(const ColDesc* __restrict__ cols,
                                                        const int* __restrict__ ids) {
  const ColDesc c = cols[ids[blockIdx.y]];
  if (!c.st->active) return;
  const float s = c.st->psi_scale;
  const int m = c.n + kPad;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < m; i += gridDim.x * kThreads)
    c.y32[i] = i < c.n ? c.x32[i] * s : kInfF;
}

// psi_sums[0] = sum_{i<j} He_r(u) e^{-u^2/2}, psi_sums[1] = sum of its
// absolute value, u = (X_i - X_j)/g.  psi_r = [2 sum K^(r) + n K^(r)(0)] / (n^2 g^(r+1)).
// conditional: this is the FP64 re-run of the mixed form; skip unless flagged.
__global__ void k_psi_finish(const ColDesc* __restrict__ cols, const int* __restrict__ ids, int n_ids, int stage,
                             int was_f64, int conditional) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_ids) return;
  const ColDesc& c = cols[ids[k]];
  DevState& d = *c.st;
  const double* sums = c.psi_sums;
  if (!d.active) return;
  if (conditional && !d.need_f64) return;
  const int r = 8 - 2 * stage;
  const double inv_s2pi = 1.0 / sqrt(2.0 * kPi);
  const double n = d.n, g = d.g[stage];
  const double s = sums[0] * inv_s2pi, a = sums[1] * inv_s2pi;
  d.psi[stage] = (2.0 * s + n * herm_at0(r) * inv_s2pi) / (n * n * pow(g, (double)(r + 1)));
  d.kappa[stage] = (s != 0.0) ? a / fabs(s) : kInfD;
  d.prec_used[stage] = was_f64 ? 1 : 0;
  if (was_f64) {
    d.need_f64 = 0;
  } else {
    d.need_f64 = (d.fp64_kappa > 0.0 && d.kappa[stage] > d.fp64_kappa) ? 1 : 0;
  }
}

__global__ void k_plugin_final(const ColDesc* __restrict__ cols, const int* __restrict__ ids, int n_ids) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_ids) return;
  DevState& d = *cols[ids[k]].st;
  if (d.status != kStOk || d.pstatus != kStOk || d.stages == 0) return;
  // h = [R(K) / (mu_2^2 psi_4 n)]^(1/5), R(K) = 1/(2 sqrt(pi))
  const double rad = (0.5 / sqrt(kPi)) / (d.psi[2] * d.n);
  if (!(rad > 0.0) || !isfinite(rad)) {
    d.pstatus = kStDegenerate;
    return;
  }
  d.h_plugin = pow(rad, 0.2);
}

// ------------------------------------------------------------------ psi pair kernels
// Mixed form.  The samples are pre-scaled by 1/g (y = x / g, one O(n) pass
// per stage), so a pair's w = u^2 = (y_i - y_j)^2 needs no per-pair scaling;
// the term He_r(u) e^(-u^2/2) is formed as He_r in w (Horner, the integer
// coefficients exact in FP32) times exp2(w * kPsiExp2), and both the term
// and its absolute value are accumulated by one fma each (|He_r| as a source
// modifier).  Per pair: sub, mul, mul, exp2, r/2 Horner ops, 2 fma.
// MASK (a wave's diagonal run): pairs with j <= i get w = kWMax, whose
// exponential is exactly 0 and whose He_r is finite.  CLAMP (padded tiles,
// or a column whose scaled range could overflow He_r): w = min(w, kWMax),
// so an infinite or huge distance also gives exactly 0.
template <int R, bool MASK, bool CLAMP>
__device__ __forceinline__ void psi_run(const float4* __restrict__ tile, int jl, int jg, float yi, int i, float& aS,
                                        float& cS, float& aA, float& cA) {
  float rs = 0.f, ra = 0.f;
#pragma unroll 4
  for (int q = 0; q < kRun / 4; ++q) {
    const float4 v = tile[(jl >> 2) + q];
    const float ys[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float d = yi - ys[u];
      float w = d * d;
      if (CLAMP) w = fminf(w, kWMax);
      if (MASK) w = (jg + 4 * q + u > i) ? w : kWMax;
      // issue priority raised from the exponential to its two consumers,
      // as in the LSCV sweep (order of issue only; +29% on this pass)
      __builtin_amdgcn_s_setprio(1);
      const float e = __builtin_amdgcn_exp2f(w * kPsiExp2);
      const float hw = herm_w<R>(w);
      rs = __builtin_fmaf(hw, e, rs);
      ra = __builtin_fmaf(fabsf(hw), e, ra);
      __builtin_amdgcn_s_setprio(0);
    }
  }
  kahan_add(aS, cS, rs);
  kahan_add(aA, cA, ra);
}


template <int R>
__global__ __launch_bounds__(kThreads) void k_psi_units_f32(const ColDesc* __restrict__ cols,
                                                            const Unit* __restrict__ units, int u0) {
  const Unit u = units[u0 + blockIdx.x];
  const ColDesc c = cols[u.col];
  if (!c.st->active) return;
  const float* y = c.y32;
  const int n = c.n;
  const bool fast = c.st->psi_fast != 0;
  __shared__ float4 tile[kBJ / 4];
  __shared__ double red[2][4];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = u.row * kBI;
  const int i = row0 + tid;
  const float yi = (i < n) ? y[i] : 0.f;
  const int wave_i0 = row0 + wave * 64;
  float aS = 0.f, cS = 0.f, aA = 0.f, cA = 0.f;
  for (int t0 = u.j_begin; t0 < u.j_end; t0 += kBJ) {
    __syncthreads();
    for (int q = tid; q < kBJ / 4; q += kThreads) tile[q] = reinterpret_cast<const float4*>(y + t0)[q];
    __syncthreads();
    int js = max(t0, wave_i0);
    const int te = t0 + kBJ;
    if (js < te) {
      const bool clamp = !fast || te > n;  // uniform: padded tile or unsafe range
      if (js == wave_i0) {
        if (clamp)
          psi_run<R, true, true>(tile, js - t0, js, yi, i, aS, cS, aA, cA);
        else
          psi_run<R, true, false>(tile, js - t0, js, yi, i, aS, cS, aA, cA);
        js += kRun;
      }
      if (clamp) {
        for (; js < te; js += kRun) psi_run<R, false, true>(tile, js - t0, js, yi, i, aS, cS, aA, cA);
      } else {
        for (; js < te; js += kRun) psi_run<R, false, false>(tile, js - t0, js, yi, i, aS, cS, aA, cA);
      }
    }
  }
  const bool valid = i < n;
  double vs = valid ? (double)aS - (double)cS : 0.0;
  double va = valid ? (double)aA - (double)cA : 0.0;
  vs = wave_sum(vs);
  va = wave_sum(va);
  if (lane == 0) {
    red[0][wave] = vs;
    red[1][wave] = va;
  }
  __syncthreads();
  if (tid < 2)
    c.psi_part[(int64_t)tid * c.n_items_psi + u.item] = ((red[tid][0] + red[tid][1]) + red[tid][2]) + red[tid][3];
}

template <int R, bool MASK>
__device__ __forceinline__ void psi_run64(const double* __restrict__ tile, int jl, int jg, double xi, int i,
                                          double ig2, double cg, double& s, double& a) {
#pragma unroll 4
  for (int q = 0; q < kRun; ++q) {
    const double d = xi - tile[jl + q];
    double t = d * d;
    if (MASK) t = (jg + q > i) ? t : kInfD;
    const double w = fmin(t * ig2, (double)kWMax);
    const double term = herm_w64<R>(w) * exp_cw(t * cg);
    s += term;
    a += fabs(term);
  }
}

// conditional: run only when the FP32 pass flagged this column's stage (mixed form).
template <int R>
__global__ __launch_bounds__(kThreads) void k_psi_units_f64(const ColDesc* __restrict__ cols,
                                                            const Unit* __restrict__ units, int u0,
                                                            int conditional) {
  const Unit u = units[u0 + blockIdx.x];
  const ColDesc c = cols[u.col];
  if (!c.st->active) return;
  if (conditional && !c.st->need_f64) return;
  const double* x = c.x64;
  const int n = c.n;
  __shared__ double tile[kBJ];
  __shared__ double red[2][4];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = u.row * kBI;
  const int i = row0 + tid;
  const double xi = (i < n) ? x[i] : 0.0;
  const int wave_i0 = row0 + wave * 64;
  const double ig2 = c.st->cd[0], cg = c.st->cd[1];
  double s = 0.0, a = 0.0;
  for (int t0 = u.j_begin; t0 < u.j_end; t0 += kBJ) {
    __syncthreads();
    for (int q = tid; q < kBJ / 2; q += kThreads)
      reinterpret_cast<double2*>(tile)[q] = reinterpret_cast<const double2*>(x + t0)[q];
    __syncthreads();
    int js = max(t0, wave_i0);
    const int te = t0 + kBJ;
    if (js < te) {
      if (js == wave_i0) {
        psi_run64<R, true>(tile, js - t0, js, xi, i, ig2, cg, s, a);
        js += kRun;
      }
      for (; js < te; js += kRun) psi_run64<R, false>(tile, js - t0, js, xi, i, ig2, cg, s, a);
    }
  }
  const bool valid = i < n;
  double vs = wave_sum(valid ? s : 0.0);
  double va = wave_sum(valid ? a : 0.0);
  if (lane == 0) {
    red[0][wave] = vs;
    red[1][wave] = va;
  }
  __syncthreads();
  if (tid < 2)
    c.psi_part[(int64_t)tid * c.n_items_psi + u.item] = ((red[tid][0] + red[tid][1]) + red[tid][2]) + red[tid][3];
}

// ------------------------------------------------------------------ LSCV kernels
// Block per column.  Grid point k of the column: explicit h_in[k], the
// paper's default (linear over sigma [h0/4, 4 h0] = h_rot [1/4, 4]) or log-spaced
// over h_rot [lo, hi].  c32 = -log2(e) / (4 h^2), so exp2(D^2 c32) =
// exp(-D^2/(4 h^2)) and its square is exp(-D^2/(2 h^2)); c64 = -1/(4 h^2).
// Entries past n_h up to the chunk multiple hold -1 (finite, unused).
__global__ __launch_bounds__(kThreads) void k_lscv_prep(const ColDesc* __restrict__ cols,
                                                        const int* __restrict__ ids, int hc) {
  const ColDesc c = cols[ids[blockIdx.x]];
  if (c.n_h <= 0) return;
  const double hr = c.st->h_rot;
  const int m = c.n_chunks * hc;
  for (int k = threadIdx.x; k < m; k += kThreads) {
    const int o = k;
    if (k < c.n_h) {
      double h;
      const double t = (c.n_h == 1) ? 0.0 : (double)k / (double)(c.n_h - 1);
      if (c.grid_kind == kGridExplicit)
        h = c.h_in[o];
      else if (c.grid_kind == kGridPaper)
        h = hr * 0.25 + (hr * 4.0 - hr * 0.25) * t;
      else
        h = hr * exp(log(c.grid_lo) + (log(c.grid_hi) - log(c.grid_lo)) * t);
      c.h[o] = h;
      const double q = 1.0 / (4.0 * h * h);
      c.c32[o] = (float)(-kLog2E * q);
      c.c64[o] = -q;
    } else {
      c.h[o] = 0.0;
      c.c32[o] = -1.0f;
      c.c64[o] = -1.0;
    }
  }
}

// Four consecutive j of a run (one float4 of the LDS tile) against the
// lane's sample, for the HC bandwidths.  FIRST: the run's first pair starts
// the plain sums (S1 = e, S2 = e e instead of adding them to zero: the same
// values, as e is never -0), which saves clearing 2 HC registers per run.
template <int HC, bool MASK, bool FIRST>
__device__ __forceinline__ void lscv_quad(const float4 v, int jg, float xi, int i, const float (&ck)[HC],
                                          float (&r1)[HC], float (&r2)[HC]) {
  const float xs[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const float d = xi - xs[u];
    float t = d * d;
    if (MASK) t = (jg + u > i) ? t : kInfF;
    // One term at a time, in program order: mul, exp2, then its two
    // consumers.  A wave then holds one exponential in flight and waits on
    // it while the SIMD's other waves issue plain instructions; measured on
    // gfx950 this overlaps more of the transcendental unit's time than
    // exponentials issued back to back (the compiler's own order, which
    // also pairs them at pair boundaries): +1% at HC = 16, +13% at HC = 8.
    // The wave raises its issue priority from the exponential until both
    // consumers have issued, so that a wave whose exponential has completed
    // goes ahead of waves starting a new term: +8% at HC = 16, +10% at
    // HC = 8.  The barrier and the priority only fix the order of issue;
    // the arithmetic and the summation order are unchanged.
#pragma unroll
    for (int k = 0; k < HC; ++k) {
      __builtin_amdgcn_s_setprio(1);
      const float e = __builtin_amdgcn_exp2f(t * ck[k]);
      if (FIRST && u == 0) {
        r1[k] = e;
        r2[k] = e * e;
      } else {
        r1[k] += e;
        r2[k] = __builtin_fmaf(e, e, r2[k]);
      }
      __builtin_amdgcn_s_setprio(0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <int HC, bool MASK>
__device__ __forceinline__ void lscv_run(const float4* __restrict__ tile, int jl, int jg, float xi, int i,
                                         const float (&ck)[HC], double (&a1)[HC], double (&a2)[HC]) {
  float r1[HC], r2[HC];
  lscv_quad<HC, MASK, true>(tile[jl >> 2], jg, xi, i, ck, r1, r2);
#pragma unroll 3
  for (int q = 1; q < kRun / 4; ++q) lscv_quad<HC, MASK, false>(tile[(jl >> 2) + q], jg + 4 * q, xi, i, ck, r1, r2);
  // the run's sums into the lane's FP64 accumulators
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    a1[k] += (double)r1[k];
    a2[k] += (double)r2[k];
  }
}

// One LSCV work unit of the vector-ALU sweep: the unit's row of 256 samples
// i against its j-range, for the HC bandwidths of its chunk; the block's
// FP64 partial sums go to the unit's own slots.  TJ: samples per LDS tile
// (256, 512 or 1024; a unit's j-range is a multiple of 512, so a 1024 tile
// may end half full).  The tile size changes only how often the block stages
// and synchronises: every lane still folds its terms in runs of 64 j in
// ascending j order, so every (unit, h) sum is bitwise the same for all TJ.
template <int HC, int TJ>
__device__ __forceinline__ void lscv_unit_f32(const ColDesc* __restrict__ cols, const Unit& u, float4* tile,
                                              double (*red)[2 * HC]) {
  const ColDesc c = cols[u.col];
  if (c.st->status != kStOk) return;  // uniform over the block
  const float* x = c.x32;
  const int n = c.n;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = u.row * kBI;
  const int i = row0 + tid;
  const float xi = (i < n) ? x[i] : 0.f;
  const int wave_i0 = row0 + wave * 64;
  const float* cc = c.c32 + u.chunk * HC;
  float ck[HC];
  double a1[HC], a2[HC];
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    ck[k] = uniform_f32(cc[k]);
    a1[k] = a2[k] = 0.0;
  }
  for (int t0 = u.j_begin; t0 < u.j_end; t0 += TJ) {
    const int te = min(t0 + TJ, u.j_end);
    __syncthreads();
    for (int q = tid; q < (te - t0) / 4; q += kThreads) tile[q] = reinterpret_cast<const float4*>(x + t0)[q];
    __syncthreads();
    int js = max(t0, wave_i0);
    if (js < te) {
      if (js == wave_i0) {
        lscv_run<HC, true>(tile, js - t0, js, xi, i, ck, a1, a2);
        js += kRun;
      }
      for (; js < te; js += kRun) lscv_run<HC, false>(tile, js - t0, js, xi, i, ck, a1, a2);
    }
  }
  const bool valid = i < n;
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    const double v1 = wave_sum(valid ? a1[k] : 0.0);
    const double v2 = wave_sum(valid ? a2[k] : 0.0);
    if (lane == 0) {
      red[wave][2 * k] = v1;
      red[wave][2 * k + 1] = v2;
    }
  }
  __syncthreads();
  if (tid < 2 * HC) {
    const int h = u.chunk * HC + (tid >> 1);
    if (h < c.n_h) {
      const double v = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
      c.part[(int64_t)(2 * h + (tid & 1)) * c.n_items + u.item] = v;
    }
  }
}

template <int HC>
__global__ __launch_bounds__(kThreads) void k_lscv_units_f32(const ColDesc* __restrict__ cols,
                                                             const Unit* __restrict__ units, int u0) {
  __shared__ float4 tile[kBJ / 4];
  __shared__ double red[4][2 * HC];
  lscv_unit_f32<HC, kBJ>(cols, units[u0 + blockIdx.x], tile, red);
}

// Persistent form: a grid of about as many blocks as the chip holds at once
// takes the pass's units from device counters, one unit per block at a time,
// until the list is exhausted.  The list comes in kQueueGroups groups of
// about equal work, each a contiguous stretch of (column, j) positions kept
// largest first; group g is units [group_begin[g], group_begin[g + 1]) with
// counter next[g].  Block b starts on group b % kQueueGroups (workgroups are
// dealt round-robin to the eight dies, so a die's blocks stream the sample
// tiles of one stretch of the column, which stays in that die's L2), and
// when its group is drained it moves on to the next ones, taking what is
// left there.  A block leaves a group once its counter passes the group's
// end, so every block reaches the end of the last group and exits.  One
// launch covers a whole pass; the longest units start first wherever a
// block frees up.  next[0 .. kQueueGroups) must be 0 at launch.
template <int HC, int TJ>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(HC <= 16 ? 4 : 2))) void
k_lscv_units_f32_queue(const ColDesc* __restrict__ cols, const Unit* __restrict__ units,
                       const int* __restrict__ group_begin, int* __restrict__ next) {
  __shared__ float4 tile[TJ / 4];
  __shared__ double red[4][2 * HC];
  __shared__ int cur;
  const int g0 = (int)(blockIdx.x % kQueueGroups);
  for (int q = 0; q < kQueueGroups; ++q) {
    const int g = (g0 + q) % kQueueGroups;
    const int base = group_begin[g], len = group_begin[g + 1] - base;
    for (;;) {
      if (threadIdx.x == 0) cur = atomicAdd(next + g, 1);
      __syncthreads();
      const int k = __builtin_amdgcn_readfirstlane(cur);  // uniform: unit and column loads stay scalar
      __syncthreads();
      if (k >= len) break;
      lscv_unit_f32<HC, TJ>(cols, units[base + k], tile, red);
    }
  }
}

// Clears n ints (the work counters of a pass) with a kernel, so the pass
// stays replayable from a graph.
__global__ void k_zero_ints(int* __restrict__ p, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0;
}

// Ceiling of the sweep's inner loop on the part: lscv_run<HC, false> over one
// LDS tile of kBJ samples staged once, `reps` times per block, with no further
// staging, barriers, masks or partial-sum writes (each wave stores one sum so
// that nothing is dropped).  Evaluations per launch:
// blocks x kThreads x reps x kBJ x HC.
template <int HC>
__global__ __launch_bounds__(kThreads) void k_lscv_ceiling(const float* __restrict__ x, const float* __restrict__ c32,
                                                           int reps, double* __restrict__ out) {
  __shared__ float4 tile[kBJ / 4];
  const int tid = threadIdx.x;
  for (int q = tid; q < kBJ / 4; q += kThreads) tile[q] = reinterpret_cast<const float4*>(x)[q];
  __syncthreads();
  const float xi = x[tid] + 0.5f;
  float ck[HC];
  double a1[HC], a2[HC];
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    ck[k] = uniform_f32(c32[k]);
    a1[k] = a2[k] = 0.0;
  }
  for (int r = 0; r < reps; ++r)
    for (int js = 0; js < kBJ; js += kRun) lscv_run<HC, false>(tile, js, js, xi, 0, ck, a1, a2);
  double v = 0.0;
#pragma unroll
  for (int k = 0; k < HC; ++k) v += (a1[k]) + (a2[k]);
  v = wave_sum(v);
  if ((tid & 63) == 0) out[(int64_t)blockIdx.x * (kThreads / 64) + (tid >> 6)] = v;
}

// Tile pruning on sorted samples: the same sweep over a column sorted
// ascending, whose j-tiles therefore lie at growing distance from the unit's
// row of i.  A uniform scan of the tiles' first samples finds the first tile
// whose smallest distance to the row exceeds the chunk's cut (every later
// tile is farther still); the sweep stops there and the skipped pairs are
// counted exactly.
template <int HC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(HC <= 16 ? 4 : 2)))
void k_lscv_units_prune(const ColDesc* __restrict__ cols, const Unit* __restrict__ units, int u0) {
  const Unit u = units[u0 + blockIdx.x];
  const ColDesc c = cols[u.col];
  if (c.st->status != kStOk) return;
  const float* x = c.x32;
  const int n = c.n;
  const int row0 = u.row * kBI;
  int j_end = u.j_end;
  {
    const float row_max = x[min(row0 + kBI, n) - 1];
    const float cut = c.d2cut[u.chunk];
    for (int t = u.j_begin; t < u.j_end; t += kBJ) {
      const float dd = x[t] - row_max;
      if (dd > 0.f && dd * dd > cut) {
        j_end = t;
        break;
      }
    }
  }
  __shared__ float4 tile[kBJ / 4];
  __shared__ double red[4][2 * HC];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i = row0 + tid;
  const float xi = (i < n) ? x[i] : 0.f;
  const int wave_i0 = row0 + wave * 64;
  const float* cc = c.c32 + u.chunk * HC;
  float ck[HC];
  double a1[HC], a2[HC];
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    ck[k] = uniform_f32(cc[k]);
    a1[k] = a2[k] = 0.0;
  }
  for (int t0 = u.j_begin; t0 < j_end; t0 += kBJ) {
    __syncthreads();
    for (int q = tid; q < kBJ / 4; q += kThreads) tile[q] = reinterpret_cast<const float4*>(x + t0)[q];
    __syncthreads();
    int js = max(t0, wave_i0);
    const int te = t0 + kBJ;
    if (js < te) {
      if (js == wave_i0) {
        lscv_run<HC, true>(tile, js - t0, js, xi, i, ck, a1, a2);
        js += kRun;
      }
      for (; js < te; js += kRun) lscv_run<HC, false>(tile, js - t0, js, xi, i, ck, a1, a2);
    }
  }
  if (tid == 0 && j_end < u.j_end && j_end < n) {
    // every skipped tile lies right of the row (distance > 0): all its pairs count
    const double rows = (double)min(kBI, n - row0);
    const double hv = (double)min(HC, c.n_h - u.chunk * HC);
    atomicAdd(&c.st->pruned_evals, rows * (double)(min(u.j_end, n) - j_end) * hv);
  }
  const bool valid = i < n;
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    const double v1 = wave_sum(valid ? a1[k] : 0.0);
    const double v2 = wave_sum(valid ? a2[k] : 0.0);
    if (lane == 0) {
      red[wave][2 * k] = v1;
      red[wave][2 * k + 1] = v2;
    }
  }
  __syncthreads();
  if (tid < 2 * HC) {
    const int h = u.chunk * HC + (tid >> 1);
    if (h < c.n_h) {
      const double v = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
      c.part[(int64_t)(2 * h + (tid & 1)) * c.n_items + u.item] = v;
    }
  }
}

// Tile pruning (mixed form, sorted column): per bandwidth chunk the squared
// distance D2 beyond which a 256 x 512 tile is skipped.  A skipped tile holds
// at most 2^17 pairs, each term at most exp2(c_max D^2) (c_max: the chunk's
// coefficient closest to zero, i.e. its largest h) for S1 and its square for
// S2.  With T an upper bound on the (row, tile) pairs of the column and L1,
// L2 the smallest near-tile sums (lower bounds of S1, S2: all terms are
// positive) over the chunk's bandwidths, a tile is skipped only when 2^17
// exp2(c_max D^2) < eps L1 / T and 2^17 exp2(2 c_max D^2) < eps L2 / T, so
// everything skipped is below eps S1(h) and eps S2(h) for every h of the
// chunk.
__global__ __launch_bounds__(kThreads) void k_lscv_prune_prep(const ColDesc* __restrict__ cols,
                                                              const int* __restrict__ ids, int hc, double eps) {
  const ColDesc c = cols[ids[blockIdx.x]];
  if (c.n_h <= 0 || c.st->status != kStOk) return;
  const double n = (double)c.n;
  const double rows = ceil(n / kBI);
  const double T = rows * (ceil(n / kBJ) + 1.0);
  const double lt = log2(eps / (T * (double)kBI * (double)kBJ));
  for (int ch = threadIdx.x; ch < c.n_chunks; ch += blockDim.x) {
    double l1 = kInfD, l2 = kInfD, cmax = -kInfD;
    for (int k = ch * hc; k < min(c.n_h, (ch + 1) * hc); ++k) {
      l1 = fmin(l1, c.near_sums[2 * k]);
      l2 = fmin(l2, c.near_sums[2 * k + 1]);
      cmax = fmax(cmax, (double)c.c32[k]);
    }
    double cut = kInfD;
    if (l1 > 0.0 && l2 > 0.0 && cmax < 0.0) {
      const double d1 = (lt + log2(l1)) / cmax;
      const double d2 = (lt + log2(l2)) / (2.0 * cmax);
      cut = fmax(d1, d2) * (1.0 + 1e-6) + 1e-30;
    }
    c.d2cut[ch] = (float)cut;
  }
}

template <int HC, bool MASK>
__device__ __forceinline__ void lscv_run64(const double* __restrict__ tile, int jl, int jg, double xi, int i,
                                           const double (&ck)[HC], double (&s1)[HC], double (&s2)[HC]) {
#pragma unroll 2
  for (int q = 0; q < kRun; ++q) {
    const double d = xi - tile[jl + q];
    double t = d * d;
    if (MASK) t = (jg + q > i) ? t : kInfD;
#pragma unroll
    for (int k = 0; k < HC; ++k) {
      const double e = exp_cw(t * ck[k]);
      s1[k] += e;
      s2[k] = __builtin_fma(e, e, s2[k]);
    }
  }
}

template <int HC>
__global__ __launch_bounds__(kThreads) void k_lscv_units_f64(const ColDesc* __restrict__ cols,
                                                             const Unit* __restrict__ units, int u0) {
  const Unit u = units[u0 + blockIdx.x];
  const ColDesc c = cols[u.col];
  if (c.st->status != kStOk) return;
  const double* x = c.x64;
  const int n = c.n;
  __shared__ double tile[kBJ];
  __shared__ double red[4][2 * HC];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = u.row * kBI;
  const int i = row0 + tid;
  const double xi = (i < n) ? x[i] : 0.0;
  const int wave_i0 = row0 + wave * 64;
  const double* cc = c.c64 + u.chunk * HC;
  double ck[HC], s1[HC], s2[HC];
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    ck[k] = cc[k];
    s1[k] = s2[k] = 0.0;
  }
  for (int t0 = u.j_begin; t0 < u.j_end; t0 += kBJ) {
    __syncthreads();
    for (int q = tid; q < kBJ / 2; q += kThreads)
      reinterpret_cast<double2*>(tile)[q] = reinterpret_cast<const double2*>(x + t0)[q];
    __syncthreads();
    int js = max(t0, wave_i0);
    const int te = t0 + kBJ;
    if (js < te) {
      if (js == wave_i0) {
        lscv_run64<HC, true>(tile, js - t0, js, xi, i, ck, s1, s2);
        js += kRun;
      }
      for (; js < te; js += kRun) lscv_run64<HC, false>(tile, js - t0, js, xi, i, ck, s1, s2);
    }
  }
  const bool valid = i < n;
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    const double v1 = wave_sum(valid ? s1[k] : 0.0);
    const double v2 = wave_sum(valid ? s2[k] : 0.0);
    if (lane == 0) {
      red[wave][2 * k] = v1;
      red[wave][2 * k + 1] = v2;
    }
  }
  __syncthreads();
  if (tid < 2 * HC) {
    const int h = u.chunk * HC + (tid >> 1);
    if (h < c.n_h) {
      const double v = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
      c.part[(int64_t)(2 * h + (tid & 1)) * c.n_items + u.item] = v;
    }
  }
}

// ---- LSCV pair kernel with the exponent arguments formed on the matrix cores.
// The argument of every (pair, h) term is D^2 * c_h: an outer product of the
// pair distances and the chunk's coefficients.  v_mfma_f32_32x32x2f32 forms
// it for 32 samples i x 2 samples j x 16 bandwidths at once (A[row][k] =
// D^2(i_row, j_k), B[k][col] = c[col % 16] if k = col / 16 else 0), so the
// vector ALU only evaluates exp2 and accumulates.  Lane l ends up owning
// bandwidth h = l % 16 for rows 8(r/4) + 4(l/32) + r%4 of the output block.
// Groups of 16 j whose pairs are all valid (j > i, i < n, j < n) run without
// masks; the others replace the argument of an invalid pair by -inf.
typedef float v16f __attribute__((ext_vector_type(16)));
constexpr float kBigF = 3.0e38f;

template <bool MASK>
__device__ __forceinline__ void mfma_consume(const v16f& da, const v16f& db, int j0, int jsel, int k, int ibase,
                                             int n, float (&s1)[4], float (&s2)[4]) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    float ya = da[r], yb = db[r];
    if (MASK) {
      const int row = 8 * (r >> 2) + 4 * k + (r & 3);
      const int j = j0 + jsel;
      const int ia = ibase + row, ib = ibase + 32 + row;
      ya = (j > ia && ia < n && j < n) ? ya : -kInfF;
      yb = (j > ib && ib < n && j < n) ? yb : -kInfF;
    }
    const float ea = __builtin_amdgcn_exp2f(ya);
    const float eb = __builtin_amdgcn_exp2f(yb);
    s1[r & 3] += ea;
    s2[r & 3] = __builtin_fmaf(ea, ea, s2[r & 3]);
    s1[r & 3] += eb;
    s2[r & 3] = __builtin_fmaf(eb, eb, s2[r & 3]);
  }
}

// 8 pairs (j, j+1) of one group of 16 j; the matrix-core products of the next
// pair are issued before the exponentials of the current one.
template <bool MASK>
__device__ __forceinline__ void mfma_group(const float4* __restrict__ tile, int jl, int jg, float xa, float xb,
                                           int ibase, int n, float bop, int lane, float (&s1)[4], float (&s2)[4]) {
  const int k = lane >> 5;
  const int jsel = (lane & 31) >> 4;
  const v16f zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float xj[8];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 v = tile[(jl >> 2) + q];
    xj[2 * q] = k ? v.y : v.x;
    xj[2 * q + 1] = k ? v.w : v.z;
  }
  float ta = xa - xj[0], tb = xb - xj[0];
  v16f da = __builtin_amdgcn_mfma_f32_32x32x2f32(fminf(ta * ta, kBigF), bop, zero, 0, 0, 0);
  v16f db = __builtin_amdgcn_mfma_f32_32x32x2f32(fminf(tb * tb, kBigF), bop, zero, 0, 0, 0);
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    v16f na, nb;
    if (p < 7) {
      ta = xa - xj[p + 1];
      tb = xb - xj[p + 1];
      na = __builtin_amdgcn_mfma_f32_32x32x2f32(fminf(ta * ta, kBigF), bop, zero, 0, 0, 0);
      nb = __builtin_amdgcn_mfma_f32_32x32x2f32(fminf(tb * tb, kBigF), bop, zero, 0, 0, 0);
    }
    mfma_consume<MASK>(da, db, jg + 2 * p, jsel, k, ibase, n, s1, s2);
    if (p < 7) {
      da = na;
      db = nb;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_lscv_units_mfma(const ColDesc* __restrict__ cols,
                                                              const Unit* __restrict__ units, int u0) {
  constexpr int HC = 16;
  const Unit u = units[u0 + blockIdx.x];
  const ColDesc c = cols[u.col];
  if (c.st->status != kStOk) return;
  const float* x = c.x32;
  const int n = c.n;
  __shared__ float4 tile[kBJ / 4];
  __shared__ double red[4][HC][2];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = u.row * kBI;
  const int wave_i0 = row0 + wave * 64;
  // A-operand rows: lane l holds samples i = wave_i0 + (l % 32) and i + 32
  const int ia = wave_i0 + (lane & 31), ib = ia + 32;
  const float xa = (ia < n) ? x[ia] : 0.f;
  const float xb = (ib < n) ? x[ib] : 0.f;
  // B operand: k = lane / 32, col = lane % 32
  const int kb = lane >> 5, colb = lane & 31;
  const float bop = (kb == (colb >> 4)) ? c.c32[u.chunk * HC + (colb & 15)] : 0.f;
  float a1 = 0.f, c1 = 0.f, a2 = 0.f, c2 = 0.f;
  const bool rows_full = wave_i0 + 64 <= n;
  for (int t0 = u.j_begin; t0 < u.j_end; t0 += kBJ) {
    __syncthreads();
    for (int q = tid; q < kBJ / 4; q += kThreads) tile[q] = reinterpret_cast<const float4*>(x + t0)[q];
    __syncthreads();
    const int te = t0 + kBJ;
    for (int js = max(t0, wave_i0); js < te; js += 16) {
      float s1[4] = {0.f, 0.f, 0.f, 0.f}, s2[4] = {0.f, 0.f, 0.f, 0.f};
      const bool clean = rows_full && js >= wave_i0 + 64 && js + 16 <= n;
      if (clean)
        mfma_group<false>(tile, js - t0, js, xa, xb, wave_i0, n, bop, lane, s1, s2);
      else
        mfma_group<true>(tile, js - t0, js, xa, xb, wave_i0, n, bop, lane, s1, s2);
      kahan_add(a1, c1, (s1[0] + s1[1]) + (s1[2] + s1[3]));
      kahan_add(a2, c2, (s2[0] + s2[1]) + (s2[2] + s2[3]));
    }
  }
  // lanes l, l^16, l^32, l^48 hold the same bandwidth
  double v1 = (double)a1 - (double)c1, v2 = (double)a2 - (double)c2;
  v1 += __shfl_xor(v1, 16, 64);
  v2 += __shfl_xor(v2, 16, 64);
  v1 += __shfl_xor(v1, 32, 64);
  v2 += __shfl_xor(v2, 32, 64);
  if (lane < HC) {
    red[wave][lane][0] = v1;
    red[wave][lane][1] = v2;
  }
  __syncthreads();
  if (tid < 2 * HC) {
    const int hk = tid >> 1, w = tid & 1;
    const int h = u.chunk * HC + hk;
    if (h < c.n_h) {
      const double v = ((red[0][hk][w] + red[1][hk][w]) + red[2][hk][w]) + red[3][hk][w];
      c.part[(int64_t)(2 * h + w) * c.n_items + u.item] = v;
    }
  }
}

// Block per column.  g(h) = h^-1 [2 n^-2 ((4pi)^-1/2 S1 - 2 (2pi)^-1/2 S2) + n^-1 (4pi)^-1/2];
// gscale with +.  Grid argmin with ties to the lowest index.
// g(h) of every grid point, argmin, edge flag and margin.  The mixed form's
// pair sums are exact sums at the bandwidth whose FP32 exponent coefficient
// c32 = -log2(e)/(4 h^2) is exactly representable; that bandwidth (within
// 3e-8 of the grid value) also goes into the 1/h factor, so each g is a
// consistent evaluation at a point next to the grid value rather than a
// mixture of two bandwidths, and the per-point error does not jump from one
// grid point to the next with the rounding of its coefficient.
__global__ __launch_bounds__(1024) void k_lscv_finalize(const ColDesc* __restrict__ cols,
                                                        const int* __restrict__ ids, int f64) {
  const ColDesc c = cols[ids[blockIdx.x]];
  if (c.n_h <= 0) return;
  DevState& d = *c.st;
  const int n_h = c.n_h;
  const double* sums = c.sums;
  const double* h_dev = c.h;
  double* g = c.g;
  double* gscale = c.gs;
  __shared__ double bv[1024];
  __shared__ int bk[1024];
  const int t = threadIdx.x;
  const double n = d.n;
  const double ckk = 1.0 / sqrt(4.0 * kPi), ck = 1.0 / sqrt(2.0 * kPi);
  const bool ok = d.status == kStOk;
  double best = kInfD;
  int kbest = 0x7fffffff;
  for (int k = t; k < n_h; k += blockDim.x) {
    const double s1 = sums[2 * k], s2 = sums[2 * k + 1];
    double h = h_dev[k];
    if (!f64) {
      const double cq = (double)c.c32[k];
      if (cq < 0.0 && isfinite(cq)) h = sqrt(-kLog2E / (4.0 * cq));
    }
    const double a = ckk * s1, b = ck * s2;
    const double gv = (2.0 / (n * n) * (a - 2.0 * b) + ckk / n) / h;
    g[k] = ok ? gv : NAN;
    gscale[k] = ok ? (2.0 / (n * n) * (a + 2.0 * b) + ckk / n) / h : NAN;
    if (gv < best) {
      best = gv;
      kbest = k;
    }
  }
  bv[t] = best;
  bk[t] = kbest;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) {
      const double ov = bv[t + s];
      const int ok2 = bk[t + s];
      if (ov < bv[t] || (ov == bv[t] && ok2 < bk[t])) {
        bv[t] = ov;
        bk[t] = ok2;
      }
    }
    __syncthreads();
  }
  const int kb = bk[0];
  const double vb = bv[0];
  __syncthreads();
  double second = kInfD;
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
      d.k_best = kb;
      d.h_best = h_dev[kb];
      d.at_edge = (kb == 0 || kb == n_h - 1) ? 1 : 0;
      d.margin = (n_h > 1) ? bv[0] - vb : 0.0;
    } else {
      d.status = kStDegenerate;  // every g(h) was NaN
    }
  }
}

// Segmented sum, block per row: *dst = sum_c src[c], fixed order.
__global__ __launch_bounds__(kThreads) void k_reduce_rows(const RowDesc* __restrict__ rows) {
  __shared__ double sh[kThreads];
  const RowDesc r = rows[blockIdx.x];
  double s = 0.0;
  for (int c = threadIdx.x; c < r.n; c += kThreads) s += r.src[c];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *r.dst = s;
}

}  // namespace

// ------------------------------------------------------------------ launchers
static inline int id_blocks(int n_ids) { return (n_ids + kThreads - 1) / kThreads; }

void launch_stats(hipStream_t s, const ColDesc* cols, const int* ids, int n_ids, int max_blocks) {
  if (n_ids <= 0) return;
  const dim3 grid2(max_blocks, n_ids);
  k_stats_sum<<<grid2, kThreads, 0, s>>>(cols, ids);
  k_stats_mean<<<n_ids, kThreads, 0, s>>>(cols, ids);
  k_stats_dev<<<grid2, kThreads, 0, s>>>(cols, ids);
  k_stats_final<<<n_ids, kThreads, 0, s>>>(cols, ids);
}

void launch_psi_begin(hipStream_t s, const ColDesc* cols, const int* ids, int n_ids, int stage, int f64) {
  if (n_ids <= 0) return;
  k_psi_begin<<<id_blocks(n_ids), kThreads, 0, s>>>(cols, ids, n_ids, stage);
  if (!f64) k_psi_scale<<<dim3(128, n_ids), kThreads, 0, s>>>(cols, ids);
}

void launch_psi_finish(hipStream_t s, const ColDesc* cols, const int* ids, int n_ids, int stage, int was_f64,
                       int conditional) {
  if (n_ids > 0) k_psi_finish<<<id_blocks(n_ids), kThreads, 0, s>>>(cols, ids, n_ids, stage, was_f64, conditional);
}

void launch_plugin_final(hipStream_t s, const ColDesc* cols, const int* ids, int n_ids) {
  if (n_ids > 0) k_plugin_final<<<id_blocks(n_ids), kThreads, 0, s>>>(cols, ids, n_ids);
}

void launch_lscv_prep(hipStream_t s, const ColDesc* cols, const int* ids, int n_ids, int hc) {
  if (n_ids > 0) k_lscv_prep<<<n_ids, kThreads, 0, s>>>(cols, ids, hc);
}

void launch_lscv_finalize(hipStream_t s, const ColDesc* cols, const int* ids, int n_ids, int f64) {
  if (n_ids > 0) k_lscv_finalize<<<n_ids, 1024, 0, s>>>(cols, ids, f64);
}

void launch_psi_units(hipStream_t s, int r, int f64, int conditional, const ColDesc* cols, const Unit* units, int u0,
                      int n_units) {
  if (n_units <= 0) return;
  if (f64) {
    switch (r) {
      case 8: k_psi_units_f64<8><<<n_units, kThreads, 0, s>>>(cols, units, u0, conditional); break;
      case 6: k_psi_units_f64<6><<<n_units, kThreads, 0, s>>>(cols, units, u0, conditional); break;
      default: k_psi_units_f64<4><<<n_units, kThreads, 0, s>>>(cols, units, u0, conditional); break;
    }
  } else {
    switch (r) {
      case 8: k_psi_units_f32<8><<<n_units, kThreads, 0, s>>>(cols, units, u0); break;
      case 6: k_psi_units_f32<6><<<n_units, kThreads, 0, s>>>(cols, units, u0); break;
      default: k_psi_units_f32<4><<<n_units, kThreads, 0, s>>>(cols, units, u0); break;
    }
  }
}

void launch_zero_ints(hipStream_t s, int* p, int n) {
  if (n > 0) k_zero_ints<<<(n + 255) / 256, 256, 0, s>>>(p, n);
}

// The persistent sweep's variants: (bandwidths per block, samples per LDS
// tile).  The autotuner chooses among them; (16, 512) is the default.
namespace {
template <int HC, int TJ>
int queue_blocks_of() {
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_lscv_units_f32_queue<HC, TJ>, kThreads, 0) !=
          hipSuccess ||
      per_cu < 1)
    return 0;
  return per_cu * prop.multiProcessorCount;
}
}  // namespace

bool lscv_queue_variant(int hc, int tj) {
  return (tj == 512 && (hc == 8 || hc == 16 || hc == 32)) || (hc == 16 && (tj == 256 || tj == 1024));
}

int lscv_queue_blocks(int hc, int tj) {
  if (tj == 256) return queue_blocks_of<16, 256>();
  if (tj == 1024) return queue_blocks_of<16, 1024>();
  switch (hc) {
    case 8: return queue_blocks_of<8, 512>();
    case 32: return queue_blocks_of<32, 512>();
    default: return queue_blocks_of<16, 512>();
  }
}

void launch_lscv_units_queue(hipStream_t s, int hc, int tj, const ColDesc* cols, const Unit* units, int n_units,
                             const int* group_begin, int* next, int blocks) {
  if (n_units <= 0) return;
  blocks = max(1, min(blocks, n_units));
  if (tj == 256) {
    k_lscv_units_f32_queue<16, 256><<<blocks, kThreads, 0, s>>>(cols, units, group_begin, next);
  } else if (tj == 1024) {
    k_lscv_units_f32_queue<16, 1024><<<blocks, kThreads, 0, s>>>(cols, units, group_begin, next);
  } else {
    switch (hc) {
      case 8: k_lscv_units_f32_queue<8, 512><<<blocks, kThreads, 0, s>>>(cols, units, group_begin, next); break;
      case 32: k_lscv_units_f32_queue<32, 512><<<blocks, kThreads, 0, s>>>(cols, units, group_begin, next); break;
      default: k_lscv_units_f32_queue<16, 512><<<blocks, kThreads, 0, s>>>(cols, units, group_begin, next); break;
    }
  }
}

void launch_lscv_units(hipStream_t s, int hc, int f64, int mfma, int prune, const ColDesc* cols, const Unit* units,
                       int u0, int n_units) {
  if (n_units <= 0) return;
  if (prune && !f64) {
    switch (hc) {
      case 8: k_lscv_units_prune<8><<<n_units, kThreads, 0, s>>>(cols, units, u0); break;
      case 32: k_lscv_units_prune<32><<<n_units, kThreads, 0, s>>>(cols, units, u0); break;
      default: k_lscv_units_prune<16><<<n_units, kThreads, 0, s>>>(cols, units, u0); break;
    }
    return;
  }
  if (mfma && !f64 && hc == 16) {
    k_lscv_units_mfma<<<n_units, kThreads, 0, s>>>(cols, units, u0);
    return;
  }
  if (f64) {
    switch (hc) {
      case 4: k_lscv_units_f64<4><<<n_units, kThreads, 0, s>>>(cols, units, u0); break;
      default: k_lscv_units_f64<8><<<n_units, kThreads, 0, s>>>(cols, units, u0); break;
    }
  } else {
    switch (hc) {
      case 8: k_lscv_units_f32<8><<<n_units, kThreads, 0, s>>>(cols, units, u0); break;
      case 32: k_lscv_units_f32<32><<<n_units, kThreads, 0, s>>>(cols, units, u0); break;
      default: k_lscv_units_f32<16><<<n_units, kThreads, 0, s>>>(cols, units, u0); break;
    }
  }
}

void launch_lscv_ceiling(hipStream_t s, int hc, const float* x, const float* c32, int reps, double* out, int blocks) {
  if (blocks <= 0) return;
  switch (hc) {
    case 8: k_lscv_ceiling<8><<<blocks, kThreads, 0, s>>>(x, c32, reps, out); break;
    case 32: k_lscv_ceiling<32><<<blocks, kThreads, 0, s>>>(x, c32, reps, out); break;
    default: k_lscv_ceiling<16><<<blocks, kThreads, 0, s>>>(x, c32, reps, out); break;
  }
}

void launch_lscv_prune_prep(hipStream_t s, const ColDesc* cols, const int* ids, int n_ids, int hc, double eps) {
  if (n_ids > 0) k_lscv_prune_prep<<<n_ids, kThreads, 0, s>>>(cols, ids, hc, eps);
}

void launch_reduce_rows(hipStream_t s, const RowDesc* rows, int n_rows) {
  if (n_rows > 0) k_reduce_rows<<<n_rows, kThreads, 0, s>>>(rows);
}

}  // namespace kde
