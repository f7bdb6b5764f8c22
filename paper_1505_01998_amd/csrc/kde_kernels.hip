// kde_kernels.hip -- gfx950 kernels for exact bandwidth-selection pair sums.
//
// Method: Andrzejewski, Gramacki, Gramacki, arXiv 1505.01998, Section 4.4
// (selectors), Section 4.5 (pair distance reused across bandwidths) and
// Section 5.4 (sums of a function of X_i - X_j over the i < j triangle).
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
// 64 consecutive j in plain FP32, then folds that run into a Kahan-
// compensated FP32 accumulator.  Lane accumulators are converted to FP64 and
// reduced across the wave (butterfly shuffles), the block (LDS, fixed order)
// and the work items (a separate row-reduction kernel, fixed order), so the
// result is deterministic and independent of scheduling.  The FP64 form
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

// He_r(0) for the kernel-derivative value K^(r)(0) = He_r(0) / sqrt(2 pi).
__device__ __forceinline__ double herm_at0(int r) {
  return r == 4 ? 3.0 : (r == 6 ? -15.0 : (r == 8 ? 105.0 : 0.0));
}

// Normal-scale functional psi_r for N(0, sigma^2):
// (-1)^(r/2) r! / ((2 sigma)^(r+1) (r/2)! sqrt(pi)); r = 8 gives 105 / (32 sqrt(pi) sigma^9).
__device__ double psi_normal_scale(int r, double sigma) {
  double num = 1.0, den = 1.0;
  for (int k = 2; k <= r; ++k) num *= (double)k;
  for (int k = 2; k <= r / 2; ++k) den *= (double)k;
  const double sgn = ((r / 2) % 2 == 0) ? 1.0 : -1.0;
  return sgn * num / (pow(2.0 * sigma, (double)(r + 1)) * den * sqrt(kPi));
}

// ------------------------------------------------------------------ statistics
template <typename T>
__global__ __launch_bounds__(kThreads) void k_stats_sum(const T* __restrict__ x, int n, double* __restrict__ part,
                                                        int* __restrict__ part_nf) {
  __shared__ double sh[kThreads];
  __shared__ int nf_sh;
  const int chunk = (n + gridDim.x - 1) / gridDim.x;
  const int b0 = blockIdx.x * chunk;
  const int b1 = min(n, b0 + chunk);
  if (threadIdx.x == 0) nf_sh = 0;
  __syncthreads();
  double s = 0.0;
  int nf = 0;
  for (int i = b0 + threadIdx.x; i < b1; i += kThreads) {
    const double v = (double)x[i];
    if (!isfinite(v)) ++nf; else s += v;
  }
  if (nf) atomicAdd(&nf_sh, nf);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s;
    part_nf[blockIdx.x] = nf_sh;
  }
}

__global__ __launch_bounds__(kThreads) void k_stats_mean(const double* __restrict__ part,
                                                         const int* __restrict__ part_nf, int nblk, int n,
                                                         int shift_by_mean, DevState* st) {
  __shared__ double sh[kThreads];
  __shared__ int nf_sh;
  if (threadIdx.x == 0) nf_sh = 0;
  __syncthreads();
  double s = 0.0;
  int nf = 0;
  for (int b = threadIdx.x; b < nblk; b += kThreads) {
    s += part[b];
    nf += part_nf[b];
  }
  if (nf) atomicAdd(&nf_sh, nf);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    st->n = (double)n;
    st->status = nf_sh ? kStInval : kStOk;
    st->mean = s / (double)n;
    st->shift = shift_by_mean ? st->mean : 0.0;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_stats_dev(const T* __restrict__ x, int n, int n_pad,
                                                        double* __restrict__ part, float* __restrict__ x32,
                                                        double* __restrict__ x64, const DevState* st) {
  __shared__ double sh[kThreads];
  const double mean = st->mean, shift = st->shift;
  const int chunk = (n + gridDim.x - 1) / gridDim.x;
  const int b0 = blockIdx.x * chunk;
  const int b1 = min(n, b0 + chunk);
  double s = 0.0;
  for (int i = b0 + threadIdx.x; i < b1; i += kThreads) {
    const double v = (double)x[i];
    const double d = v - mean;
    s += d * d;
    x32[i] = (float)(v - shift);
    if (x64) x64[i] = v;
  }
  for (int i = n + blockIdx.x * kThreads + threadIdx.x; i < n_pad; i += gridDim.x * kThreads) {
    x32[i] = kInfF;
    if (x64) x64[i] = kInfD;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_stats_final(const double* __restrict__ part, int nblk, DevState* st) {
  __shared__ double sh[kThreads];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kThreads) s += part[b];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    const double n = st->n;
    st->var = s / (n - 1.0);
    st->sigma = sqrt(st->var);
    // normal-reference rule: (4/3)^(1/5) sigma n^(-1/5)
    st->h_rot = pow(4.0 / 3.0, 0.2) * pow(n, -0.2) * st->sigma;
    if (st->status == kStOk && !(st->sigma > 0.0 && isfinite(st->sigma))) st->status = kStDegenerate;
  }
}

// ------------------------------------------------------------------ plug-in scalar steps
// Stage s in {0, 1, 2} estimates psi_r with r = 8 - 2 s.
__global__ void k_psi_begin(DevState* st, int stage) {
  if (st->status != kStOk) return;
  const int r = 8 - 2 * stage;
  double psi_next;
  if (stage == 0) {
    psi_next = psi_normal_scale(10, st->sigma);
  } else if (stage == 1) {
    if (st->stages == 2) st->psi[0] = psi_normal_scale(8, st->sigma);
    psi_next = st->psi[0];
  } else {
    psi_next = st->psi[1];
  }
  // AMSE pilot: g = [-2 K^(r)(0) / (mu_2 psi_{r+2} n)]^(1/(r+3)), mu_2 = 1
  const double k0 = herm_at0(r) / sqrt(2.0 * kPi);
  const double rad = -2.0 * k0 / (psi_next * st->n);
  if (!(rad > 0.0) || !isfinite(rad)) {
    st->status = kStDegenerate;
    return;
  }
  const double g = pow(rad, 1.0 / (double)(r + 3));
  st->g[stage] = g;
  const double ig2 = 1.0 / (g * g);
  st->cf[0] = (float)ig2;
  st->cf[1] = (float)(-0.5 * kLog2E * ig2);
  st->cd[0] = ig2;
  st->cd[1] = -0.5 * ig2;
  st->need_f64 = 0;
}

// sums[0] = sum_{i<j} He_r(u) e^{-u^2/2}, sums[1] = sum of its absolute value,
// u = (X_i - X_j)/g.  psi_r = [2 sum K^(r) + n K^(r)(0)] / (n^2 g^(r+1)).
// conditional: this is the FP64 re-run of the mixed form; skip unless flagged.
__global__ void k_psi_finish(DevState* st, int stage, const double* __restrict__ sums, int was_f64,
                             int conditional) {
  if (st->status != kStOk) return;
  if (conditional && !st->need_f64) return;
  const int r = 8 - 2 * stage;
  const double inv_s2pi = 1.0 / sqrt(2.0 * kPi);
  const double n = st->n, g = st->g[stage];
  const double s = sums[0] * inv_s2pi, a = sums[1] * inv_s2pi;
  st->psi[stage] = (2.0 * s + n * herm_at0(r) * inv_s2pi) / (n * n * pow(g, (double)(r + 1)));
  st->kappa[stage] = (s != 0.0) ? a / fabs(s) : kInfD;
  st->prec_used[stage] = was_f64 ? 1 : 0;
  if (was_f64) {
    st->need_f64 = 0;
  } else {
    st->need_f64 = (st->fp64_kappa > 0.0 && st->kappa[stage] > st->fp64_kappa) ? 1 : 0;
  }
}

__global__ void k_plugin_final(DevState* st) {
  if (st->status != kStOk) return;
  // h = [R(K) / (mu_2^2 psi_4 n)]^(1/5), R(K) = 1/(2 sqrt(pi))
  const double rad = (0.5 / sqrt(kPi)) / (st->psi[2] * st->n);
  if (!(rad > 0.0) || !isfinite(rad)) {
    st->status = kStDegenerate;
    return;
  }
  st->h_plugin = pow(rad, 0.2);
}

// ------------------------------------------------------------------ psi pair kernels
template <int R, bool MASK>
__device__ __forceinline__ void psi_run(const float4* __restrict__ tile, int jl, int jg, float xi, int i, float ig2,
                                        float cg, float& aS, float& cS, float& aA, float& cA) {
  float rs = 0.f, ra = 0.f;
#pragma unroll 4
  for (int q = 0; q < kRun / 4; ++q) {
    const float4 v = tile[(jl >> 2) + q];
    const float xs[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float d = xi - xs[u];
      float t = d * d;
      if (MASK) t = (jg + 4 * q + u > i) ? t : kInfF;
      const float w = fminf(t * ig2, kWMax);
      const float e = __builtin_amdgcn_exp2f(t * cg);
      const float term = herm_w<R>(w) * e;
      rs += term;
      ra += fabsf(term);
    }
  }
  kahan_add(aS, cS, rs);
  kahan_add(aA, cA, ra);
}

template <int R>
__global__ __launch_bounds__(kThreads) void k_psi_pairs_f32(const float* __restrict__ x, int n,
                                                            const Item* __restrict__ items, int n_items, int bid0,
                                                            double* __restrict__ part,
                                                            const DevState* __restrict__ st) {
  if (st->status != kStOk) return;
  __shared__ float4 tile[kBJ / 4];
  __shared__ double red[2][4];
  const int item = bid0 + blockIdx.x;
  const Item it = items[item];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = it.row * kBI;
  const int i = row0 + tid;
  const float xi = (i < n) ? x[i] : 0.f;
  const int wave_i0 = row0 + wave * 64;
  const float ig2 = st->cf[0], cg = st->cf[1];
  float aS = 0.f, cS = 0.f, aA = 0.f, cA = 0.f;
  for (int t0 = it.j_begin; t0 < it.j_end; t0 += kBJ) {
    __syncthreads();
    for (int q = tid; q < kBJ / 4; q += kThreads) tile[q] = reinterpret_cast<const float4*>(x + t0)[q];
    __syncthreads();
    int js = max(t0, wave_i0);
    const int te = t0 + kBJ;
    if (js < te) {
      if (js == wave_i0) {
        psi_run<R, true>(tile, js - t0, js, xi, i, ig2, cg, aS, cS, aA, cA);
        js += kRun;
      }
      for (; js < te; js += kRun) psi_run<R, false>(tile, js - t0, js, xi, i, ig2, cg, aS, cS, aA, cA);
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
  if (tid < 2) part[(size_t)tid * n_items + item] = ((red[tid][0] + red[tid][1]) + red[tid][2]) + red[tid][3];
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
    const double term = herm_w64<R>(w) * exp(t * cg);
    s += term;
    a += fabs(term);
  }
}

// conditional: run only when the FP32 pass flagged this stage (mixed form).
template <int R>
__global__ __launch_bounds__(kThreads) void k_psi_pairs_f64(const double* __restrict__ x, int n,
                                                            const Item* __restrict__ items, int n_items, int bid0,
                                                            double* __restrict__ part, const DevState* __restrict__ st,
                                                            int conditional) {
  if (st->status != kStOk) return;
  if (conditional && !st->need_f64) return;
  __shared__ double tile[kBJ];
  __shared__ double red[2][4];
  const int item = bid0 + blockIdx.x;
  const Item it = items[item];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = it.row * kBI;
  const int i = row0 + tid;
  const double xi = (i < n) ? x[i] : 0.0;
  const int wave_i0 = row0 + wave * 64;
  const double ig2 = st->cd[0], cg = st->cd[1];
  double s = 0.0, a = 0.0;
  for (int t0 = it.j_begin; t0 < it.j_end; t0 += kBJ) {
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
  if (tid < 2) part[(size_t)tid * n_items + item] = ((red[tid][0] + red[tid][1]) + red[tid][2]) + red[tid][3];
}

// ------------------------------------------------------------------ LSCV kernels
// c32[k] = -log2(e) / (4 h_k^2), so exp2(D^2 c32[k]) = exp(-D^2/(4 h^2)) and its
// square is exp(-D^2/(2 h^2)).  Padded chunk entries hold -1 (finite, unused).
__global__ __launch_bounds__(kThreads) void k_lscv_prep(const double* __restrict__ h_in, int n_h, int n_h_pad,
                                                        DevState* st, double* __restrict__ h_dev,
                                                        float* __restrict__ c32, double* __restrict__ c64) {
  const bool dflt = (h_in == nullptr);
  const double lo = st->h_rot * 0.25, hi = st->h_rot * 4.0;
  for (int k = threadIdx.x; k < n_h_pad; k += kThreads) {
    if (k < n_h) {
      double h;
      if (dflt)
        h = (n_h == 1) ? lo : lo + (hi - lo) * (double)k / (double)(n_h - 1);
      else
        h = h_in[k];
      h_dev[k] = h;
      const double q = 1.0 / (4.0 * h * h);
      c32[k] = (float)(-kLog2E * q);
      c64[k] = -q;
    } else {
      c32[k] = -1.0f;
      c64[k] = -1.0;
    }
  }
}

template <int HC, bool MASK>
__device__ __forceinline__ void lscv_run(const float4* __restrict__ tile, int jl, int jg, float xi, int i,
                                         const float (&ck)[HC], float (&a1)[HC], float (&c1)[HC], float (&a2)[HC],
                                         float (&c2)[HC]) {
  float r1[HC], r2[HC];
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    r1[k] = 0.f;
    r2[k] = 0.f;
  }
#pragma unroll 2
  for (int q = 0; q < kRun / 4; ++q) {
    const float4 v = tile[(jl >> 2) + q];
    const float xs[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float d = xi - xs[u];
      float t = d * d;
      if (MASK) t = (jg + 4 * q + u > i) ? t : kInfF;
#pragma unroll
      for (int k = 0; k < HC; ++k) {
        const float e = __builtin_amdgcn_exp2f(t * ck[k]);
        r1[k] += e;
        r2[k] = __builtin_fmaf(e, e, r2[k]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    kahan_add(a1[k], c1[k], r1[k]);
    kahan_add(a2[k], c2[k], r2[k]);
  }
}

template <int HC>
__global__ __launch_bounds__(kThreads) void k_lscv_pairs_f32(const float* __restrict__ x, int n,
                                                             const Item* __restrict__ items, int n_items,
                                                             int n_chunks, const float* __restrict__ c32, int n_h,
                                                             int bid0, double* __restrict__ part,
                                                             const DevState* __restrict__ st) {
  if (st->status != kStOk) return;
  __shared__ float4 tile[kBJ / 4];
  __shared__ double red[4][2 * HC];
  const int bid = bid0 + blockIdx.x;
  const int item = bid / n_chunks;
  const int chunk = bid - item * n_chunks;
  const Item it = items[item];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = it.row * kBI;
  const int i = row0 + tid;
  const float xi = (i < n) ? x[i] : 0.f;
  const int wave_i0 = row0 + wave * 64;
  float ck[HC], a1[HC], c1[HC], a2[HC], c2[HC];
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    ck[k] = c32[chunk * HC + k];
    a1[k] = c1[k] = a2[k] = c2[k] = 0.f;
  }
  for (int t0 = it.j_begin; t0 < it.j_end; t0 += kBJ) {
    __syncthreads();
    for (int q = tid; q < kBJ / 4; q += kThreads) tile[q] = reinterpret_cast<const float4*>(x + t0)[q];
    __syncthreads();
    int js = max(t0, wave_i0);
    const int te = t0 + kBJ;
    if (js < te) {
      if (js == wave_i0) {
        lscv_run<HC, true>(tile, js - t0, js, xi, i, ck, a1, c1, a2, c2);
        js += kRun;
      }
      for (; js < te; js += kRun) lscv_run<HC, false>(tile, js - t0, js, xi, i, ck, a1, c1, a2, c2);
    }
  }
  const bool valid = i < n;
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    const double v1 = wave_sum(valid ? (double)a1[k] - (double)c1[k] : 0.0);
    const double v2 = wave_sum(valid ? (double)a2[k] - (double)c2[k] : 0.0);
    if (lane == 0) {
      red[wave][2 * k] = v1;
      red[wave][2 * k + 1] = v2;
    }
  }
  __syncthreads();
  if (tid < 2 * HC) {
    const int h = chunk * HC + (tid >> 1);
    if (h < n_h) {
      const double v = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
      part[(size_t)(2 * h + (tid & 1)) * n_items + item] = v;
    }
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
      const double e = exp(t * ck[k]);
      s1[k] += e;
      s2[k] = __builtin_fma(e, e, s2[k]);
    }
  }
}

template <int HC>
__global__ __launch_bounds__(kThreads) void k_lscv_pairs_f64(const double* __restrict__ x, int n,
                                                             const Item* __restrict__ items, int n_items,
                                                             int n_chunks, const double* __restrict__ c64, int n_h,
                                                             int bid0, double* __restrict__ part,
                                                             const DevState* __restrict__ st) {
  if (st->status != kStOk) return;
  __shared__ double tile[kBJ];
  __shared__ double red[4][2 * HC];
  const int bid = bid0 + blockIdx.x;
  const int item = bid / n_chunks;
  const int chunk = bid - item * n_chunks;
  const Item it = items[item];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = it.row * kBI;
  const int i = row0 + tid;
  const double xi = (i < n) ? x[i] : 0.0;
  const int wave_i0 = row0 + wave * 64;
  double ck[HC], s1[HC], s2[HC];
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    ck[k] = c64[chunk * HC + k];
    s1[k] = s2[k] = 0.0;
  }
  for (int t0 = it.j_begin; t0 < it.j_end; t0 += kBJ) {
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
    const int h = chunk * HC + (tid >> 1);
    if (h < n_h) {
      const double v = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
      part[(size_t)(2 * h + (tid & 1)) * n_items + item] = v;
    }
  }
}

// g(h) = h^-1 [2 n^-2 ((4pi)^-1/2 S1 - 2 (2pi)^-1/2 S2) + n^-1 (4pi)^-1/2]; gscale with +.
// Grid argmin with ties to the lowest index.
__global__ __launch_bounds__(1024) void k_lscv_finalize(const double* __restrict__ sums, int n_h,
                                                        const double* __restrict__ h_dev, DevState* st,
                                                        double* __restrict__ g, double* __restrict__ gscale) {
  __shared__ double bv[1024];
  __shared__ int bk[1024];
  const int t = threadIdx.x;
  const double n = st->n;
  const double ckk = 1.0 / sqrt(4.0 * kPi), ck = 1.0 / sqrt(2.0 * kPi);
  const bool ok = st->status == kStOk;
  double best = kInfD;
  int kbest = 0x7fffffff;
  for (int k = t; k < n_h; k += blockDim.x) {
    const double s1 = sums[2 * k], s2 = sums[2 * k + 1], h = h_dev[k];
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
      st->k_best = kb;
      st->h_best = h_dev[kb];
      st->at_edge = (kb == 0 || kb == n_h - 1) ? 1 : 0;
      st->margin = (n_h > 1) ? bv[0] - vb : 0.0;
    } else {
      st->status = kStDegenerate;  // every g(h) was NaN
    }
  }
}

// out[r] = sum_c part[r * n_cols + c], in a fixed order.
__global__ __launch_bounds__(kThreads) void k_reduce_rows(const double* __restrict__ part, int n_cols,
                                                          double* __restrict__ out) {
  __shared__ double sh[kThreads];
  const double* p = part + (size_t)blockIdx.x * n_cols;
  double s = 0.0;
  for (int c = threadIdx.x; c < n_cols; c += kThreads) s += p[c];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

}  // namespace

// ------------------------------------------------------------------ launchers
void launch_stats_sum(hipStream_t s, const void* x, int is_f64, int n, double* part, int* part_nf, int nblk) {
  if (is_f64)
    k_stats_sum<double><<<nblk, kThreads, 0, s>>>((const double*)x, n, part, part_nf);
  else
    k_stats_sum<float><<<nblk, kThreads, 0, s>>>((const float*)x, n, part, part_nf);
}

void launch_stats_mean(hipStream_t s, const double* part, const int* part_nf, int nblk, int n, int shift_by_mean,
                       DevState* st) {
  k_stats_mean<<<1, kThreads, 0, s>>>(part, part_nf, nblk, n, shift_by_mean, st);
}

void launch_stats_dev(hipStream_t s, const void* x, int is_f64, int n, int n_pad, double* part, float* x32,
                      double* x64, int nblk, DevState* st) {
  if (is_f64)
    k_stats_dev<double><<<nblk, kThreads, 0, s>>>((const double*)x, n, n_pad, part, x32, x64, st);
  else
    k_stats_dev<float><<<nblk, kThreads, 0, s>>>((const float*)x, n, n_pad, part, x32, x64, st);
}

void launch_stats_final(hipStream_t s, const double* part, int nblk, DevState* st) {
  k_stats_final<<<1, kThreads, 0, s>>>(part, nblk, st);
}

void launch_psi_begin(hipStream_t s, DevState* st, int stage) { k_psi_begin<<<1, 1, 0, s>>>(st, stage); }

void launch_psi_finish(hipStream_t s, DevState* st, int stage, const double* sums, int was_f64, int conditional) {
  k_psi_finish<<<1, 1, 0, s>>>(st, stage, sums, was_f64, conditional);
}

void launch_plugin_final(hipStream_t s, DevState* st) { k_plugin_final<<<1, 1, 0, s>>>(st); }

void launch_psi_pairs(hipStream_t s, int r, int f64, int conditional, const float* x32, const double* x64, int n,
                      const Item* items, int n_items, int bid0, int nblk, double* part, const DevState* st) {
  if (f64) {
    switch (r) {
      case 8: k_psi_pairs_f64<8><<<nblk, kThreads, 0, s>>>(x64, n, items, n_items, bid0, part, st, conditional); break;
      case 6: k_psi_pairs_f64<6><<<nblk, kThreads, 0, s>>>(x64, n, items, n_items, bid0, part, st, conditional); break;
      default: k_psi_pairs_f64<4><<<nblk, kThreads, 0, s>>>(x64, n, items, n_items, bid0, part, st, conditional); break;
    }
  } else {
    switch (r) {
      case 8: k_psi_pairs_f32<8><<<nblk, kThreads, 0, s>>>(x32, n, items, n_items, bid0, part, st); break;
      case 6: k_psi_pairs_f32<6><<<nblk, kThreads, 0, s>>>(x32, n, items, n_items, bid0, part, st); break;
      default: k_psi_pairs_f32<4><<<nblk, kThreads, 0, s>>>(x32, n, items, n_items, bid0, part, st); break;
    }
  }
}

void launch_lscv_prep(hipStream_t s, const double* h_in, int n_h, int n_h_pad, DevState* st, double* h_dev,
                      float* c32, double* c64) {
  k_lscv_prep<<<1, kThreads, 0, s>>>(h_in, n_h, n_h_pad, st, h_dev, c32, c64);
}

void launch_lscv_pairs(hipStream_t s, int hc, int f64, const float* x32, const double* x64, int n,
                       const Item* items, int n_items, int n_chunks, const float* c32, const double* c64, int n_h,
                       int bid0, int nblk, double* part, const DevState* st) {
  if (f64) {
    switch (hc) {
      case 4: k_lscv_pairs_f64<4><<<nblk, kThreads, 0, s>>>(x64, n, items, n_items, n_chunks, c64, n_h, bid0, part, st); break;
      default: k_lscv_pairs_f64<8><<<nblk, kThreads, 0, s>>>(x64, n, items, n_items, n_chunks, c64, n_h, bid0, part, st); break;
    }
  } else {
    switch (hc) {
      case 8: k_lscv_pairs_f32<8><<<nblk, kThreads, 0, s>>>(x32, n, items, n_items, n_chunks, c32, n_h, bid0, part, st); break;
      case 32: k_lscv_pairs_f32<32><<<nblk, kThreads, 0, s>>>(x32, n, items, n_items, n_chunks, c32, n_h, bid0, part, st); break;
      default: k_lscv_pairs_f32<16><<<nblk, kThreads, 0, s>>>(x32, n, items, n_items, n_chunks, c32, n_h, bid0, part, st); break;
    }
  }
}

void launch_lscv_finalize(hipStream_t s, const double* sums, int n_h, const double* h_dev, DevState* st, double* g,
                          double* gscale) {
  k_lscv_finalize<<<1, 1024, 0, s>>>(sums, n_h, h_dev, st, g, gscale);
}

void launch_reduce_rows(hipStream_t s, const double* part, int n_cols, int n_rows, double* out) {
  k_reduce_rows<<<n_rows, kThreads, 0, s>>>(part, n_cols, out);
}

}  // namespace kde
