// kde_lscv_H.hip -- LSCV_H (Section 4.4.3): the objective g(H) at full
// bandwidth matrices, eq. (LSCV_MULTI-gh) with (LSCV_MULTI-Tx),
// (LSCV_MULTI-Kx), (LSCV_MULTI-KKx) and (LSCV_MULTI-rk), and its Nelder-Mead
// minimisation over positive definite H from the rule-of-thumb start of
// eq. (LSCV-H-start).  The samples are staged and sphered as for LSCV_h
// (kde_md.h): Y = L^-1 (X - mean), Sigma = L L^T.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "kde_md.h"

namespace kde {

namespace {

// ---- device part.  With G = L^-1 H L^-T = L_G L_G^T (Sigma = L L^T, Y the
// sphered samples) the quadratic form of a pair is v^T H^-1 v = |L_G^-1 w|^2,
// w = Y_i - Y_j.  Each matrix therefore gets the samples whitened for it,
// Z = c M (X - mean) with M = L_G^-1 L^-1 (lower triangular; c folds the
// exponent's factor: c^2 = log2(e)/4 in the mixed form, 1/4 in FP64), and
// one sweep of the pair triangle in the layout of the sphered LSCV_h kernel:
// a block holds 256 samples i (D coordinates in registers) and walks its
// item's j-range in LDS tiles of D x 512 coordinates; each pair costs D
// differences, the squared norm and one exponential (exp2(-|dz|^2) in FP32,
// S2 from its square), with no per-pair coefficient.  Every matrix is
// processed the same way whatever the batch, so g of a matrix does not
// depend on the other matrices of the call.  The mixed form rounds Z to FP32
// (compensated 64-term runs, FP64 above the lane); both forms evaluate g at H
// itself.  Padding samples hold +inf in the first coordinate.
struct HDesc {
  double logdet;  // log |H|
  int valid;      // H and G positive definite
  int pad0;
};

// one thread per matrix (H row-major d x d, its lower triangle read): the
// whitening map c M (row stride KDE_MAX_D) and log|H|
__global__ void k_H_prep(const MdState* st, const double* H, int m, int f64, HDesc* out, double* Mout) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int d = st->d;
  double A[KDE_MAX_D][KDE_MAX_D], L[KDE_MAX_D][KDE_MAX_D], T[KDE_MAX_D][KDE_MAX_D];
  double* M = Mout + (int64_t)k * KDE_MAX_D * KDE_MAX_D;
  for (int q = 0; q < KDE_MAX_D * KDE_MAX_D; ++q) M[q] = 0.0;
  HDesc o;
  o.logdet = 0.0;
  o.valid = 0;
  o.pad0 = 0;
  const double* Hk = H + (int64_t)k * d * d;
  // Cholesky factor of A with the library's pivot rule (a pivot at most
  // 1e-12 of its diagonal entry fails) and log|A|
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
  const double cf = f64 ? 0.5 : sqrt(0.25 * kLog2ED);
  for (int a = 0; a < d; ++a)  // M = c L_G^-1 L^-1
    for (int b = 0; b <= a; ++b) {
      double s = 0.0;
      for (int c = b; c <= a; ++c) s += T[a][c] * st->linv[c * KDE_MAX_D + b];
      M[a * KDE_MAX_D + b] = cf * s;
    }
  o.logdet = st->logdet + ldG;
  o.valid = 1;
  out[k] = o;
}

// 64 consecutive j of the tile for lane i: exp2(-|z_i - z_j|^2) summed, and
// its squares; MASK drops j <= i (the diagonal run of a wave)
template <int D, bool MASK>
__device__ __forceinline__ void hz_run(const float (*tile)[kBJ], int jl, int jg, const float (&zi)[D], int i,
                                       float& a1, float& c1, float& a2, float& c2) {
  float r1 = 0.f, r2 = 0.f;
#pragma unroll 4
  for (int q = 0; q < kMdRun; ++q) {
    float s = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const float dd = zi[a] - tile[a][jl + q];
      s = __builtin_fmaf(dd, dd, s);
    }
    if (MASK) s = (jg + q > i) ? s : __builtin_inff();
    const float e = __builtin_amdgcn_exp2f(-s);
    r1 += e;
    r2 = __builtin_fmaf(e, e, r2);
  }
  md_fold(a1, c1, r1);
  md_fold(a2, c2, r2);
}

// one block per unit of one matrix: part[2 k + {0, 1}][item] of that matrix
template <int D>
__global__ __launch_bounds__(kThreads) void k_HZ_units_f32(const float* __restrict__ z, int npad,
                                                           const MdState* __restrict__ st,
                                                           const Unit* __restrict__ units, int u0,
                                                           double* __restrict__ part, int n_items) {
  if (st->status != kStOk) return;
  const Unit u = units[u0 + blockIdx.x];
  const int n = st->n;
  __shared__ float tile[D][kBJ];
  __shared__ double red[4][2];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = u.row * kBI;
  const int i = row0 + tid;
  float zi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) zi[a] = (i < n) ? z[(int64_t)a * npad + i] : 0.f;
  const int wave_i0 = row0 + wave * 64;
  float a1 = 0.f, c1 = 0.f, a2 = 0.f, c2 = 0.f;
  for (int t0 = u.j_begin; t0 < u.j_end; t0 += kBJ) {
    __syncthreads();
    for (int a = 0; a < D; ++a)
      for (int q = tid; q < kBJ; q += kThreads) tile[a][q] = z[(int64_t)a * npad + t0 + q];
    __syncthreads();
    int js = max(t0, wave_i0);
    const int te = t0 + kBJ;
    if (js < te) {
      if (js == wave_i0) {
        hz_run<D, true>(tile, js - t0, js, zi, i, a1, c1, a2, c2);
        js += kMdRun;
      }
      for (; js < te; js += kMdRun) hz_run<D, false>(tile, js - t0, js, zi, i, a1, c1, a2, c2);
    }
  }
  const bool valid = i < n;
  const double v1 = md_wave_sum(valid ? (double)a1 - (double)c1 : 0.0);
  const double v2 = md_wave_sum(valid ? (double)a2 - (double)c2 : 0.0);
  if (lane == 0) {
    red[wave][0] = v1;
    red[wave][1] = v2;
  }
  __syncthreads();
  if (tid < 2) part[(int64_t)tid * n_items + u.item] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

// The same sweep for wide samples (D = 8, 16), where the LDS reads of the
// tile (D per pair) become the limit: the j coordinates are the same for
// every lane of a wave, so they are read with uniform addresses (scalar
// loads through the scalar cache) and enter the arithmetic as scalar
// operands, with no tile and no barrier.  Measured at n = 1e5, d = 8: 20%
// faster than the tiled kernel; at D <= 3 the tiled kernel is faster.
template <int D, bool MASK>
__device__ __forceinline__ void hz_run_s(const float* __restrict__ z, int npad, int jg, const float (&zi)[D], int i,
                                       float& a1, float& c1, float& a2, float& c2) {
  float r1 = 0.f, r2 = 0.f;
#pragma unroll 8
  for (int q = 0; q < kMdRun; ++q) {
    float s = 0.f;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const float dd = zi[a] - z[(int64_t)a * npad + jg + q];
      s = __builtin_fmaf(dd, dd, s);
    }
    if (MASK) s = (jg + q > i) ? s : __builtin_inff();
    const float e = __builtin_amdgcn_exp2f(-s);
    r1 += e;
    r2 = __builtin_fmaf(e, e, r2);
  }
  md_fold(a1, c1, r1);
  md_fold(a2, c2, r2);
}

template <int D>
__global__ __launch_bounds__(kThreads) void k_HZ_units_f32s(const float* __restrict__ z, int npad,
                                                           const MdState* __restrict__ st,
                                                           const Unit* __restrict__ units, int u0,
                                                           double* __restrict__ part, int n_items) {
  if (st->status != kStOk) return;
  const Unit u = units[u0 + blockIdx.x];
  const int n = st->n;
  __shared__ double red[4][2];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = u.row * kBI;
  const int i = row0 + tid;
  float zi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) zi[a] = (i < n) ? z[(int64_t)a * npad + i] : 0.f;
  const int wave_i0 = __builtin_amdgcn_readfirstlane(row0 + wave * 64);
  float a1 = 0.f, c1 = 0.f, a2 = 0.f, c2 = 0.f;
  int js = __builtin_amdgcn_readfirstlane(max(u.j_begin, wave_i0));
  const int je = __builtin_amdgcn_readfirstlane(u.j_end);
  if (js < je && js == wave_i0) {
    hz_run_s<D, true>(z, npad, js, zi, i, a1, c1, a2, c2);
    js += kMdRun;
  }
  for (; js < je; js += kMdRun) hz_run_s<D, false>(z, npad, js, zi, i, a1, c1, a2, c2);
  const bool valid = i < n;
  const double v1 = md_wave_sum(valid ? (double)a1 - (double)c1 : 0.0);
  const double v2 = md_wave_sum(valid ? (double)a2 - (double)c2 : 0.0);
  if (lane == 0) {
    red[wave][0] = v1;
    red[wave][1] = v2;
  }
  __syncthreads();
  if (tid < 2) part[(int64_t)tid * n_items + u.item] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

template <int D>
__global__ __launch_bounds__(kThreads) void k_HZ_units_f64(const double* __restrict__ z, int npad,
                                                           const MdState* __restrict__ st,
                                                           const Unit* __restrict__ units, int u0,
                                                           double* __restrict__ part, int n_items) {
  if (st->status != kStOk) return;
  constexpr int kT = kBJ / 2;
  const Unit u = units[u0 + blockIdx.x];
  const int n = st->n;
  __shared__ double tile[D][kT];
  __shared__ double red[4][2];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i = u.row * kBI + tid;
  double zi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) zi[a] = (i < n) ? z[(int64_t)a * npad + i] : 0.0;
  double s1 = 0.0, s2 = 0.0;
  for (int t0 = u.j_begin; t0 < u.j_end; t0 += kT) {
    __syncthreads();
    for (int a = 0; a < D; ++a)
      for (int q = tid; q < kT; q += kThreads) tile[a][q] = z[(int64_t)a * npad + t0 + q];
    __syncthreads();
    const int qa = max(0, i + 1 - t0), qb = min(kT, n - t0);
    for (int q = qa; q < qb; ++q) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double dd = zi[a] - tile[a][q];
        s = fma(dd, dd, s);
      }
      const double e = exp_cw(-s);
      s1 += e;
      s2 = fma(e, e, s2);
    }
  }
  const bool valid = i < n;
  const double v1 = md_wave_sum(valid ? s1 : 0.0);
  const double v2 = md_wave_sum(valid ? s2 : 0.0);
  if (lane == 0) {
    red[wave][0] = v1;
    red[wave][1] = v2;
  }
  __syncthreads();
  if (tid < 2) part[(int64_t)tid * n_items + u.item] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

// g(H) = 2 n^-2 (A S1 - 2 B S2) + n^-1 R with A = (4 pi)^(-d/2) |H|^(-1/2),
// B = (2 pi)^(-d/2) |H|^(-1/2), R = 2^-d pi^(-d/2) |H|^(-1/2) (eq. LSCV_MULTI-gh
// with LSCV_MULTI-Kx, -KKx, -rk), and the scale of its terms
// 2 n^-2 (A S1 + 2 B S2) + n^-1 R; +inf (scale 0) for a matrix that is not
// positive definite, NaN when the samples were rejected
__global__ void k_H_final(const MdState* st, const HDesc* hd, int m, const double* sums, double* g, double* gs) {
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
  const double sq = exp(-0.5 * hd[k].logdet);
  const double A = pow(4.0 * kPiD, -0.5 * d) * sq, B = pow(2.0 * kPiD, -0.5 * d) * sq;
  const double R = pow(2.0, -(double)d) * pow(kPiD, -0.5 * d) * sq;
  g[k] = 2.0 / (n * n) * (A * sums[2 * k] - 2.0 * B * sums[2 * k + 1]) + R / n;
  gs[k] = 2.0 / (n * n) * (A * sums[2 * k] + 2.0 * B * sums[2 * k + 1]) + R / n;
}

void launch_HZ(hipStream_t s, int D, bool f64, const float* z32, const double* z64, int npad, const MdState* st,
               const Unit* units, int u0, int cnt, double* part, int n_items) {
#define KDE_HZ_CASE(DD)                                                                                  \
  if (f64)                                                                                               \
    k_HZ_units_f64<DD><<<cnt, kThreads, 0, s>>>(z64, npad, st, units, u0, part, n_items);                \
  else if constexpr (DD >= 8)                                                                            \
    k_HZ_units_f32s<DD><<<cnt, kThreads, 0, s>>>(z32, npad, st, units, u0, part, n_items);               \
  else                                                                                                   \
    k_HZ_units_f32<DD><<<cnt, kThreads, 0, s>>>(z32, npad, st, units, u0, part, n_items);                \
  return
  switch (D) {
    case 2: KDE_HZ_CASE(2);
    case 3: KDE_HZ_CASE(3);
    case 4: KDE_HZ_CASE(4);
    case 8: KDE_HZ_CASE(8);
    default: KDE_HZ_CASE(16);
  }
#undef KDE_HZ_CASE
}

}  // namespace

// ---- LSCV_H on the host side: staging once per call (moments, Sigma, its
// Cholesky factor), then passes of at most kHPass matrices each (prep, per
// matrix a whitening and a sweep, row reduction, finalize).
namespace {

constexpr int kHPass = 64;

struct HRun {
  kde_ctx* c = nullptr;
  int n = 0, d = 0, D = 0, npad = 0, n_items = 0;
  bool f64 = false;
  const void* raw = nullptr;  // the samples on the device
  bool raw_f64 = false;
  std::vector<double> pairs;  // per item
  char* b = nullptr;
  size_t o_st = 0, o_y32 = 0, o_y64 = 0, o_hin = 0, o_hd = 0, o_part = 0, o_sums = 0, o_g = 0, o_gs = 0,
         o_units = 0, o_rows = 0, o_hm = 0;
  MdState state{};
  int passes = 0;
};

// Item length of an LSCV_H pass: about 8192 blocks for a single matrix
// (an explicit "seg" option wins).
int64_t h_seg(const kde_ctx* c, int64_t n) {
  if (c->opt_seg >= 0) return pick_seg(c, n, 1);
  int64_t seg = (int64_t)(0.5 * (double)n * (double)n / 8192.0 / kBI) / kBJ * kBJ;
  seg = std::max<int64_t>(kBJ, seg);
  return seg >= n ? 0 : seg;
}

// Stages the samples into `buf` (the context's workspace, or a prepared
// handle's own buffer); with own_samples the samples are copied into it even
// when they are on the device, so the staged state outlives the caller's.
kde_status h_stage(kde_ctx* c, const kde_matrix& x, HRun& r, DevBuf<char>& buf, bool own_samples) {
  if (!x.data || x.n < 2 || x.n > KDE_MAX_N || x.d < 1 || x.d > KDE_MAX_D ||
      (x.dtype != KDE_F32 && x.dtype != KDE_F64))
    return fail(c, KDE_E_INVAL, "need a row-major n x d matrix, 2 <= n <= KDE_MAX_N, 1 <= d <= KDE_MAX_D");
  r.c = c;
  r.f64 = c->prec == KDE_PREC_FP64;
  r.n = (int)x.n;
  r.d = x.d;
  r.D = md_width(r.d);
  r.npad = r.n + kPad;
  const int n = r.n, d = r.d, D = r.D;
  const int esz = x.dtype == KDE_F64 ? 8 : 4;
  const int nblk = std::min(kMdBlocks, std::max(1, (n + 2047) / 2048));
  ColItems items;
  make_items(n, h_seg(c, n), items);
  r.n_items = (int)items.pairs.size();
  r.pairs = items.pairs;
  // one unit per item (each matrix's sweep launches all of them)
  std::vector<Unit> units;
  units.reserve(r.n_items);
  for (int it = 0; it < r.n_items; ++it) units.push_back(Unit{0, items.row[it], items.jb[it], items.je[it], it, 0});
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t o = at;
    at += al256(bytes);
    return o;
  };
  const bool copy_raw = !x.on_device || own_samples;
  const size_t o_raw = copy_raw ? take((size_t)n * d * esz) : 0;
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
  r.o_hm = take(8 * (size_t)kHPass * KDE_MAX_D * KDE_MAX_D);
  kde_status s;
  if ((s = ensure(c, buf, at))) return s;
  char* b = r.b = buf.p;
  double* part = (double*)(b + r.o_part);
  double* sums = (double*)(b + r.o_sums);
  std::vector<RowDesc> rows;
  for (int q = 0; q < 2 * kHPass; ++q) rows.push_back(RowDesc{part + (size_t)q * r.n_items, sums + q, r.n_items, 0});
  hipStream_t st = c->stream;
  const void* raw = r.raw = copy_raw ? (const void*)(b + o_raw) : x.data;
  r.raw_f64 = x.dtype == KDE_F64;
  if (copy_raw)
    KDE_HIP_TRY(c, hipMemcpyAsync(b + o_raw, x.data, (size_t)n * d * esz,
                                  x.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
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
  kde_status s;
  char* b = r.b;
  const MdState* dst = (const MdState*)(b + r.o_st);
  const HDesc* hd = (const HDesc*)(b + r.o_hd);
  const double* hm = (const double*)(b + r.o_hm);
  double* part = (double*)(b + r.o_part);
  float* z32 = r.f64 ? nullptr : (float*)(b + r.o_y32);
  double* z64 = r.f64 ? (double*)(b + r.o_y64) : nullptr;
  KDE_HIP_TRY(c, hipMemcpyAsync(b + r.o_hin, H, 8 * (size_t)m * r.d * r.d, hipMemcpyHostToDevice, st));
  k_H_prep<<<1, kHPass, 0, st>>>(dst, (const double*)(b + r.o_hin), m, r.f64 ? 1 : 0, (HDesc*)(b + r.o_hd),
                                 (double*)hm);
  // launches of at most launch_evals pair-term evaluations and at least 2048 blocks
  const double budget = r.f64 ? c->opt_launch_evals / 5.0 : c->opt_launch_evals;
  for (int k = 0; k < m; ++k) {
    md_whiten(st, r.raw, r.raw_f64, r.n, r.D, r.npad, dst, hm + (size_t)k * KDE_MAX_D * KDE_MAX_D, z32, z64);
    for (size_t u0 = 0; u0 < (size_t)r.n_items;) {
      double acc = r.pairs[u0];
      size_t u1 = u0 + 1;
      while (u1 < (size_t)r.n_items && (acc + r.pairs[u1] <= budget || u1 - u0 < 2048)) acc += r.pairs[u1++];
      kde_ctx::Pending pd{nullptr, nullptr, kFamMd, acc};
      if ((s = timed_begin(c, pd))) return s;
      launch_HZ(st, r.D, r.f64, z32, z64, r.npad, dst, (const Unit*)(b + r.o_units), (int)u0, (int)(u1 - u0),
                part + (size_t)2 * k * r.n_items, r.n_items);
      if ((s = timed_end(c, pd))) return s;
      u0 = u1;
    }
  }
  launch_reduce_rows(st, (const RowDesc*)(b + r.o_rows), 2 * m);
  k_H_final<<<1, kHPass, 0, st>>>(dst, hd, m, (const double*)(b + r.o_sums), (double*)(b + r.o_g),
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

}  // namespace kde

// A prepared sample for repeated g(H) evaluations: the staged, sphered
// samples, Sigma and the pass layout, in a device buffer of the handle's own
// (the caller's samples are copied in), so calls on the context in between
// do not disturb it.
struct kde_lscv_H_prep {
  kde_ctx* c = nullptr;
  kde::HRun r;
  kde::DevBuf<char> buf;
};

namespace {

kde_status check_H(kde_ctx* c, int d, const double* H, int32_t m) {
  if (m < 1 || m > KDE_MAX_H_EVAL) return kde::fail(c, KDE_E_INVAL, "matrix count outside [1, KDE_MAX_H_EVAL]");
  if (d >= 1 && d <= KDE_MAX_D)
    for (int64_t q = 0; q < (int64_t)m * d * d; ++q)
      if (!std::isfinite(H[q])) return kde::fail(c, KDE_E_INVAL, "bandwidth matrix holds a non-finite value");
  return KDE_OK;
}

}  // namespace

extern "C" {

kde_status kde_lscv_H_prepare(kde_ctx* c, kde_matrix x, kde_lscv_H_prep** out) {
  if (!c || !out) return KDE_E_INVAL;
  *out = nullptr;
  if (c->server && kde::server_running(c->server.get())) return kde::fail(c, KDE_E_BUSY, "a server is running");
  if (hipSetDevice(c->device) != hipSuccess) return kde::fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  std::unique_ptr<kde_lscv_H_prep> p(new kde_lscv_H_prep());
  p->c = c;
  kde_status s = kde::h_stage(c, x, p->r, p->buf, true);
  if (s) {
    if (p->buf.p) (void)hipFree(p->buf.p);
    return s;
  }
  c->preps.push_back(p.get());
  *out = p.release();
  return KDE_OK;
}

kde_status kde_lscv_H_eval_prepared(kde_lscv_H_prep* p, const double* H, int32_t m, double* g_out,
                                    double* gscale_out) {
  if (!p || !g_out || !H) return KDE_E_INVAL;
  kde_ctx* c = p->c;
  if (c->server && kde::server_running(c->server.get())) return kde::fail(c, KDE_E_BUSY, "a server is running");
  if ((c->prec == KDE_PREC_FP64) != p->r.f64)
    return kde::fail(c, KDE_E_INVAL, "the context's precision changed since the sample was prepared");
  kde_status s = check_H(c, p->r.d, H, m);
  if (s) return s;
  if (hipSetDevice(c->device) != hipSuccess) return kde::fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  return kde::h_eval(p->r, H, m, g_out, gscale_out);
}

void kde_lscv_H_release(kde_lscv_H_prep* p) {
  if (!p) return;
  kde_ctx* c = p->c;
  auto& v = c->preps;
  v.erase(std::remove(v.begin(), v.end(), p), v.end());
  (void)hipSetDevice(c->device);
  if (p->buf.p) (void)hipFree(p->buf.p);
  delete p;
}

kde_status kde_lscv_H_eval(kde_ctx* c, kde_matrix x, const double* H, int32_t m, double* g_out,
                           double* gscale_out) {
  if (!c || !g_out || !H) return KDE_E_INVAL;
  if (c->server && kde::server_running(c->server.get())) return kde::fail(c, KDE_E_BUSY, "a server is running");
  kde_status s0 = check_H(c, x.d, H, m);
  if (s0) return s0;
  if (hipSetDevice(c->device) != hipSuccess) return kde::fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde::HRun r;
  kde_status s = kde::h_stage(c, x, r, c->mdbuf, false);
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
  kde_status s = kde::h_stage(c, x, r, c->mdbuf, false);
  if (s) return s;
  return kde::h_search(r, ftol, xtol, max_evals, H_out, info);
}


}  // extern "C"
