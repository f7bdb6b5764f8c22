// kde_query_md.hip -- the estimate's consumers for d-dimensional samples:
// the density with a bandwidth matrix at query points (eq. kde-def-H) and
// 2-D range COUNT/SUM/AVG over boxes (eq. count-sum-2D).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "kde_md.h"

namespace kde {

namespace {

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
          s64 += exp_cw(-0.5 * d2);
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
  const bool fx = x.dtype == KDE_F64;
  md_moments(st, raw, fx, n, d, nblk, (double*)(b + o_ps), (int*)(b + o_nf), dst);
  k_dq_factor<<<1, 64, 0, st>>>(dst, (const double*)(b + o_H));
  double* y = (double*)(b + o_y);
  double* zq = (double*)(b + o_zq);
  md_whiten(st, raw, fx, n, D, npad, dst, dst->linv, nullptr, y);
  md_whiten(st, b + o_qr, true, m, D, mpad, dst, dst->linv, nullptr, zq);
  const dim3 grid(qblocks, pieces);
  double* part = (double*)(b + o_part);
  kde_ctx::Pending pd{nullptr, nullptr, kFamMd, (double)m * (double)n};
  if ((s = timed_begin(c, pd))) return s;
  switch (D) {
    case 2: launch_dq<2>(st, f64, grid, zq, m, mpad, y, npad, dst, piece_len, pieces, part); break;
    case 3: launch_dq<3>(st, f64, grid, zq, m, mpad, y, npad, dst, piece_len, pieces, part); break;
    case 4: launch_dq<4>(st, f64, grid, zq, m, mpad, y, npad, dst, piece_len, pieces, part); break;
    case 8: launch_dq<8>(st, f64, grid, zq, m, mpad, y, npad, dst, piece_len, pieces, part); break;
    default: launch_dq<16>(st, f64, grid, zq, m, mpad, y, npad, dst, piece_len, pieces, part); break;
  }
  if ((s = timed_end(c, pd))) return s;
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
  md_moments(st, raw, fx != 0, n, 2, nblk, (double*)(b + o_ps), (int*)(b + o_nf), dst);
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
