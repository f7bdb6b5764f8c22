// kde_query.hip -- the estimate's consumers: the density at query points and
// approximate range aggregates (Section 3.2: COUNT, SUM and AVG over a range
// of a numeric column from the estimated PDF), at a bandwidth chosen by the
// selectors.
//
// Density, eq. (kde-def) with d = 1 and the Gaussian kernel:
//   f(x) = (n h)^-1 sum_i phi((x - X_i) / h).
// A block holds 256 query points, one per lane, and sweeps a piece of the
// column in 512-sample LDS tiles (broadcast reads, as in the pair kernels);
// mixed form: FP32 terms via exp2 in 64-term runs folded into a compensated
// FP32 sum, FP64 across pieces, the query point carried as an FP32 pair so
// its own rounding does not shift the estimate; FP64 form: every term in
// FP64.  Padding samples hold +inf and contribute exactly zero.
//
// Range aggregates, eq. (count) and eq. (sum) with the estimate for f: the
// Gaussian kernel integrates in closed form, so for a range [a, b]
//   Count = n int_a^b f = sum_i [Phi(beta_i) - Phi(alpha_i)],
//   Sum   = n int_a^b x f = sum_i [X_i (Phi(beta_i) - Phi(alpha_i)) + h (phi(alpha_i) - phi(beta_i))],
// alpha_i = (a - X_i)/h, beta_i = (b - X_i)/h, and AVG = Sum / Count.  The
// differences of Phi are taken between tails (erfc) so that ranges far from a
// sample lose no digits; everything is FP64 (O(n) terms per range).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "kde_runtime.h"

namespace kde {

namespace {

constexpr double kLog2E = 1.4426950408889634074;
constexpr double kInvSqrt2Pi = 0.39894228040143267794;
constexpr double kInvSqrt2 = 0.70710678118654752440;
constexpr int kRunQ = 64;  // samples per plain-FP32 run before a compensated fold

__device__ __forceinline__ void fold(float& a, float& comp, float v) {
  const float y = v - comp;
  const float t = a + y;
  comp = (t - a) - y;
  a = t;
}

__device__ __forceinline__ double block_sum_q(double v, double* sh) {
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

// grid (query blocks, pieces); part[q * pieces + piece]
__global__ __launch_bounds__(kThreads) void k_density_f32(const ColDesc* __restrict__ col,
                                                          const double* __restrict__ q, int m, double h, int piece_len,
                                                          int pieces, double* __restrict__ part) {
  const ColDesc c = *col;
  const float* x = c.x32;
  const int qi = blockIdx.x * kThreads + threadIdx.x;
  // the query point as an FP32 pair (hi + lo): the sample differences near it
  // are then exact to FP32 rounding of the difference, not of the point
  const double xq64 = qi < m ? q[qi] - c.st->shift : 0.0;
  const float xq = (float)xq64;
  const float xl = (float)(xq64 - (double)xq);
  const float cf = (float)(-kLog2E / (2.0 * h * h));
  const int n_pad = (c.n + kBJ - 1) / kBJ * kBJ;
  const int j0 = blockIdx.y * piece_len;
  const int j1 = min(j0 + piece_len, n_pad);
  __shared__ float4 tile[kBJ / 4];
  float a = 0.f, comp = 0.f;
  for (int t0 = j0; t0 < j1; t0 += kBJ) {
    __syncthreads();
    for (int k = threadIdx.x; k < kBJ / 4; k += kThreads) tile[k] = reinterpret_cast<const float4*>(x + t0)[k];
    __syncthreads();
    for (int r0 = 0; r0 < kBJ; r0 += kRunQ) {
      float run = 0.f;
#pragma unroll 4
      for (int k = 0; k < kRunQ / 4; ++k) {
        const float4 v = tile[(r0 >> 2) + k];
        const float d0 = (xq - v.x) + xl, d1 = (xq - v.y) + xl, d2 = (xq - v.z) + xl, d3 = (xq - v.w) + xl;
        run += __builtin_amdgcn_exp2f(d0 * d0 * cf);
        run += __builtin_amdgcn_exp2f(d1 * d1 * cf);
        run += __builtin_amdgcn_exp2f(d2 * d2 * cf);
        run += __builtin_amdgcn_exp2f(d3 * d3 * cf);
      }
      fold(a, comp, run);
    }
  }
  if (qi < m) part[(int64_t)qi * pieces + blockIdx.y] = (double)a - (double)comp;
}

__global__ __launch_bounds__(kThreads) void k_density_f64(const ColDesc* __restrict__ col,
                                                          const double* __restrict__ q, int m, double h, int piece_len,
                                                          int pieces, double* __restrict__ part) {
  const ColDesc c = *col;
  const double* x = c.x64;
  const int qi = blockIdx.x * kThreads + threadIdx.x;
  const double xq = qi < m ? q[qi] : 0.0;
  const double cd = -1.0 / (2.0 * h * h);
  const int n_pad = (c.n + kBJ - 1) / kBJ * kBJ;
  const int j0 = blockIdx.y * piece_len;
  const int j1 = min(j0 + piece_len, n_pad);
  __shared__ double tile[kBJ];
  double s = 0.0;
  for (int t0 = j0; t0 < j1; t0 += kBJ) {
    __syncthreads();
    for (int k = threadIdx.x; k < kBJ; k += kThreads) tile[k] = x[t0 + k];
    __syncthreads();
    for (int k = 0; k < kBJ; ++k) {
      const double d = xq - tile[k];
      s += exp_cw(d * d * cd);
    }
  }
  if (qi < m) part[(int64_t)qi * pieces + blockIdx.y] = s;
}

// block per query point: fixed-order sum over pieces, then the normalisation
__global__ __launch_bounds__(kThreads) void k_density_final(const ColDesc* __restrict__ col,
                                                            const double* __restrict__ part, int pieces, double h,
                                                            double* __restrict__ out) {
  __shared__ double sh[kThreads];
  const int qi = blockIdx.x;
  double s = 0.0;
  for (int p = threadIdx.x; p < pieces; p += kThreads) s += part[(int64_t)qi * pieces + p];
  s = block_sum_q(s, sh);
  if (threadIdx.x == 0) {
    const ColDesc c = *col;
    out[qi] = c.st->status != kStInval ? s * kInvSqrt2Pi / ((double)c.n * h) : NAN;
  }
}

// Upper tail Q(z) = 1 - Phi(z).
__device__ __forceinline__ double upper_tail(double z) { return 0.5 * erfc(z * kInvSqrt2); }

// Phi(beta) - Phi(alpha), alpha <= beta, from the tails on the side away from
// the bulk of the kernel.
__device__ __forceinline__ double phi_diff(double alpha, double beta) {
  if (alpha >= 0.0) return upper_tail(alpha) - upper_tail(beta);
  if (beta <= 0.0) return upper_tail(-beta) - upper_tail(-alpha);
  return 1.0 - upper_tail(-alpha) - upper_tail(beta);
}

__device__ __forceinline__ double std_normal(double z) { return isinf(z) ? 0.0 : kInvSqrt2Pi * exp(-0.5 * z * z); }

// grid (ranges, pieces): one range per block, lanes stride over the piece's samples
__global__ __launch_bounds__(kThreads) void k_range_f64(const ColDesc* __restrict__ col, const double* __restrict__ lo,
                                                        const double* __restrict__ hi, double h, int piece_len,
                                                        int pieces, double* __restrict__ part) {
  const ColDesc c = *col;
  const int r = blockIdx.x;
  const double a = lo[r], b = hi[r];
  const int i0 = blockIdx.y * piece_len;
  const int i1 = min(c.n, i0 + piece_len);
  double cnt = 0.0, sum = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kThreads) {
    const double xi = c.raw_f64 ? reinterpret_cast<const double*>(c.raw)[i]
                                : (double)reinterpret_cast<const float*>(c.raw)[i];
    const double al = (a - xi) / h, be = (b - xi) / h;
    const double dp = phi_diff(al, be);
    cnt += dp;
    sum += xi * dp + h * (std_normal(al) - std_normal(be));
  }
  __shared__ double sh[kThreads];
  cnt = block_sum_q(cnt, sh);
  sum = block_sum_q(sum, sh);
  if (threadIdx.x == 0) {
    part[((int64_t)r * pieces + blockIdx.y) * 2] = cnt;
    part[((int64_t)r * pieces + blockIdx.y) * 2 + 1] = sum;
  }
}

// block per range: fixed-order sums over pieces; AVG = SUM / COUNT
__global__ __launch_bounds__(kThreads) void k_range_final(const ColDesc* __restrict__ col,
                                                          const double* __restrict__ part, int pieces,
                                                          double* __restrict__ out) {
  __shared__ double sh[kThreads];
  const int r = blockIdx.x;
  double cnt = 0.0, sum = 0.0;
  for (int p = threadIdx.x; p < pieces; p += kThreads) {
    cnt += part[((int64_t)r * pieces + p) * 2];
    sum += part[((int64_t)r * pieces + p) * 2 + 1];
  }
  cnt = block_sum_q(cnt, sh);
  sum = block_sum_q(sum, sh);
  if (threadIdx.x == 0) {
    const bool ok = col->st->status != kStInval;
    out[3 * r] = ok ? cnt : NAN;
    out[3 * r + 1] = ok ? sum : NAN;
    out[3 * r + 2] = ok && cnt > 0.0 ? sum / cnt : NAN;
  }
}

// pieces so that a launch has about 4096 blocks, each piece at least 4096 samples
int pieces_for(int64_t n, int64_t other_blocks) {
  const int64_t want = std::max<int64_t>(1, 4096 / std::max<int64_t>(1, other_blocks));
  const int64_t most = std::max<int64_t>(1, n / 4096);
  return (int)std::min(want, most);
}

}  // namespace

}  // namespace kde

namespace {

using kde::fail;

bool finite_all(const double* v, int32_t m) {
  for (int32_t k = 0; k < m; ++k)
    if (!std::isfinite(v[k])) return false;
  return true;
}

}  // namespace

extern "C" {

kde_status kde_density(kde_ctx* c, kde_column x, double h, const double* points, int32_t m, double* f_out) {
  if (!c || !points || !f_out) return KDE_E_INVAL;
  if (c->server && kde::server_running(c->server.get())) return fail(c, KDE_E_BUSY, "a server is running");
  if (!(h > 0.0) || !std::isfinite(h) || m < 1 || m > KDE_MAX_QUERIES || !finite_all(points, m))
    return fail(c, KDE_E_INVAL, "need h > 0 finite, 1 <= m <= KDE_MAX_QUERIES finite points");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  const kde::ColDesc* dcol = nullptr;
  if ((s = kde::stage_column(c, x, &dcol))) return s;
  const bool f64 = c->prec == KDE_PREC_FP64;
  const int n = (int)x.n;
  const int qblocks = (m + kde::kThreads - 1) / kde::kThreads;
  const int n_pad = (n + kde::kBJ - 1) / kde::kBJ * kde::kBJ;
  int pieces = kde::pieces_for(n_pad, qblocks);
  int piece_len = (n_pad + pieces - 1) / pieces;
  piece_len = (piece_len + kde::kBJ - 1) / kde::kBJ * kde::kBJ;
  pieces = (n_pad + piece_len - 1) / piece_len;
  const size_t q_bytes = 8 * (size_t)m, part_bytes = 8 * (size_t)m * pieces;
  if ((s = kde::ensure(c, c->qbuf, q_bytes + part_bytes + q_bytes + 768))) return s;
  char* base = c->qbuf.p;
  double* dq = (double*)base;
  double* dpart = (double*)(base + (q_bytes + 255) / 256 * 256);
  double* dout = (double*)((char*)dpart + (part_bytes + 255) / 256 * 256);
  KDE_HIP_TRY(c, hipMemcpyAsync(dq, points, q_bytes, hipMemcpyHostToDevice, c->stream));
  const dim3 grid(qblocks, pieces);
  if (f64)
    kde::k_density_f64<<<grid, kde::kThreads, 0, c->stream>>>(dcol, dq, m, h, piece_len, pieces, dpart);
  else
    kde::k_density_f32<<<grid, kde::kThreads, 0, c->stream>>>(dcol, dq, m, h, piece_len, pieces, dpart);
  kde::k_density_final<<<m, kde::kThreads, 0, c->stream>>>(dcol, dpart, pieces, h, dout);
  KDE_HIP_TRY(c, hipMemcpyAsync(f_out, dout, q_bytes, hipMemcpyDeviceToHost, c->stream));
  return kde::sync_and_check(c);
}

kde_status kde_range_aggregates(kde_ctx* c, kde_column x, double h, const double* lo, const double* hi, int32_t q,
                                double* count_out, double* sum_out, double* avg_out) {
  if (!c || !lo || !hi || !count_out || !sum_out) return KDE_E_INVAL;
  if (c->server && kde::server_running(c->server.get())) return fail(c, KDE_E_BUSY, "a server is running");
  if (!(h > 0.0) || !std::isfinite(h) || q < 1 || q > KDE_MAX_QUERIES)
    return fail(c, KDE_E_INVAL, "need h > 0 finite and 1 <= q <= KDE_MAX_QUERIES");
  for (int32_t k = 0; k < q; ++k)
    if (std::isnan(lo[k]) || std::isnan(hi[k]) || !(lo[k] <= hi[k]))
      return fail(c, KDE_E_INVAL, "every range needs lo <= hi (infinite ends allowed)");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  kde_status s;
  const kde::ColDesc* dcol = nullptr;
  if ((s = kde::stage_column(c, x, &dcol))) return s;
  const int n = (int)x.n;
  int pieces = kde::pieces_for(n, q);
  const int piece_len = (n + pieces - 1) / pieces;
  pieces = (n + piece_len - 1) / piece_len;
  const size_t r_bytes = 8 * (size_t)q, part_bytes = 16 * (size_t)q * pieces, out_bytes = 24 * (size_t)q;
  if ((s = kde::ensure(c, c->qbuf, 2 * r_bytes + part_bytes + out_bytes + 1024))) return s;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  char* base = c->qbuf.p;
  double* dlo = (double*)base;
  double* dhi = (double*)(base + al(r_bytes));
  double* dpart = (double*)(base + 2 * al(r_bytes));
  double* dout = (double*)(base + 2 * al(r_bytes) + al(part_bytes));
  KDE_HIP_TRY(c, hipMemcpyAsync(dlo, lo, r_bytes, hipMemcpyHostToDevice, c->stream));
  KDE_HIP_TRY(c, hipMemcpyAsync(dhi, hi, r_bytes, hipMemcpyHostToDevice, c->stream));
  kde::k_range_f64<<<dim3(q, pieces), kde::kThreads, 0, c->stream>>>(dcol, dlo, dhi, h, piece_len, pieces, dpart);
  kde::k_range_final<<<q, kde::kThreads, 0, c->stream>>>(dcol, dpart, pieces, dout);
  std::vector<double> out(3 * (size_t)q);
  KDE_HIP_TRY(c, hipMemcpyAsync(out.data(), dout, out_bytes, hipMemcpyDeviceToHost, c->stream));
  if ((s = kde::sync_and_check(c))) return s;
  for (int32_t k = 0; k < q; ++k) {
    count_out[k] = out[3 * (size_t)k];
    sum_out[k] = out[3 * (size_t)k + 1];
    if (avg_out) avg_out[k] = out[3 * (size_t)k + 2];
  }
  return KDE_OK;
}

}  // extern "C"
