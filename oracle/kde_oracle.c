/*
 * kde_oracle.c -- plain FP64 reference for exact KDE bandwidth-selection sums.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU library is
 * compared against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it; the library never links, calls or falls back to it.
 * It shares no code, header, table or constant with the GPU path.
 *
 * Source: Andrzejewski, Gramacki, Gramacki, "Density Estimations for
 * Approximate Query Processing on SIMD Architectures" (arXiv 1505.01998),
 * Section 4.4 (formulas for bandwidth selection).  Every function below cites
 * the equation it writes out.  Sums are exact FP64 sums written as plain loops:
 * each row i of the pair triangle (j > i) is summed in FP64, and the row sums
 * are combined by Neumaier compensated summation in row order, so the result
 * does not depend on the thread count.
 *
 * Readings of the paper taken here (the paper is silent or garbled):
 *  - psi-hat normalisation: the n*K^(r)(0) diagonal term is inside the
 *    1/(n^2 g^(r+1)) factor, i.e. psi_r(g) = n^-2 sum_{i,j} K^(r)_g(X_i-X_j).
 *  - LSCV_h in one dimension is written in data units: the kernel at h is
 *    N(0, h^2); R(K) = (4 pi)^(-1/2).  The paper's LSCV_h takes the bandwidth
 *    matrix h^2 * Sigma (a kernel N(0, h^2 sigma^2) on the data), so its
 *    objective at h is this one at sigma*h: g_paper(h) = g_data(sigma*h).
 *  - variance: two-pass form, equal in exact arithmetic to the one-pass form
 *    of eq. (PLUGIN-VarianceEstimator), same n-1 denominator.
 *  - K^(r) for r = 8 (three-stage plug-in) follows from the Hermite recurrence;
 *    the paper prints only r = 4 and r = 6.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_INVAL 1
#define ORC_DEGENERATE 2
#define ORC_NOMEM 3

static const double ORC_PI = 3.14159265358979323846;

/* Neumaier's improvement of Kahan summation over v[0..m), in index order. */
static double neumaier_sum(const double* v, long m) {
  double s = 0.0, c = 0.0;
  for (long k = 0; k < m; ++k) {
    double t = s + v[k];
    if (fabs(s) >= fabs(v[k]))
      c += (s - t) + v[k];
    else
      c += (v[k] - t) + s;
    s = t;
  }
  return s + c;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* Input check: n >= 2 and every sample finite. */
int orc_validate(const double* x, long n) {
  if (n < 2 || x == NULL) return ORC_INVAL;
  for (long i = 0; i < n; ++i)
    if (!isfinite(x[i])) return ORC_INVAL;
  return ORC_OK;
}

/* Sample mean and variance estimator, eq. (PLUGIN-VarianceEstimator) and
 * (PLUGIN-StdDevEstimator) (also eq. (LSCV-variance) with d = 1).
 * Two-pass: mean first, then sum of squared deviations over n-1. */
int orc_moments(const double* x, long n, double* mean, double* var) {
  int st = orc_validate(x, n);
  if (st) return st;
  double* tmp = (double*)malloc(sizeof(double) * (size_t)n);
  if (!tmp) return ORC_NOMEM;
  memcpy(tmp, x, sizeof(double) * (size_t)n);
  double m = neumaier_sum(tmp, n) / (double)n;
  for (long i = 0; i < n; ++i) tmp[i] = (x[i] - m) * (x[i] - m);
  double v = neumaier_sum(tmp, n) / (double)(n - 1);
  free(tmp);
  *mean = m;
  *var = v;
  return ORC_OK;
}

/* Normal-reference bandwidth.  With d = 1, eq. (LSCV-H-start) gives
 * h = (4/3)^(1/5) n^(-1/5) sigma, the same value as sigma * h0 of
 * eq. (LSCV-h0). */
int orc_rot(const double* x, long n, double* sigma_out, double* h_out) {
  double m, v;
  int st = orc_moments(x, n, &m, &v);
  if (st) return st;
  double s = sqrt(v);
  if (!(s > 0.0)) return ORC_DEGENERATE;
  *sigma_out = s;
  *h_out = pow(4.0 / 3.0, 0.2) * pow((double)n, -0.2) * s;
  return ORC_OK;
}

/* Probabilists' Hermite polynomial He_r(u) by the three-term recurrence
 * He_{k+1}(u) = u He_k(u) - k He_{k-1}(u), He_0 = 1, He_1 = u.
 * K^(r)(u) = He_r(u) phi(u) for the Gaussian kernel; the paper prints
 * He_6 with eq. (PLUGIN-Psi6Estimate) and He_4 with eq. (PLUGIN-Psi4Estimate). */
double orc_hermite_e(int r, double u) {
  double a = 1.0, b = u;
  if (r == 0) return a;
  for (int k = 1; k < r; ++k) {
    double c = u * b - (double)k * a;
    a = b;
    b = c;
  }
  return b;
}

/* r-th derivative of the standard normal density K at u. */
double orc_kernel_deriv(int r, double u) {
  return orc_hermite_e(r, u) * exp(-0.5 * u * u) / sqrt(2.0 * ORC_PI);
}

/* Pair sum of K^(r)((X_i - X_j)/g) over i < j, and of its absolute value.
 * This is the double sum of eq. (PLUGIN-Psi6Estimate)/(PLUGIN-Psi4Estimate). */
int orc_pair_sum_kr(const double* x, long n, int r, double g, double* sum_out, double* abs_out) {
  int st = orc_validate(x, n);
  if (st) return st;
  if (!(g > 0.0) || !isfinite(g)) return ORC_INVAL;
  double* rs = (double*)malloc(sizeof(double) * (size_t)n);
  double* ra = (double*)malloc(sizeof(double) * (size_t)n);
  if (!rs || !ra) { free(rs); free(ra); return ORC_NOMEM; }
#pragma omp parallel for schedule(dynamic, 16)
  for (long i = 0; i < n; ++i) {
    double s = 0.0, a = 0.0;
    for (long j = i + 1; j < n; ++j) {
      double t = orc_kernel_deriv(r, (x[i] - x[j]) / g);
      s += t;
      a += fabs(t);
    }
    rs[i] = s;
    ra[i] = a;
  }
  *sum_out = neumaier_sum(rs, n);
  *abs_out = neumaier_sum(ra, n);
  free(rs);
  free(ra);
  return ORC_OK;
}

/* Functional estimate psi_r(g) = [2 sum_{i<j} K^(r)((X_i-X_j)/g) + n K^(r)(0)]
 *                               / (n^2 g^(r+1)),
 * eq. (PLUGIN-Psi6Estimate) (r = 6) and (PLUGIN-Psi4Estimate) (r = 4), read
 * with the diagonal term inside the normalisation.  kappa = sum|t| / |sum t|
 * over the pair terms (the condition number of the pair sum). */
int orc_psi(const double* x, long n, int r, double g, double* psi_out, double* kappa_out,
            double* pair_sum_out, double* pair_abs_out) {
  double s, a;
  int st = orc_pair_sum_kr(x, n, r, g, &s, &a);
  if (st) return st;
  double nn = (double)n;
  *psi_out = (2.0 * s + nn * orc_kernel_deriv(r, 0.0)) / (nn * nn * pow(g, r + 1));
  if (kappa_out) *kappa_out = (s != 0.0) ? a / fabs(s) : INFINITY;
  if (pair_sum_out) *pair_sum_out = s;
  if (pair_abs_out) *pair_abs_out = a;
  return ORC_OK;
}

/* Normal-scale functional psi_r^NS = (-1)^(r/2) r! / ((2 sigma)^(r+1) (r/2)! sqrt(pi)),
 * the value of psi_r for N(0, sigma^2); r = 8 gives eq. (PLUGIN-Psi8Estimate). */
double orc_psi_ns(int r, double sigma) {
  double num = 1.0, den = 1.0;
  for (int k = 2; k <= r; ++k) num *= (double)k;
  for (int k = 2; k <= r / 2; ++k) den *= (double)k;
  double sgn = ((r / 2) % 2 == 0) ? 1.0 : -1.0;
  return sgn * num / (pow(2.0 * sigma, r + 1) * den * sqrt(ORC_PI));
}

/* AMSE pilot bandwidth for estimating psi_r, given an estimate of psi_{r+2}:
 * g = [-2 K^(r)(0) / (mu_2(K) psi_{r+2} n)]^(1/(r+3)), mu_2(K) = 1;
 * eq. (PLUGIN-g1) (r = 6) and (PLUGIN-g2) (r = 4). */
int orc_pilot(int r, double psi_next, long n, double* g_out) {
  double rad = -2.0 * orc_kernel_deriv(r, 0.0) / (psi_next * (double)n);
  if (!(rad > 0.0) || !isfinite(rad)) return ORC_DEGENERATE;
  *g_out = pow(rad, 1.0 / (double)(r + 3));
  return ORC_OK;
}

typedef struct {
  double sigma, h_rot;
  int stages;
  double g[3], psi[3], kappa[3]; /* stage order: psi8, psi6, psi4 */
  double h;
} orc_plugin_info;

/* Direct plug-in selector, Section 4.4.1: variance -> normal-scale psi ->
 * pilot g -> pairwise psi-hat -> ... -> eq. (PLUGIN-Final_h).
 * stages = 2 is the paper's chain (psi_8 by its normal-scale value, then
 * pairwise psi_6 and psi_4); stages = 3 starts one level higher (psi_10
 * normal scale, then pairwise psi_8, psi_6, psi_4).  Unused slots hold NaN. */
int orc_plugin(const double* x, long n, int stages, orc_plugin_info* info) {
  if (stages != 2 && stages != 3) return ORC_INVAL;
  memset(info, 0, sizeof(*info));
  for (int k = 0; k < 3; ++k) info->g[k] = info->psi[k] = info->kappa[k] = NAN;
  info->stages = stages;
  int st = orc_rot(x, n, &info->sigma, &info->h_rot);
  if (st) return st;
  double psi_next;
  if (stages == 3) {
    double g8;
    st = orc_pilot(8, orc_psi_ns(10, info->sigma), n, &g8);
    if (st) return st;
    info->g[0] = g8;
    st = orc_psi(x, n, 8, g8, &info->psi[0], &info->kappa[0], NULL, NULL);
    if (st) return st;
    psi_next = info->psi[0];
  } else {
    psi_next = orc_psi_ns(8, info->sigma);
    info->psi[0] = psi_next;
  }
  double g6, g4;
  st = orc_pilot(6, psi_next, n, &g6);
  if (st) return st;
  info->g[1] = g6;
  st = orc_psi(x, n, 6, g6, &info->psi[1], &info->kappa[1], NULL, NULL);
  if (st) return st;
  st = orc_pilot(4, info->psi[1], n, &g4);
  if (st) return st;
  info->g[2] = g4;
  st = orc_psi(x, n, 4, g4, &info->psi[2], &info->kappa[2], NULL, NULL);
  if (st) return st;
  double rk = 1.0 / (2.0 * sqrt(ORC_PI));
  double rad = rk / (info->psi[2] * (double)n);
  if (!(rad > 0.0) || !isfinite(rad)) return ORC_DEGENERATE;
  info->h = pow(rad, 0.2);
  return ORC_OK;
}

/* Default LSCV grid: n_h points (150 when n_h <= 0) spaced linearly over
 * sigma * Z(h0) = sigma * [h0/4, 4 h0], eq. (LSCV-Zh0), with
 * h0 = (4/(3n))^(1/5), eq. (LSCV-h0) for d = 1. */
int orc_default_grid(const double* x, long n, int n_h, double* grid_out) {
  double s, hr;
  int st = orc_rot(x, n, &s, &hr);
  if (st) return st;
  if (n_h <= 0) n_h = 150;
  double lo = hr / 4.0, hi = 4.0 * hr;
  for (int k = 0; k < n_h; ++k)
    grid_out[k] = (n_h == 1) ? lo : lo + (hi - lo) * (double)k / (double)(n_h - 1);
  return ORC_OK;
}

/* LSCV objective, eq. (LSCV-gh) with eq. (LSCV-Tx), (LSCV-Kx), (LSCV-KKx), in
 * data units for d = 1:
 *   g(h) = h^-1 [ 2 n^-2 sum_{i<j} T((X_i - X_j)/h) + n^-1 R(K) ],
 *   T(u) = (K*K)(u) - 2 K(u),  K*K = N(0,2) density,  R(K) = (4 pi)^(-1/2).
 * A = sum (4pi)^(-1/2) exp(-D^2/(4h^2)), B = sum (2pi)^(-1/2) exp(-D^2/(2h^2))
 * are computed with separate exp calls; g = h^-1 [2 n^-2 (A - 2B) + n^-1 R(K)].
 * gscale(h) is the same expression with A + 2B: the magnitude g is a
 * difference of, used to express errors in g relative to its terms.
 * Optional outputs a_out / b_out receive the pair sums of exp(-D^2/(4h^2)) and
 * exp(-D^2/(2h^2)) without the constant factors. */
int orc_lscv_curve(const double* x, long n, const double* grid, int n_h, double* g_out,
                   double* gscale_out, double* a_out, double* b_out) {
  int st = orc_validate(x, n);
  if (st) return st;
  if (n_h < 1 || grid == NULL) return ORC_INVAL;
  for (int k = 0; k < n_h; ++k) {
    if (!(grid[k] > 0.0) || !isfinite(grid[k])) return ORC_INVAL;
    if (k > 0 && !(grid[k] > grid[k - 1])) return ORC_INVAL;
  }
  double* ra = (double*)malloc(sizeof(double) * (size_t)n);
  double* rb = (double*)malloc(sizeof(double) * (size_t)n);
  if (!ra || !rb) { free(ra); free(rb); return ORC_NOMEM; }
  double nn = (double)n;
  double c_kk = 1.0 / sqrt(4.0 * ORC_PI), c_k = 1.0 / sqrt(2.0 * ORC_PI);
  for (int k = 0; k < n_h; ++k) {
    double h = grid[k];
#pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < n; ++i) {
      double sa = 0.0, sb = 0.0;
      for (long j = i + 1; j < n; ++j) {
        double d = x[i] - x[j];
        sa += exp(-d * d / (4.0 * h * h));
        sb += exp(-d * d / (2.0 * h * h));
      }
      ra[i] = sa;
      rb[i] = sb;
    }
    double s1 = neumaier_sum(ra, n), s2 = neumaier_sum(rb, n);
    double A = c_kk * s1, B = c_k * s2;
    g_out[k] = (2.0 / (nn * nn) * (A - 2.0 * B) + c_kk / nn) / h;
    if (gscale_out) gscale_out[k] = (2.0 / (nn * nn) * (A + 2.0 * B) + c_kk / nn) / h;
    if (a_out) a_out[k] = s1;
    if (b_out) b_out[k] = s2;
  }
  free(ra);
  free(rb);
  return ORC_OK;
}

/* The two LSCV pair sums of eq. (LSCV-gh) restricted to one block of the
 * i < j triangle: i in [i0, i1), j in [j0, j1), pairs with j <= i or an index
 * >= n excluded.  s1 sums exp(-D^2/(4h^2)), s2 sums exp(-D^2/(2h^2)), with
 * separate exp calls, per grid point.  Summing the blocks of any partition of
 * the triangle gives the sums of orc_lscv_curve. */
int orc_lscv_block_sums(const double* x, long n, long i0, long i1, long j0, long j1, const double* grid, int n_h,
                        double* s1_out, double* s2_out) {
  int st = orc_validate(x, n);
  if (st) return st;
  if (n_h < 1 || grid == NULL || i0 < 0 || j0 < 0) return ORC_INVAL;
  if (i1 > n) i1 = n;
  if (j1 > n) j1 = n;
  long rows = (i1 > i0) ? i1 - i0 : 0;
  double* ra = (double*)malloc(sizeof(double) * (size_t)(rows > 0 ? rows : 1));
  double* rb = (double*)malloc(sizeof(double) * (size_t)(rows > 0 ? rows : 1));
  if (!ra || !rb) { free(ra); free(rb); return ORC_NOMEM; }
  for (int k = 0; k < n_h; ++k) {
    double h = grid[k];
#pragma omp parallel for schedule(dynamic, 1)
    for (long r = 0; r < rows; ++r) {
      long i = i0 + r;
      long jb = (j0 > i + 1) ? j0 : i + 1;
      double sa = 0.0, sb = 0.0;
      for (long j = jb; j < j1; ++j) {
        double d = x[i] - x[j];
        sa += exp(-d * d / (4.0 * h * h));
        sb += exp(-d * d / (2.0 * h * h));
      }
      ra[r] = sa;
      rb[r] = sb;
    }
    s1_out[k] = neumaier_sum(ra, rows);
    s2_out[k] = neumaier_sum(rb, rows);
  }
  free(ra);
  free(rb);
  return ORC_OK;
}

/* Brute-force grid minimum, eq. (LSCV-finalH): lowest index among equal
 * minima; at_edge = 1 when it is the first or last grid point; margin is the
 * gap to the second-smallest value (0 if n_h == 1). */
int orc_argmin(const double* g, int n_h, int* k_out, int* at_edge, double* margin) {
  if (n_h < 1) return ORC_INVAL;
  int kb = 0;
  for (int k = 1; k < n_h; ++k)
    if (g[k] < g[kb]) kb = k;
  double second = INFINITY;
  for (int k = 0; k < n_h; ++k)
    if (k != kb && g[k] < second) second = g[k];
  *k_out = kb;
  if (at_edge) *at_edge = (kb == 0 || kb == n_h - 1) ? 1 : 0;
  if (margin) *margin = (n_h > 1) ? second - g[kb] : 0.0;
  return ORC_OK;
}

/* LSCV selector: the grid point minimising g(h). */
int orc_lscv(const double* x, long n, const double* grid, int n_h, double* h_out, int* k_out,
             int* at_edge) {
  double* g = (double*)malloc(sizeof(double) * (size_t)(n_h > 0 ? n_h : 1));
  if (!g) return ORC_NOMEM;
  int st = orc_lscv_curve(x, n, grid, n_h, g, NULL, NULL, NULL);
  if (!st) {
    int k;
    st = orc_argmin(g, n_h, &k, at_edge, NULL);
    if (!st) {
      *h_out = grid[k];
      if (k_out) *k_out = k;
    }
  }
  free(g);
  return st;
}

/* LSCV bandwidth by search (Section 4.4.2 names a golden-ratio type search as
 * the alternative to the brute-force grid).  Each step evaluates g(h) at m
 * points spaced evenly in log h over the bracket [a, b], ends included, takes
 * the smallest (lowest index on ties) and narrows the bracket to its two
 * neighbours, until b/a - 1 <= tol.  Returns the best point of the last step,
 * its g, the steps taken and the last bracket. */
int orc_lscv_min(const double* x, long n, double lo, double hi, double tol, int m, double* h_out, double* g_out,
                 int* steps_out, double* a_out, double* b_out) {
  if (!(lo > 0.0) || !(hi > lo) || !isfinite(hi) || !(tol > 0.0) || m < 4) return ORC_INVAL;
  double* grid = (double*)malloc(sizeof(double) * (size_t)m);
  double* g = (double*)malloc(sizeof(double) * (size_t)m);
  if (!grid || !g) {
    free(grid);
    free(g);
    return ORC_NOMEM;
  }
  double a = lo, b = hi, hb = 0.0, gb = 0.0;
  int steps = 0, st = ORC_OK;
  for (; steps < 200; ++steps) {
    for (int j = 0; j < m; ++j) grid[j] = a * pow(b / a, (double)j / (double)(m - 1));
    grid[m - 1] = b;
    int ascending = 1;
    for (int j = 1; j < m; ++j) ascending = ascending && grid[j] > grid[j - 1];
    if (!ascending) break;
    st = orc_lscv_curve(x, n, grid, m, g, NULL, NULL, NULL);
    if (st) break;
    int k;
    orc_argmin(g, m, &k, NULL, NULL);
    hb = grid[k];
    gb = g[k];
    if (b / a - 1.0 <= tol) {
      ++steps;
      break;
    }
    const double na = grid[k > 0 ? k - 1 : 0], nb = grid[k < m - 1 ? k + 1 : m - 1];
    a = na;
    b = nb;
  }
  free(grid);
  free(g);
  if (st) return st;
  *h_out = hb;
  if (g_out) *g_out = gb;
  if (steps_out) *steps_out = steps;
  if (a_out) *a_out = a;
  if (b_out) *b_out = b;
  return ORC_OK;
}

/* Density estimate at m points, eq. (kde-def) with d = 1 and the Gaussian
 * kernel of eq. (gaussian): f(p) = (n h)^-1 sum_i phi((p - X_i)/h).  Each
 * point's sum is a Neumaier-compensated FP64 sum in sample order. */
int orc_density(const double* x, long n, double h, const double* pts, int m, double* out) {
  int st = orc_validate(x, n);
  if (st) return st;
  if (!(h > 0.0) || !isfinite(h) || m < 1) return ORC_INVAL;
  const double norm = 1.0 / ((double)n * h * sqrt(2.0 * ORC_PI));
#pragma omp parallel for schedule(dynamic, 16)
  for (int k = 0; k < m; ++k) {
    double s = 0.0, c = 0.0;
    for (long i = 0; i < n; ++i) {
      const double u = (pts[k] - x[i]) / h;
      const double t = exp(-0.5 * u * u);
      const double y = s + t;
      c += (fabs(s) >= fabs(t)) ? (s - y) + t : (t - y) + s;
      s = y;
    }
    out[k] = (s + c) * norm;
  }
  return ORC_OK;
}

/* Approximate range aggregates over [lo, hi] (Section 3.2, eq. (count) and
 * eq. (sum)) with the density estimate for f.  With the Gaussian kernel the
 * integrals are closed forms: n int_lo^hi f = sum_i [Phi(b_i) - Phi(a_i)] and
 * n int_lo^hi x f = sum_i [X_i (Phi(b_i) - Phi(a_i)) + h (phi(a_i) - phi(b_i))],
 * a_i = (lo - X_i)/h, b_i = (hi - X_i)/h, Phi(z) = erfc(-z/sqrt 2)/2. */
int orc_range_aggregates(const double* x, long n, double h, const double* lo, const double* hi, int q,
                         double* count_out, double* sum_out) {
  int st = orc_validate(x, n);
  if (st) return st;
  if (!(h > 0.0) || !isfinite(h) || q < 1) return ORC_INVAL;
  for (int k = 0; k < q; ++k)
    if (isnan(lo[k]) || isnan(hi[k]) || !(lo[k] <= hi[k])) return ORC_INVAL;
  const double inv_sqrt2 = 1.0 / sqrt(2.0), inv_sqrt2pi = 1.0 / sqrt(2.0 * ORC_PI);
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < q; ++k) {
    double cnt = 0.0, sum = 0.0;
    for (long i = 0; i < n; ++i) {
      const double a = (lo[k] - x[i]) / h, b = (hi[k] - x[i]) / h;
      const double dphi = 0.5 * erfc(-b * inv_sqrt2) - 0.5 * erfc(-a * inv_sqrt2);
      const double pa = isinf(a) ? 0.0 : inv_sqrt2pi * exp(-0.5 * a * a);
      const double pb = isinf(b) ? 0.0 : inv_sqrt2pi * exp(-0.5 * b * b);
      cnt += dphi;
      sum += x[i] * dphi + h * (pa - pb);
    }
    count_out[k] = cnt;
    sum_out[k] = sum;
  }
  return ORC_OK;
}

/* ---- LSCV_h for d >= 1 (Section 4.4.2, the sphered form of eq. (LSCV-gh)):
 * x is row-major n x d.  Sigma from eq. (LSCV-variance)/(LSCV-covariance)
 * written two-pass (mean first), S(v) = v^T Sigma^-1 v of eq. (LSCV_MOD-Pv)
 * evaluated as its double sum for every pair, and
 *   g(h) = h^-d [2 n^-2 sum_{i<j} ((K*K)~(v) - 2 K~(v)) + n^-1 R(K)]
 * with K~, (K*K)~ of eq. (LSCV_MOD-Kv2)/(LSCV_MOD-KKv) (two separate exp
 * calls) and R(K) = (4 pi)^(-d/2) |Sigma|^(-1/2) (eq. LSCV_MULTI-rk with
 * H = Sigma).  Sigma is factored by Cholesky; not positive definite (a pivot
 * at most 1e-12 of its diagonal entry) -> DEGENERATE. */
static int orc_cov_inverse(const double* x, long n, int d, double* inv, double* logdet) {
  double* m = (double*)calloc((size_t)d, sizeof(double));
  double* S = (double*)calloc((size_t)d * d, sizeof(double));
  double* L = (double*)calloc((size_t)d * d, sizeof(double));
  double* Li = (double*)calloc((size_t)d * d, sizeof(double));
  int st = ORC_OK;
  if (!m || !S || !L || !Li) {
    st = ORC_NOMEM;
    goto out;
  }
  for (int a = 0; a < d; ++a) {
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += x[i * d + a];
    m[a] = s / (double)n;
  }
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b) {
      double s = 0.0;
      for (long i = 0; i < n; ++i) s += (x[i * d + a] - m[a]) * (x[i * d + b] - m[b]);
      S[a * d + b] = S[b * d + a] = s / (double)(n - 1);
    }
  /* Cholesky S = L L^T */
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b) {
      double s = S[a * d + b];
      for (int k = 0; k < b; ++k) s -= L[a * d + k] * L[b * d + k];
      if (a == b) {
        /* a pivot below 1e-12 of its diagonal entry: singular to working precision */
        if (!(s > 1e-12 * S[a * d + a]) || !isfinite(s)) {
          st = ORC_DEGENERATE;
          goto out;
        }
        L[a * d + a] = sqrt(s);
      } else {
        L[a * d + b] = s / L[b * d + b];
      }
    }
  *logdet = 0.0;
  for (int a = 0; a < d; ++a) *logdet += 2.0 * log(L[a * d + a]);
  /* L^-1 by forward substitution, then Sigma^-1 = L^-T L^-1 */
  for (int c = 0; c < d; ++c)
    for (int a = 0; a < d; ++a) {
      double s = (a == c) ? 1.0 : 0.0;
      for (int k = 0; k < a; ++k) s -= L[a * d + k] * Li[k * d + c];
      Li[a * d + c] = s / L[a * d + a];
    }
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double s = 0.0;
      for (int k = 0; k < d; ++k) s += Li[k * d + a] * Li[k * d + b];
      inv[a * d + b] = s;
    }
out:
  free(m);
  free(S);
  free(L);
  free(Li);
  return st;
}

int orc_lscv_md_curve(const double* x, long n, int d, const double* grid, int n_h, double* g_out,
                      double* gscale_out, double* s1_out, double* s2_out) {
  if (n < 2 || d < 1 || n_h < 1) return ORC_INVAL;
  for (long i = 0; i < n * d; ++i)
    if (!isfinite(x[i])) return ORC_INVAL;
  for (int k = 0; k < n_h; ++k)
    if (!(grid[k] > 0.0) || !isfinite(grid[k]) || (k > 0 && !(grid[k] > grid[k - 1]))) return ORC_INVAL;
  double* inv = (double*)malloc(sizeof(double) * (size_t)d * d);
  double* rows1 = (double*)calloc((size_t)n * n_h, sizeof(double));
  double* rows2 = (double*)calloc((size_t)n * n_h, sizeof(double));
  double logdet = 0.0;
  int st = ORC_OK;
  if (!inv || !rows1 || !rows2) {
    st = ORC_NOMEM;
    goto done;
  }
  st = orc_cov_inverse(x, n, d, inv, &logdet);
  if (st) goto done;
#pragma omp parallel
  {
    double* v = (double*)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(dynamic, 16)
    for (long i = 0; i < n; ++i)
      for (long j = i + 1; j < n; ++j) {
        for (int a = 0; a < d; ++a) v[a] = x[i * d + a] - x[j * d + a];
        double S = 0.0;
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b) S += v[a] * inv[a * d + b] * v[b];
        for (int k = 0; k < n_h; ++k) {
          const double h2 = grid[k] * grid[k];
          rows1[i * n_h + k] += exp(-S / (4.0 * h2));
          rows2[i * n_h + k] += exp(-S / (2.0 * h2));
        }
      }
    free(v);
  }
  {
    double* col = (double*)malloc(sizeof(double) * (size_t)n);
    if (!col) {
      st = ORC_NOMEM;
      goto done;
    }
    const double sq = exp(-0.5 * logdet);
    const double A = pow(4.0 * ORC_PI, -0.5 * d) * sq, B = pow(2.0 * ORC_PI, -0.5 * d) * sq;
    const double nn = (double)n;
    for (int k = 0; k < n_h; ++k) {
      for (long i = 0; i < n; ++i) col[i] = rows1[i * n_h + k];
      const double s1 = neumaier_sum(col, n);
      for (long i = 0; i < n; ++i) col[i] = rows2[i * n_h + k];
      const double s2 = neumaier_sum(col, n);
      const double hd = pow(grid[k], -(double)d);
      g_out[k] = hd * (2.0 / (nn * nn) * (A * s1 - 2.0 * B * s2) + A / nn);
      if (gscale_out) gscale_out[k] = hd * (2.0 / (nn * nn) * (A * s1 + 2.0 * B * s2) + A / nn);
      if (s1_out) s1_out[k] = s1;
      if (s2_out) s2_out[k] = s2;
    }
    free(col);
  }
done:
  free(inv);
  free(rows1);
  free(rows2);
  return st;
}

/* Cholesky factor of a symmetric positive definite d x d matrix A (row-major):
 * L (lower, row-major), log|A| and A^-1.  A pivot at most 1e-12 of its
 * diagonal entry counts as singular. */
static int orc_spd(const double* A, int d, double* L, double* inv, double* logdet) {
  for (int i = 0; i < d * d; ++i) L[i] = 0.0;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b) {
      double s = A[a * d + b];
      for (int k = 0; k < b; ++k) s -= L[a * d + k] * L[b * d + k];
      if (a == b) {
        if (!(s > 1e-12 * A[a * d + a]) || !isfinite(s)) return ORC_DEGENERATE;
        L[a * d + a] = sqrt(s);
      } else {
        L[a * d + b] = s / L[b * d + b];
      }
    }
  double ld = 0.0;
  for (int a = 0; a < d; ++a) ld += 2.0 * log(L[a * d + a]);
  *logdet = ld;
  if (inv) {
    double Li[16 * 16];
    for (int c = 0; c < d; ++c)
      for (int a = 0; a < d; ++a) {
        double s = (a == c) ? 1.0 : 0.0;
        for (int k = 0; k < a; ++k) s -= L[a * d + k] * Li[k * d + c];
        Li[a * d + c] = s / L[a * d + a];
      }
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) s += Li[k * d + a] * Li[k * d + b];
        inv[a * d + b] = s;
      }
  }
  return ORC_OK;
}

/* LSCV_H objective at a bandwidth matrix H (Section 4.4.3, eq. (LSCV_MULTI-gh)
 * with (LSCV_MULTI-Kx), (LSCV_MULTI-KKx), (LSCV_MULTI-rk)):
 *   g(H) = 2 n^-2 sum_{i<j} [(K*K)_H - 2 K_H](X_i - X_j) + n^-1 R(K),
 * (K*K)_H(v) = (4 pi)^(-d/2) |H|^(-1/2) exp(-v^T H^-1 v / 4),
 * K_H(v) = (2 pi)^(-d/2) |H|^(-1/2) exp(-v^T H^-1 v / 2),
 * R(K) = 2^-d pi^(-d/2) |H|^(-1/2).  x row-major n x d, H row-major d x d,
 * d <= 16.  H not positive definite -> DEGENERATE. */
int orc_lscv_H(const double* x, long n, int d, const double* H, double* g_out) {
  if (n < 2 || d < 1 || d > 16) return ORC_INVAL;
  for (long i = 0; i < n * d; ++i)
    if (!isfinite(x[i])) return ORC_INVAL;
  double L[256], inv[256], logdet;
  int st = orc_spd(H, d, L, inv, &logdet);
  if (st) return st;
  double* rows1 = (double*)calloc((size_t)n, sizeof(double));
  double* rows2 = (double*)calloc((size_t)n, sizeof(double));
  if (!rows1 || !rows2) {
    free(rows1);
    free(rows2);
    return ORC_NOMEM;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (long i = 0; i < n; ++i) {
    double v[16];
    double r1 = 0.0, r2 = 0.0;
    for (long j = i + 1; j < n; ++j) {
      for (int a = 0; a < d; ++a) v[a] = x[i * d + a] - x[j * d + a];
      double q = 0.0;
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) q += v[a] * inv[a * d + b] * v[b];
      r1 += exp(-q / 4.0);
      r2 += exp(-q / 2.0);
    }
    rows1[i] = r1;
    rows2[i] = r2;
  }
  const double s1 = neumaier_sum(rows1, n), s2 = neumaier_sum(rows2, n);
  free(rows1);
  free(rows2);
  const double sq = exp(-0.5 * logdet), nn = (double)n;
  const double A = pow(4.0 * ORC_PI, -0.5 * d) * sq, B = pow(2.0 * ORC_PI, -0.5 * d) * sq;
  const double R = pow(2.0, -(double)d) * pow(ORC_PI, -0.5 * d) * sq;
  *g_out = 2.0 / (nn * nn) * (A * s1 - 2.0 * B * s2) + R / nn;
  return ORC_OK;
}

/* ---- Nelder-Mead over H (Section 4.4.3 names the method; the search space
 * is kept to positive definite matrices by the parametrisation): theta holds
 * the lower triangle of C, row by row, with the logarithm on the diagonal,
 * H = C C^T.  Start: eq. (LSCV-H-start) read as the squared bandwidth
 * H0 = s^2 Sigma, s = (4/(d+2))^(1/(d+4)) n^(-1/(d+4)).  Initial steps 0.25 on
 * the log-diagonal and 0.25 sqrt(C_aa C_bb) off it.  Moves: reflection 1,
 * expansion 2, contractions 1/2, shrink 1/2 towards the best vertex.  Stops
 * when the spread of g over the simplex is at most ftol |g_best| and every
 * vertex is within xtol of the best in every parameter, or after max_evals
 * evaluations. */
static void orc_theta_to_H(const double* th, int d, double* H) {
  double C[256];
  int p = 0;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) C[a * d + b] = 0.0;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b) C[a * d + b] = (a == b) ? exp(th[p++]) : th[p++];
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double s = 0.0;
      for (int k = 0; k < d; ++k) s += C[a * d + k] * C[b * d + k];
      H[a * d + b] = s;
    }
}

int orc_lscv_H_min(const double* x, long n, int d, double ftol, double xtol, int max_evals, double* H_out,
                   double* g_out, int* evals_out) {
  if (n < 2 || d < 1 || d > 16 || !(ftol > 0.0) || !(xtol > 0.0) || max_evals < 1) return ORC_INVAL;
  const int p = d * (d + 1) / 2;
  double Sinv[256], L[256], logdet;
  int st = orc_cov_inverse(x, n, d, Sinv, &logdet);
  if (st) return st;
  /* Sigma itself, for the start */
  double S[256], Ls[256], dummy;
  {
    double* m = (double*)calloc((size_t)d, sizeof(double));
    for (int a = 0; a < d; ++a) {
      for (long i = 0; i < n; ++i) m[a] += x[i * d + a];
      m[a] /= (double)n;
    }
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        double s = 0.0;
        for (long i = 0; i < n; ++i) s += (x[i * d + a] - m[a]) * (x[i * d + b] - m[b]);
        S[a * d + b] = s / (double)(n - 1);
      }
    free(m);
  }
  const double s = pow(4.0 / (d + 2.0), 1.0 / (d + 4.0)) * pow((double)n, -1.0 / (d + 4.0));
  for (int i = 0; i < d * d; ++i) S[i] *= s * s;
  st = orc_spd(S, d, Ls, NULL, &dummy);
  if (st) return st;
  (void)L;
  double V[17 * 136], F[17], H[256];
  int q = 0;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b) V[q++] = (a == b) ? log(Ls[a * d + a]) : Ls[a * d + b];
  for (int k = 1; k <= p; ++k) {
    for (int j = 0; j < p; ++j) V[k * p + j] = V[j];
    int a = 0, b = 0, idx = 0;
    for (a = 0; a < d; ++a) {
      for (b = 0; b <= a; ++b, ++idx)
        if (idx == k - 1) goto found;
    }
  found:
    V[k * p + (k - 1)] += (a == b) ? 0.25 : 0.25 * sqrt(Ls[a * d + a] * Ls[b * d + b]);
  }
  int evals = 0;
  for (int k = 0; k <= p; ++k) {
    orc_theta_to_H(V + k * p, d, H);
    if (orc_lscv_H(x, n, d, H, &F[k])) F[k] = INFINITY;
    ++evals;
  }
  double c[136], r[136], e[136], t[136], fr, fe, ft;
  for (;;) {
    /* order: insertion sort by F (stable: ties keep their order) */
    for (int i = 1; i <= p; ++i)
      for (int j = i; j > 0 && F[j] < F[j - 1]; --j) {
        double tf = F[j];
        F[j] = F[j - 1];
        F[j - 1] = tf;
        for (int m2 = 0; m2 < p; ++m2) {
          double tv = V[j * p + m2];
          V[j * p + m2] = V[(j - 1) * p + m2];
          V[(j - 1) * p + m2] = tv;
        }
      }
    double xs = 0.0;
    for (int i = 1; i <= p; ++i)
      for (int j = 0; j < p; ++j) xs = fmax(xs, fabs(V[i * p + j] - V[j]));
    if ((F[p] - F[0] <= ftol * fabs(F[0]) && xs <= xtol) || evals >= max_evals) break;
    for (int j = 0; j < p; ++j) {
      c[j] = 0.0;
      for (int i = 0; i < p; ++i) c[j] += V[i * p + j];
      c[j] /= (double)p;
    }
#define ORC_EVAL(vec, out)                         \
  do {                                             \
    orc_theta_to_H(vec, d, H);                     \
    if (orc_lscv_H(x, n, d, H, &(out))) out = INFINITY; \
    ++evals;                                       \
  } while (0)
    for (int j = 0; j < p; ++j) r[j] = c[j] + (c[j] - V[p * p + j]);
    ORC_EVAL(r, fr);
    int shrink = 0;
    if (fr < F[0]) {
      for (int j = 0; j < p; ++j) e[j] = c[j] + 2.0 * (c[j] - V[p * p + j]);
      ORC_EVAL(e, fe);
      if (fe < fr) {
        for (int j = 0; j < p; ++j) V[p * p + j] = e[j];
        F[p] = fe;
      } else {
        for (int j = 0; j < p; ++j) V[p * p + j] = r[j];
        F[p] = fr;
      }
    } else if (fr < F[p - 1]) {
      for (int j = 0; j < p; ++j) V[p * p + j] = r[j];
      F[p] = fr;
    } else if (fr < F[p]) {
      for (int j = 0; j < p; ++j) t[j] = c[j] + 0.5 * (r[j] - c[j]);
      ORC_EVAL(t, ft);
      if (ft <= fr) {
        for (int j = 0; j < p; ++j) V[p * p + j] = t[j];
        F[p] = ft;
      } else {
        shrink = 1;
      }
    } else {
      for (int j = 0; j < p; ++j) t[j] = c[j] + 0.5 * (V[p * p + j] - c[j]);
      ORC_EVAL(t, ft);
      if (ft < F[p]) {
        for (int j = 0; j < p; ++j) V[p * p + j] = t[j];
        F[p] = ft;
      } else {
        shrink = 1;
      }
    }
    if (shrink)
      for (int i = 1; i <= p; ++i) {
        for (int j = 0; j < p; ++j) V[i * p + j] = V[j] + 0.5 * (V[i * p + j] - V[j]);
        ORC_EVAL(V + i * p, F[i]);
      }
#undef ORC_EVAL
  }
  orc_theta_to_H(V, d, H_out);
  if (g_out) *g_out = F[0];
  if (evals_out) *evals_out = evals;
  return ORC_OK;
}

/* Density estimate with a bandwidth matrix at m points, eq. (kde-def-H) with
 * K_H of eq. (K_H) and K of eq. (gaussian):
 *   f(p) = n^-1 sum_i (2 pi)^(-d/2) |H|^(-1/2) exp(-(p - X_i)^T H^-1 (p - X_i) / 2).
 * x row-major n x d, H row-major d x d (lower triangle read), pts row-major
 * m x d.  H^-1 and |H| from its Cholesky factor; the quadratic form is the
 * double sum per pair; each point's sum is Neumaier-compensated in sample
 * order.  H not positive definite -> DEGENERATE. */
int orc_density_H(const double* x, long n, int d, const double* H, const double* pts, int m, double* out) {
  if (n < 1 || d < 1 || d > 16 || m < 1) return ORC_INVAL;
  for (long i = 0; i < n * d; ++i)
    if (!isfinite(x[i])) return ORC_INVAL;
  for (long i = 0; i < (long)m * d; ++i)
    if (!isfinite(pts[i])) return ORC_INVAL;
  double Hs[256], L[256], inv[256], logdet;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b <= a; ++b) Hs[a * d + b] = Hs[b * d + a] = H[a * d + b];
  for (int i = 0; i < d * d; ++i)
    if (!isfinite(Hs[i])) return ORC_INVAL;
  int st = orc_spd(Hs, d, L, inv, &logdet);
  if (st) return st;
  const double norm = pow(2.0 * ORC_PI, -0.5 * d) * exp(-0.5 * logdet) / (double)n;
#pragma omp parallel for schedule(dynamic, 4)
  for (int k = 0; k < m; ++k) {
    double v[16];
    double s = 0.0, c = 0.0;
    for (long i = 0; i < n; ++i) {
      for (int a = 0; a < d; ++a) v[a] = pts[(long)k * d + a] - x[i * d + a];
      double q = 0.0;
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) q += v[a] * inv[a * d + b] * v[b];
      const double t = exp(-0.5 * q);
      const double y = s + t;
      c += (fabs(s) >= fabs(t)) ? (s - y) + t : (t - y) + s;
      s = y;
    }
    out[k] = (s + c) * norm;
  }
  return ORC_OK;
}
