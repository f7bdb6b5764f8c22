"""Pins for the FP64 oracle against facts other than itself.

Each test checks an oracle function against something the paper prints
(tests/golden/paper_values.json), a closed form, a library routine (numpy's
Hermite module, numpy.var, scipy quadrature), an expectation over seeds, or a
brute-force computation that takes a different route (full n x n matrix
instead of the i < j triangle).  None of these re-types the oracle's formula.
"""
import json
import math
import os

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He
from scipy import integrate

import oracle
import workloads

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
SQRT2PI = math.sqrt(2.0 * math.pi)


def phi(u):
    return np.exp(-0.5 * np.asarray(u) ** 2) / SQRT2PI


def kr_numpy(r, u):
    """K^(r)(u) = He_r(u) phi(u) through numpy's Hermite_e module."""
    c = np.zeros(r + 1)
    c[r] = 1.0
    return He.hermeval(np.asarray(u, dtype=np.float64), c) * phi(u)


# ---------------------------------------------------------------- kernel derivatives
@pytest.mark.parametrize("r", range(0, 11))
def test_hermite_matches_numpy(r):
    c = np.zeros(r + 1)
    c[r] = 1.0
    for u in (-3.7, -1.0, -0.3, 0.0, 0.25, 1.5, 2.9, 6.0):
        ref = He.hermeval(u, c)
        assert oracle.hermite_e(r, u) == pytest.approx(ref, rel=1e-13, abs=1e-12)


@pytest.mark.parametrize("name,r", [("He6_coefficients_high_to_low", 6), ("He4_coefficients_high_to_low", 4)])
def test_kernel_deriv_matches_printed_polynomial(name, r):
    coef = GOLD[name]["c"]
    for u in np.linspace(-5, 5, 41):
        printed = np.polyval(coef, u) * phi(u)
        assert oracle.kernel_deriv(r, u) == pytest.approx(printed, rel=1e-12, abs=1e-14)


def test_kernel_deriv_at_zero_matches_printed():
    k6 = GOLD["K6_at_0"]["numerator"] / SQRT2PI
    k4 = GOLD["K4_at_0"]["numerator"] / SQRT2PI
    assert oracle.kernel_deriv(6, 0.0) == pytest.approx(k6, rel=1e-15)
    assert oracle.kernel_deriv(4, 0.0) == pytest.approx(k4, rel=1e-15)


@pytest.mark.parametrize("r", [4, 6, 8])
def test_kernel_deriv_moments(r):
    """Integration by parts: int u^k phi^(r)(u) du = 0 for k < r and r! for k = r (r even)."""
    for k in range(0, r + 1):
        val, _ = integrate.quad(lambda u: u**k * oracle.kernel_deriv(r, u), -40, 40, limit=400)
        ref = float(math.factorial(r)) if k == r else 0.0
        assert val == pytest.approx(ref, abs=1e-8 * max(1.0, ref))


# ---------------------------------------------------------------- moments and rule of thumb
@pytest.mark.parametrize("family", ["normal", "lognormal", "uniform"])
def test_moments_match_numpy(family):
    x = workloads.draw(family, 5003, 11, np.float64)
    m, v = oracle.moments(x)
    assert m == pytest.approx(float(np.mean(x)), rel=1e-14, abs=1e-15)
    assert v == pytest.approx(float(np.var(x, ddof=1)), rel=1e-13)


def test_moments_large_offset_is_stable():
    """Two-pass variance keeps accuracy where the one-pass printed form would cancel."""
    x = 1e8 + workloads.draw("normal", 4000, 5, np.float64)
    _, v = oracle.moments(x)
    assert v == pytest.approx(float(np.var(x, ddof=1)), rel=1e-9)


def test_rot_matches_both_printed_forms_and_quadrature():
    x = workloads.draw("normal", 1000, 1998001, np.float64)
    n = x.size
    sigma, h = oracle.bw_rot(x)
    assert sigma == pytest.approx(float(np.std(x, ddof=1)), rel=1e-13)
    # eq. (LSCV-h0), d = 1, with the printed constants
    d = GOLD["h0_constants_d1"]["d"]
    rk_mu = 1.0 / (2**d * math.pi ** (d / 2) * d**2)
    rf2 = d * (d + 2) / (2 ** (d + 2) * math.pi ** (d / 2))
    h0 = (rk_mu / (rf2 * n)) ** (1.0 / (d + 4))
    assert h == pytest.approx(sigma * h0, rel=1e-14)
    # eq. (LSCV-H-start), d = 1
    hs = (4.0 / (d + 2)) ** (1.0 / (d + 4)) * n ** (-1.0 / (d + 4)) * sigma
    assert h == pytest.approx(hs, rel=1e-14)
    # AMISE-optimal h for a N(0, sigma^2) density: R(f'') by quadrature
    rf2_q, _ = integrate.quad(lambda t: (kr_numpy(2, t)) ** 2, -30, 30)
    h_amise = ((1.0 / (2.0 * math.sqrt(math.pi))) / (rf2_q * n)) ** 0.2 * sigma
    assert h == pytest.approx(h_amise, rel=1e-9)
    # worked value: h0 = 0.266065 for n = 1000 (to the printed digits)
    assert h0 == pytest.approx(0.266065, abs=5e-7)


# ---------------------------------------------------------------- normal-scale functionals and pilots
@pytest.mark.parametrize("r", [4, 6, 8, 10])
@pytest.mark.parametrize("sigma", [0.37, 1.0, 2.5])
def test_psi_ns_matches_quadrature(r, sigma):
    """psi_r = int f^(r) f dx for the N(0, sigma^2) density, by scipy quadrature."""
    f = lambda t: phi(t / sigma) / sigma
    fr = lambda t: kr_numpy(r, t / sigma) / sigma ** (r + 1)
    val, _ = integrate.quad(lambda t: fr(t) * f(t), -40 * sigma, 40 * sigma, limit=400)
    assert oracle.psi_ns(r, sigma) == pytest.approx(val, rel=1e-9)


def test_psi8_ns_matches_printed():
    g = GOLD["psi8_NS"]
    for s in (0.5, 1.0, 3.0):
        printed = g["numerator"] / (g["denominator"] * math.sqrt(math.pi) * s ** g["sigma_power"])
        assert oracle.psi_ns(8, s) == pytest.approx(printed, rel=1e-14)


@pytest.mark.parametrize("r", [4, 6, 8])
def test_pilot_cancels_amse_leading_terms(r):
    """The AMSE-optimal pilot makes the variance-like and bias terms cancel:
    K^(r)(0) / (n g^(r+1)) + mu_2 g^2 psi_{r+2} / 2 = 0 (K^(r)(0) from numpy)."""
    n = 12345
    psi_next = oracle.psi_ns(r + 2, 1.3)
    g = oracle.pilot(r, psi_next, n)
    k0 = float(kr_numpy(r, 0.0))
    lead = k0 / (n * g ** (r + 1))
    bias = 0.5 * GOLD["mu2_K"]["value"] * g**2 * psi_next
    assert lead + bias == pytest.approx(0.0, abs=1e-12 * abs(lead))


def test_pilot_rejects_wrong_sign():
    with pytest.raises(oracle.OracleError) as e:
        oracle.pilot(6, -1.0, 100)  # psi_8 must be positive
    assert e.value.code == oracle.DEGENERATE


# ---------------------------------------------------------------- pairwise functionals
@pytest.mark.parametrize("r", [4, 6, 8])
@pytest.mark.parametrize("family", ["normal", "bimodal"])
def test_psi_hat_brute_force_full_matrix(r, family):
    """n^-2 g^-(r+1) sum over ALL (i, j), diagonal included, by numpy on the full matrix."""
    x = workloads.draw(family, 301, 7, np.float64)
    g = 0.41
    u = (x[:, None] - x[None, :]) / g
    full = kr_numpy(r, u)
    ref = full.sum() / (x.size**2 * g ** (r + 1))
    val, kappa, s, a = oracle.psi(x, r, g)
    assert val == pytest.approx(ref, rel=1e-11)
    off = full[np.triu_indices(x.size, 1)]
    assert s == pytest.approx(off.sum(), rel=1e-11, abs=1e-9)
    assert a == pytest.approx(np.abs(off).sum(), rel=1e-12)
    assert kappa == pytest.approx(np.abs(off).sum() / abs(off.sum()), rel=1e-9)


@pytest.mark.parametrize("r", [4, 6])
def test_psi_hat_expectation_on_normal_data(r):
    """E[psi_r(g)] = n^-1 g^-(r+1) K^(r)(0) + (1 - n^-1) (g^2 + 2 s^2)^(-(r+1)/2) K^(r)(0)
    for N(0, s^2) samples; the printed form with n K^(r)(0) outside the
    normalisation would be off by orders of magnitude."""
    n, g, s, reps = 200, 0.6, 1.0, 120
    vals = np.array([oracle.psi(workloads.draw("normal", n, 1000 + k, np.float64), r, g)[0] for k in range(reps)])
    k0 = float(kr_numpy(r, 0.0))
    expect = k0 / (n * g ** (r + 1)) + (1 - 1 / n) * (g * g + 2 * s * s) ** (-(r + 1) / 2) * k0
    se = vals.std(ddof=1) / math.sqrt(reps)
    assert abs(vals.mean() - expect) < 4 * se + 1e-12


def test_plugin_approaches_amise_bandwidth():
    """For large n the plug-in h approaches the AMISE-optimal h of the true
    density: (R(K) / (psi_4 n))^(1/5) with psi_4 = int (f'')^2 by quadrature."""
    n = 20000
    for family, dens in [
        ("normal", lambda t: phi(t)),
        ("mixture", lambda t: 0.5 * phi((t + 2) / 0.5) / 0.5 + 0.5 * phi(t - 1)),
    ]:
        x = workloads.draw(family, n, 424242, np.float64)
        if family == "normal":
            f2 = lambda t: kr_numpy(2, t)
        else:
            f2 = lambda t: 0.5 * kr_numpy(2, (t + 2) / 0.5) / 0.5**3 + 0.5 * kr_numpy(2, t - 1)
        psi4, _ = integrate.quad(lambda t: f2(t) ** 2, -30, 30, limit=400)
        h_amise = (1.0 / (2 * math.sqrt(math.pi)) / (psi4 * n)) ** 0.2
        for stages in (2, 3):
            info = oracle.bw_plugin(x, stages)
            assert info.h == pytest.approx(h_amise, rel=0.08), (family, stages, info.h, h_amise)


# ---------------------------------------------------------------- LSCV objective
def _fhat_sq_integral(x, h):
    f = lambda t: phi((t - x) / h).sum() / (x.size * h)
    lo, hi = x.min() - 12 * h, x.max() + 12 * h
    pts = np.sort(x)
    val, _ = integrate.quad(lambda t: f(t) ** 2, lo, hi, points=pts, limit=800, epsabs=1e-14, epsrel=1e-13)
    return val


@pytest.mark.parametrize("h", [0.05, 0.2, 0.45, 1.0, 3.0])
def test_lscv_toy_dataset_by_quadrature(h):
    """g(h) = int fhat^2 - 2 n^-2 sum_{i != j} K_h(X_i - X_j) on the paper's
    8-point toy sample, with the integral by adaptive quadrature."""
    x = np.array(GOLD["toy_dataset"]["x"], dtype=np.float64)
    n = x.size
    d = x[:, None] - x[None, :]
    kh = phi(d / h) / h
    np.fill_diagonal(kh, 0.0)
    ref = _fhat_sq_integral(x, h) - 2.0 / n**2 * kh.sum()
    g = oracle.lscv_curve(x, [h]).g[0]
    assert g == pytest.approx(ref, rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("family", ["normal", "lognormal"])
def test_lscv_brute_force_full_matrix(family):
    x = workloads.draw(family, 400, 99, np.float64)
    grid = np.geomspace(0.01, 2.0, 17)
    cur = oracle.lscv_curve(x, grid)
    d2 = (x[:, None] - x[None, :]) ** 2
    iu = np.triu_indices(x.size, 1)
    n = x.size
    for k, h in enumerate(grid):
        kk = np.exp(-d2 / (4 * h * h)) / math.sqrt(4 * math.pi) / h  # (K_h * K_h)
        kh = np.exp(-d2 / (2 * h * h)) / math.sqrt(2 * math.pi) / h
        np.fill_diagonal(kk, 0.0)
        np.fill_diagonal(kh, 0.0)
        ref = (kk.sum() - 2 * kh.sum()) / n**2 + 1.0 / (n * h * math.sqrt(4 * math.pi))
        assert cur.g[k] == pytest.approx(ref, rel=1e-10, abs=1e-14)
        assert cur.s1[k] == pytest.approx(np.exp(-d2[iu] / (4 * h * h)).sum(), rel=1e-12)
        assert cur.s2[k] == pytest.approx(np.exp(-d2[iu] / (2 * h * h)).sum(), rel=1e-12)


def test_lscv_block_sums_partition_the_triangle():
    """Blocks of any partition of the i < j triangle add up to the full pair
    sums, and one block matches a numpy brute force."""
    x = workloads.draw("lognormal", 700, 21, np.float64)
    grid = np.geomspace(0.02, 1.5, 7)
    full = oracle.lscv_curve(x, grid)
    acc1 = np.zeros(grid.size)
    acc2 = np.zeros(grid.size)
    for i0 in range(0, 700, 256):
        for j0 in range(i0, 700, 300):
            s1, s2 = oracle.lscv_block_sums(x, i0, i0 + 256, j0, j0 + 300, grid)
            acc1 += s1
            acc2 += s2
    assert np.allclose(acc1, full.s1, rtol=1e-12)
    assert np.allclose(acc2, full.s2, rtol=1e-12)
    s1, s2 = oracle.lscv_block_sums(x, 256, 512, 300, 600, grid)
    d2 = (x[256:512, None] - x[None, 300:600]) ** 2
    mask = np.arange(300, 600)[None, :] > np.arange(256, 512)[:, None]
    for k, h in enumerate(grid):
        assert s1[k] == pytest.approx((np.exp(-d2 / (4 * h * h)) * mask).sum(), rel=1e-12)
        assert s2[k] == pytest.approx((np.exp(-d2 / (2 * h * h)) * mask).sum(), rel=1e-12)


def test_lscv_expectation_on_normal_data():
    """E[g(h)] = 1/(2 sqrt(pi) n h) + (1 - 1/n) [(4 pi (h^2 + s^2))^(-1/2) - 2 (2 pi (h^2 + 2 s^2))^(-1/2)]."""
    n, reps = 150, 150
    grid = np.array([0.1, 0.35, 0.8])
    vals = np.array([oracle.lscv_curve(workloads.draw("normal", n, 5000 + k, np.float64), grid).g for k in range(reps)])
    for k, h in enumerate(grid):
        e = 1 / (2 * math.sqrt(math.pi) * n * h) + (1 - 1 / n) * (
            (4 * math.pi * (h * h + 1)) ** -0.5 - 2 * (2 * math.pi * (h * h + 2)) ** -0.5)
        se = vals[:, k].std(ddof=1) / math.sqrt(reps)
        assert abs(vals[:, k].mean() - e) < 4 * se


def test_default_grid_spans_printed_range():
    x = workloads.draw("gamma", 777, 3, np.float64)
    s, hr = oracle.bw_rot(x)
    grid = oracle.default_grid(x, 0)
    assert grid.size == GOLD["grid_points_experiments"]["n_h"]
    assert grid[0] == pytest.approx(GOLD["search_range"]["lo_factor"] * hr, rel=1e-14)
    assert grid[-1] == pytest.approx(GOLD["search_range"]["hi_factor"] * hr, rel=1e-14)
    assert np.allclose(np.diff(grid), np.diff(grid)[0], rtol=1e-9)


def test_argmin_ties_edges_and_margin():
    assert oracle.argmin([3.0, 1.0, 1.0, 2.0]) == (1, False, 0.0)
    k, e, m = oracle.argmin([0.5, 1.0, 2.0])
    assert (k, e, m) == (0, True, 0.5)
    g = workloads.draw("normal", 50, 1, np.float64)
    assert oracle.argmin(g)[0] == int(np.argmin(g))


# ---------------------------------------------------------------- invariances and error paths
def test_invariances():
    x = workloads.draw("bimodal", 257, 17, np.float64)
    grid = np.geomspace(0.05, 1.5, 9)
    base = oracle.lscv_curve(x, grid).g
    p2 = oracle.bw_plugin(x, 3)
    perm = np.random.Generator(np.random.PCG64(3)).permutation(x.size)
    for y in (x + 1234.5, -x, x[perm]):
        assert np.allclose(oracle.lscv_curve(y, grid).g, base, rtol=1e-9, atol=1e-13)
        q = oracle.bw_plugin(y, 3)
        assert q.h == pytest.approx(p2.h, rel=1e-9)
        assert np.allclose(q.psi, p2.psi, rtol=1e-8)
    a = 3.7
    scaled = oracle.lscv_curve(a * x, a * grid).g
    assert np.allclose(scaled, base / a, rtol=1e-10, atol=1e-14)
    assert oracle.bw_plugin(a * x, 3).h == pytest.approx(a * p2.h, rel=1e-10)
    assert oracle.bw_plugin(a * x, 2).h == pytest.approx(a * oracle.bw_plugin(x, 2).h, rel=1e-10)
    for r_idx, r in enumerate((8, 6, 4)):
        if r_idx == 0:
            continue
        assert oracle.bw_plugin(a * x, 3).psi[r_idx] == pytest.approx(p2.psi[r_idx] / a ** (r + 1), rel=1e-9)
    assert oracle.bw_rot(a * x)[1] == pytest.approx(a * oracle.bw_rot(x)[1], rel=1e-13)


def test_error_paths():
    with pytest.raises(oracle.OracleError) as e:
        oracle.bw_rot([1.0])
    assert e.value.code == oracle.INVAL
    with pytest.raises(oracle.OracleError) as e:
        oracle.bw_rot([1.0, float("nan"), 2.0])
    assert e.value.code == oracle.INVAL
    with pytest.raises(oracle.OracleError) as e:
        oracle.bw_plugin([2.0] * 10, 2)
    assert e.value.code == oracle.DEGENERATE
    with pytest.raises(oracle.OracleError) as e:
        oracle.lscv_curve([0.0, 1.0, 2.0], [0.5, 0.2])
    assert e.value.code == oracle.INVAL
    # duplicates are allowed: the pair contributes exp(0) = 1
    c = oracle.lscv_curve([1.0, 1.0], [0.5])
    assert c.s1[0] == 1.0 and c.s2[0] == 1.0


def test_lscv_search_matches_a_library_minimiser():
    """The k-section search (Section 4.4.2's alternative to the grid) lands on
    the minimiser scipy's bounded Brent method finds for the same g(h) in
    log h, near the same local minimum; for an interior minimum its step count
    follows from the bracket shrinking by 2/(m - 1) in log h per step."""
    from scipy.optimize import minimize_scalar

    for fam, n, seed in (("normal", 400, 3), ("bimodal", 600, 8), ("lognormal", 500, 2)):
        x = workloads.draw(fam, n, seed, np.float64)
        lo, hi, tol, m = 0.01, 3.0, 1e-7, 16
        h, g, steps, (a, b) = oracle.lscv_min(x, lo, hi, tol, m)
        assert a <= h <= b and b / a - 1 <= tol

        def f(t):
            return oracle.lscv_curve(x, np.array([np.exp(t)])).g[0]

        # the same local minimum: Brent on a bracket of +-5% around the search's point
        r = minimize_scalar(f, bounds=(np.log(h) - 0.05, np.log(h) + 0.05), method="bounded",
                            options={"xatol": 1e-10})
        assert np.exp(r.x) == pytest.approx(h, rel=1e-5), fam
        assert g <= r.fun + 1e-12 * abs(r.fun), fam
        assert g == pytest.approx(f(np.log(h)), rel=1e-14)
        # and no coarse grid point over the whole range is lower
        coarse = oracle.lscv_curve(x, np.geomspace(lo, hi, 200)).g
        assert g <= coarse.min() + 1e-12 * abs(coarse.min()), fam
        # interior minimum: steps = first j with (hi/lo)^((2/(m-1))^j) - 1 <= tol, plus one
        w0, rr = np.log(hi / lo), 2.0 / (m - 1)
        j = next(j for j in range(200) if np.expm1(w0 * rr**j) <= tol)
        assert steps == j + 1, (fam, steps, j)


def test_lscv_search_edge_and_errors():
    x = workloads.draw("normal", 300, 5, np.float64)
    # a range entirely above the optimum: g rises, the search closes on the lower end
    h, g, steps, (a, b) = oracle.lscv_min(x, 2.0, 5.0, 1e-6, 8)
    assert a == 2.0 and h == 2.0
    for bad in ((0.0, 1.0, 1e-3, 8), (1.0, 0.5, 1e-3, 8), (0.1, 1.0, 0.0, 8), (0.1, 1.0, 1e-3, 3)):
        with pytest.raises(oracle.OracleError) as e:
            oracle.lscv_min(x, *bad)
        assert e.value.code == oracle.INVAL


TOY = np.array([0.0, 1.0, 1.1, 1.5, 1.9, 2.8, 2.9, 3.5])  # the 8-point example of Section 2


def test_density_matches_a_library_kde_and_its_moments():
    """f(p) = (n h)^-1 sum phi((p - X_i)/h): scipy's gaussian_kde with its
    bandwidth factor set to h / sigma-hat is the same estimator; the estimate
    integrates to 1, has the sample mean as its mean and (n-1)/n V + h^2 as
    its variance (composite Simpson on a grid of step h/64)."""
    from scipy import integrate
    from scipy.stats import gaussian_kde

    for x, h in ((TOY, 0.4), (workloads.draw("bimodal", 700, 4, np.float64), 0.3),
                 (workloads.draw("lognormal", 500, 9, np.float64), 0.05)):
        pts = np.linspace(x.min() - 1, x.max() + 1, 41)
        f = oracle.density(x, h, pts)
        ref = gaussian_kde(x, bw_method=h / np.std(x, ddof=1))(pts)
        assert np.allclose(f, ref, rtol=1e-12, atol=1e-15)
        t = np.arange(x.min() - 12 * h, x.max() + 12 * h, h / 64)
        ft = oracle.density(x, h, t)
        assert integrate.simpson(ft, x=t) == pytest.approx(1.0, abs=1e-9)
        assert integrate.simpson(t * ft, x=t) == pytest.approx(x.mean(), rel=1e-9, abs=1e-9)
        assert integrate.simpson((t - x.mean())**2 * ft, x=t) == pytest.approx(np.var(x) + h * h, rel=1e-8)
    # two equal samples: the kernel itself
    p = np.array([0.2, 1.5, 3.0])
    assert oracle.density([1.5, 1.5], 0.7, p) == pytest.approx(
        np.exp(-0.5 * ((p - 1.5) / 0.7)**2) / (0.7 * np.sqrt(2 * np.pi)), rel=1e-14)


def test_range_aggregates_match_quadrature_and_a_library_kde():
    """COUNT = n int f and SUM = n int x f over [a, b] (eq. (count), (sum)):
    against scipy's gaussian_kde box integral and adaptive quadrature of the
    oracle's own density; the whole line gives n and the sum of the samples."""
    from scipy import integrate
    from scipy.stats import gaussian_kde

    x = workloads.draw("gamma", 600, 12, np.float64)
    h = 0.25
    lo = np.array([-np.inf, 0.5, 1.0, 2.0, 7.0, 3.0, -5.0])
    hi = np.array([np.inf, 1.5, 1.0, 6.0, 30.0, 3.1, -1.0])
    cnt, sm = oracle.range_aggregates(x, h, lo, hi)
    kde = gaussian_kde(x, bw_method=h / np.std(x, ddof=1))
    assert cnt[0] == pytest.approx(x.size, rel=1e-14) and sm[0] == pytest.approx(x.sum(), rel=1e-13)
    assert cnt[2] == 0.0 and sm[2] == 0.0  # an empty range
    for k in range(1, lo.size):
        assert cnt[k] == pytest.approx(x.size * kde.integrate_box_1d(lo[k], hi[k]), rel=1e-10, abs=1e-12)
        if hi[k] > lo[k]:
            a_, b_ = max(lo[k], x.min() - 12 * h), min(hi[k], x.max() + 12 * h)
            if b_ <= a_:
                assert cnt[k] < 1e-20
                continue
            t = np.linspace(a_, b_, 2 * int((b_ - a_) / (h / 64)) + 3)
            ft = oracle.density(x, h, t)
            assert cnt[k] == pytest.approx(x.size * integrate.simpson(ft, x=t), rel=1e-8, abs=1e-9)
            assert sm[k] == pytest.approx(x.size * integrate.simpson(t * ft, x=t), rel=1e-8, abs=1e-9)


def test_consumer_error_paths():
    for call in (lambda: oracle.density(TOY, 0.0, [1.0]), lambda: oracle.density(TOY, np.inf, [1.0]),
                 lambda: oracle.density([1.0, np.nan], 0.5, [1.0]),
                 lambda: oracle.range_aggregates(TOY, 0.5, [2.0], [1.0]),
                 lambda: oracle.range_aggregates(TOY, 0.5, [np.nan], [1.0])):
        with pytest.raises(oracle.OracleError) as e:
            call()
        assert e.value.code == oracle.INVAL


def test_lscv_md_reduces_to_one_dimension_and_matches_brute_force():
    """LSCV_h in d dimensions (eq. LSCV-gh with S(v) = v^T Sigma^-1 v): at
    d = 1 the sphered objective equals the data-unit objective at sigma h
    exactly; for d = 2, 3 the pair sums match a numpy all-pairs computation
    whose inverse covariance comes from numpy.linalg."""
    x = workloads.draw("bimodal", 500, 3, np.float64)
    grid = np.geomspace(0.05, 1.5, 12)
    md = oracle.lscv_md_curve(x[:, None], grid)
    one = oracle.lscv_curve(x, np.std(x, ddof=1) * grid)
    assert np.allclose(md.g, one.g, rtol=1e-12) and np.allclose(md.s1, one.s1, rtol=1e-12)
    rng = np.random.Generator(np.random.PCG64(11))
    for d in (2, 3):
        n = 300
        z = rng.standard_normal((n, d)) @ rng.standard_normal((d, d)) + rng.uniform(-2, 2, d)
        inv = np.linalg.inv(np.cov(z, rowvar=False))
        iu = np.triu_indices(n, 1)
        v = z[:, None, :] - z[None, :, :]
        S = np.einsum("ija,ab,ijb->ij", v, inv, v)[iu]
        c = oracle.lscv_md_curve(z, grid)
        for k, h in enumerate(grid):
            assert c.s1[k] == pytest.approx(np.exp(-S / (4 * h * h)).sum(), rel=1e-11)
            assert c.s2[k] == pytest.approx(np.exp(-S / (2 * h * h)).sum(), rel=1e-11)


def test_lscv_md_affine_invariance_and_errors():
    """The sphered objective is invariant in shape under x -> A x + b:
    S(v) is unchanged and |Sigma|^-1/2 scales by 1/|det A|, so
    g_{Ax+b}(h) = g_x(h) / |det A|; collinear samples have a singular Sigma."""
    rng = np.random.Generator(np.random.PCG64(12))
    z = rng.standard_normal((250, 3)) * [1.0, 2.0, 0.5]
    A = np.array([[2.0, 0.3, 0.0], [-0.5, 1.0, 0.7], [0.1, 0.0, -1.5]])
    grid = np.geomspace(0.1, 2.0, 9)
    g0 = oracle.lscv_md_curve(z, grid).g
    g1 = oracle.lscv_md_curve(z @ A.T + [5.0, -3.0, 100.0], grid).g
    assert np.allclose(g1, g0 / abs(np.linalg.det(A)), rtol=1e-9)
    col = np.stack([z[:, 0], 2 * z[:, 0] + 1], axis=1)
    with pytest.raises(oracle.OracleError) as e:
        oracle.lscv_md_curve(col, grid)
    assert e.value.code == oracle.DEGENERATE
    with pytest.raises(oracle.OracleError) as e:
        oracle.lscv_md_curve(z, grid[::-1])
    assert e.value.code == oracle.INVAL


def test_lscv_H_reductions_brute_force_and_invariance():
    """LSCV_H, eq. (LSCV_MULTI-gh): at H = h^2 Sigma it is the sphered LSCV_h
    objective, at d = 1 the univariate one at h = sqrt(H); its pair sums match
    numpy with a library inverse; g_{Ax}(A H A^T) = g_x(H) / |det A|."""
    rng = np.random.Generator(np.random.PCG64(21))
    for d in (2, 3):
        z = rng.standard_normal((300, d)) @ (rng.standard_normal((d, d)) + 2 * np.eye(d)).T
        S = np.cov(z, rowvar=False)
        for h in (0.2, 0.5, 1.1):
            assert oracle.lscv_H(z, h * h * S) == pytest.approx(oracle.lscv_md_curve(z, [h]).g[0], rel=1e-12)
        M = rng.standard_normal((d, d))
        H = M @ M.T + 0.3 * np.eye(d)
        inv = np.linalg.inv(H)
        iu = np.triu_indices(z.shape[0], 1)
        v = z[:, None, :] - z[None, :, :]
        q = np.einsum("ija,ab,ijb->ij", v, inv, v)[iu]
        n = z.shape[0]
        sq = np.linalg.det(H) ** -0.5
        g = (2 / n**2 * ((4 * np.pi) ** (-d / 2) * sq * np.exp(-q / 4).sum()
                         - 2 * (2 * np.pi) ** (-d / 2) * sq * np.exp(-q / 2).sum())
             + (2.0 ** -d) * np.pi ** (-d / 2) * sq / n)
        assert oracle.lscv_H(z, H) == pytest.approx(g, rel=1e-11)
        A = rng.standard_normal((d, d)) + 3 * np.eye(d)
        assert oracle.lscv_H(z @ A.T + 7.0, A @ H @ A.T) == pytest.approx(
            oracle.lscv_H(z, H) / abs(np.linalg.det(A)), rel=1e-10)
    x = workloads.draw("mixture", 400, 5, np.float64)
    for h in (0.1, 0.3):
        assert oracle.lscv_H(x[:, None], [[h * h]]) == pytest.approx(oracle.lscv_curve(x, [h]).g[0], rel=1e-12)
    with pytest.raises(oracle.OracleError) as e:
        oracle.lscv_H(z, -np.eye(3))
    assert e.value.code == oracle.DEGENERATE


def test_lscv_H_nelder_mead_matches_scipy():
    """The oracle's Nelder-Mead (Section 4.4.3) over H = C C^T, C lower
    triangular with log-diagonal, lands where scipy's Nelder-Mead on the same
    objective and start does, and a full H does at least as well as the best
    H = h^2 Sigma of the LSCV_h family."""
    from scipy.optimize import minimize

    rng = np.random.Generator(np.random.PCG64(22))
    z = rng.standard_normal((350, 2)) @ np.array([[1.0, 0.0], [0.8, 0.4]]).T
    z[:120] = 0.5 * z[:120] + [2.5, 1.0]
    H, g, evals = oracle.lscv_H_min(z, ftol=1e-12, xtol=1e-8, max_evals=4000)
    assert evals < 4000
    n, d = z.shape
    s = (4 / (d + 2)) ** (1 / (d + 4)) * n ** (-1 / (d + 4))
    C0 = np.linalg.cholesky(s * s * np.cov(z, rowvar=False))
    th0 = np.array([np.log(C0[0, 0]), C0[1, 0], np.log(C0[1, 1])])

    def f(th):
        C = np.array([[np.exp(th[0]), 0.0], [th[1], np.exp(th[2])]])
        return oracle.lscv_H(z, C @ C.T)

    r = minimize(f, th0, method="Nelder-Mead", options={"xatol": 1e-9, "fatol": 1e-14, "maxfev": 5000})
    Cr = np.array([[np.exp(r.x[0]), 0.0], [r.x[1], np.exp(r.x[2])]])
    assert g == pytest.approx(r.fun, rel=1e-9)
    assert np.allclose(H, Cr @ Cr.T, rtol=1e-4, atol=1e-7)
    best_h = min(oracle.lscv_md_curve(z, np.geomspace(0.1, 2.0, 400)).g)
    assert g <= best_h + 1e-12


def test_density_H_reductions_and_library_forms():
    """Eq. (kde-def-H): at d = 1 it is the univariate estimate with h = sqrt(H);
    with H = h^2 Sigma it is scipy's gaussian_kde with bandwidth factor h; a
    single sample gives scipy's multivariate normal density; a diagonal H is a
    product of univariate normal densities; an affine map of samples, point
    and H divides f by |det A|."""
    from scipy.stats import gaussian_kde, multivariate_normal, norm

    rng = np.random.Generator(np.random.PCG64(31))
    x1 = workloads.draw("bimodal", 300, 2, np.float64)
    p1 = np.linspace(-4, 4, 17)
    assert np.allclose(oracle.density_H(x1, [[0.09]], p1[:, None]), oracle.density(x1, 0.3, p1), rtol=1e-13)
    for d in (2, 3):
        z = rng.standard_normal((250, d)) @ (rng.standard_normal((d, d)) + 2 * np.eye(d)).T
        pts = z[:9] + 0.3 * rng.standard_normal((9, d))
        S = np.cov(z, rowvar=False)
        for h in (0.2, 0.6):
            ref = gaussian_kde(z.T, bw_method=h)(pts.T)
            assert np.allclose(oracle.density_H(z, h * h * S, pts), ref, rtol=1e-11)
        M = rng.standard_normal((d, d))
        H = M @ M.T + 0.2 * np.eye(d)
        assert oracle.density_H(z[:1], H, pts) == pytest.approx(multivariate_normal(z[0], H).pdf(pts), rel=1e-12)
        hd = np.array([0.3, 0.7, 1.1][:d])
        prod = np.mean(np.prod(norm.pdf(pts[:, None, :], loc=z[None, :, :], scale=hd), axis=2), axis=1)
        assert np.allclose(oracle.density_H(z, np.diag(hd * hd), pts), prod, rtol=1e-12)
        A = rng.standard_normal((d, d)) + 2 * np.eye(d)
        fa = oracle.density_H(z @ A.T + 1.5, A @ H @ A.T, pts @ A.T + 1.5)
        assert np.allclose(fa, oracle.density_H(z, H, pts) / abs(np.linalg.det(A)), rtol=1e-11)


def test_density_H_integrates_to_one_with_the_sample_moments():
    """d = 2 on a grid of step 1/40 over +-8 deviations: mass 1, mean the
    sample mean, covariance (n-1)/n Sigma + H (composite Simpson)."""
    from scipy import integrate

    rng = np.random.Generator(np.random.PCG64(32))
    z = rng.standard_normal((40, 2)) @ np.array([[1.0, 0.0], [0.6, 0.5]]).T
    H = np.array([[0.09, 0.03], [0.03, 0.05]])
    g0 = np.arange(z[:, 0].min() - 3, z[:, 0].max() + 3, 1 / 40)
    g1 = np.arange(z[:, 1].min() - 3, z[:, 1].max() + 3, 1 / 40)
    G0, G1 = np.meshgrid(g0, g1, indexing="ij")
    f = oracle.density_H(z, H, np.stack([G0.ravel(), G1.ravel()], 1)).reshape(G0.shape)

    def I2(v):
        return integrate.simpson(integrate.simpson(v, x=g1, axis=1), x=g0)

    assert I2(f) == pytest.approx(1.0, abs=1e-9)
    m = z.mean(0)
    assert I2(G0 * f) == pytest.approx(m[0], abs=1e-9) and I2(G1 * f) == pytest.approx(m[1], abs=1e-9)
    C = np.cov(z, rowvar=False) * (z.shape[0] - 1) / z.shape[0] + H
    assert I2((G0 - m[0]) * (G1 - m[1]) * f) == pytest.approx(C[0, 1], rel=1e-8)
    assert I2((G0 - m[0]) ** 2 * f) == pytest.approx(C[0, 0], rel=1e-8)


def test_range_aggregates_2d_against_closed_forms_and_libraries():
    """Eq. (count-sum-2D) with the estimate of eq. (kde-def-H): the whole plane
    gives n and the coordinate sums; a box over the whole second axis gives
    the univariate aggregates of the first coordinate with h = sqrt(H11)
    (the kernel's marginal), whatever the correlation; a diagonal H gives
    products of univariate normal masses; COUNT matches scipy's rectangle
    probability of the multivariate normal (Genz's algorithm); adjacent
    boxes add up; and COUNT and SUM agree with 2-D Simpson integration of the
    oracle's own density."""
    from scipy import integrate
    from scipy.special import ndtr
    from scipy.stats import multivariate_normal

    rng = np.random.Generator(np.random.PCG64(33))
    z = rng.standard_normal((60, 2)) @ np.array([[1.0, 0.0], [0.7, 0.6]]).T
    H = np.array([[0.16, 0.09], [0.09, 0.12]])
    inf = np.inf
    c, sx, sy = oracle.range_aggregates_2d(z, H, [[-inf, inf, -inf, inf]])
    assert c[0] == pytest.approx(60, rel=1e-12)
    assert sx[0] == pytest.approx(z[:, 0].sum(), abs=1e-11) and sy[0] == pytest.approx(z[:, 1].sum(), abs=1e-11)
    lo, hi = np.array([-0.5, 0.2, 1.0]), np.array([0.8, 0.9, 4.0])
    c, sx, _ = oracle.range_aggregates_2d(z, H, np.stack([lo, hi, np.full(3, -inf), np.full(3, inf)], 1))
    c1, s1 = oracle.range_aggregates(z[:, 0], 0.4, lo, hi)
    assert np.allclose(c, c1, rtol=1e-11, atol=1e-13) and np.allclose(sx, s1, rtol=1e-11, atol=1e-13)
    boxes = np.array([[-1.0, 0.5, -0.3, 1.2], [0.0, 2.0, -2.0, 0.0], [-3.0, -1.0, 1.0, 3.0], [0.1, 0.1, 0.0, 1.0]])
    D = np.diag([0.2, 0.05])
    cd, sxd, syd = oracle.range_aggregates_2d(z, D, boxes)
    sd = np.sqrt(np.diag(D))
    for k, (a, b, cc, dd) in enumerate(boxes):
        pa = ndtr((b - z[:, 0]) / sd[0]) - ndtr((a - z[:, 0]) / sd[0])
        pb = ndtr((dd - z[:, 1]) / sd[1]) - ndtr((cc - z[:, 1]) / sd[1])
        assert cd[k] == pytest.approx(np.sum(pa * pb), rel=1e-11, abs=1e-14)
    cf, sxf, syf = oracle.range_aggregates_2d(z, H, boxes)
    assert cf[3] == 0.0 and sxf[3] == 0.0  # an empty box
    for k, (a, b, cc, dd) in enumerate(boxes[:3]):
        ref = sum(multivariate_normal.cdf([b, dd], mean=p, cov=H, lower_limit=[a, cc], abseps=1e-12,
                                          releps=1e-12, maxpts=10**6) for p in z)
        assert cf[k] == pytest.approx(ref, rel=1e-9, abs=1e-10)
    # additivity: [-1, 0.5] = [-1, 0] + [0, 0.5] in the first coordinate
    parts = oracle.range_aggregates_2d(z, H, [[-1.0, 0.0, -0.3, 1.2], [0.0, 0.5, -0.3, 1.2]])
    for whole, pr in zip((cf[0], sxf[0], syf[0]), parts):
        assert whole == pytest.approx(pr.sum(), rel=1e-11, abs=1e-13)
    # 2-D Simpson of the density over the first box
    a, b, cc, dd = boxes[0]
    g0, g1 = np.linspace(a, b, 241), np.linspace(cc, dd, 241)
    G0, G1 = np.meshgrid(g0, g1, indexing="ij")
    f = oracle.density_H(z, H, np.stack([G0.ravel(), G1.ravel()], 1)).reshape(G0.shape)

    def I2(v):
        return 60 * integrate.simpson(integrate.simpson(v, x=g1, axis=1), x=g0)

    assert cf[0] == pytest.approx(I2(f), rel=1e-8)
    assert sxf[0] == pytest.approx(I2(G0 * f), rel=1e-8, abs=1e-9)
    assert syf[0] == pytest.approx(I2(G1 * f), rel=1e-8, abs=1e-9)


def test_range_aggregates_2d_strong_correlation_and_errors():
    """rho = 0.995: COUNT against scipy's rectangle probability; boxes along
    and across the kernel's long axis.  Bad boxes and singular H fail."""
    from scipy.stats import multivariate_normal

    rng = np.random.Generator(np.random.PCG64(34))
    z = rng.standard_normal((30, 2))
    H = np.array([[0.04, 0.0398], [0.0398, 0.04]])
    boxes = np.array([[-0.5, 0.5, -0.5, 0.5], [-0.2, 0.3, 0.25, 0.6], [1.0, 1.5, -1.5, -1.0]])
    c, _, _ = oracle.range_aggregates_2d(z, H, boxes)
    for k, (a, b, cc, dd) in enumerate(boxes):
        ref = sum(multivariate_normal.cdf([b, dd], mean=p, cov=H, lower_limit=[a, cc], abseps=1e-12,
                                          releps=1e-12, maxpts=10**6) for p in z)
        assert c[k] == pytest.approx(ref, rel=1e-8, abs=1e-10)
    for bad in ([[1.0, 0.0, 0.0, 1.0]], [[0.0, 1.0, np.nan, 1.0]]):
        with pytest.raises(oracle.OracleError) as e:
            oracle.range_aggregates_2d(z, H, bad)
        assert e.value.code == oracle.INVAL
    with pytest.raises(oracle.OracleError) as e:
        oracle.range_aggregates_2d(z, [[1.0, 1.0], [1.0, 1.0]], [[0, 1, 0, 1]])
    assert e.value.code == oracle.DEGENERATE
    with pytest.raises(oracle.OracleError) as e:
        oracle.density_H(z, [[1.0, 2.0], [2.0, 1.0]], z[:2])
    assert e.value.code == oracle.DEGENERATE


def test_lscv_H_nelder_mead_path_matches_scipy_from_the_same_simplex():
    """The oracle's search step by step: from the start of eq. (LSCV-H-start)
    read as H0 = s^2 Sigma (Cholesky parameters, log-diagonal) and the stated
    initial steps, scipy's Nelder-Mead with the standard coefficients
    (reflection 1, expansion 2, contractions 1/2, shrink 1/2) reaches the same
    best vertex after the same number of evaluations; the initial simplex
    alone (max_evals = p + 1) gives one of its vertices, the one with the
    smallest g."""
    from scipy.optimize import minimize

    rng = np.random.Generator(np.random.PCG64(23))
    z = rng.standard_normal((300, 2)) @ np.array([[1.0, 0.0], [0.5, 0.7]]).T
    z[:90] = 0.5 * z[:90] + [2.0, -1.0]
    n, d = z.shape
    s = (4 / (d + 2)) ** (1 / (d + 4)) * n ** (-1 / (d + 4))
    C0 = np.linalg.cholesky(s * s * np.cov(z, rowvar=False))
    th0 = np.array([np.log(C0[0, 0]), C0[1, 0], np.log(C0[1, 1])])
    steps = np.array([0.25, 0.25 * np.sqrt(C0[0, 0] * C0[1, 1]), 0.25])
    simplex = np.vstack([th0] + [th0 + np.eye(3)[k] * steps[k] for k in range(3)])

    def H_of(th):
        C = np.array([[np.exp(th[0]), 0.0], [th[1], np.exp(th[2])]])
        return C @ C.T

    f = [oracle.lscv_H(z, H_of(t)) for t in simplex]
    H4, g4, ev4 = oracle.lscv_H_min(z, ftol=1e-300, xtol=1e-300, max_evals=4)
    assert ev4 == 4 and np.allclose(H4, H_of(simplex[int(np.argmin(f))]), rtol=1e-14) and g4 == min(f)
    for k in (12, 40, 90):
        # the oracle stops at the first step boundary with at least k
        # evaluations; scipy, given exactly that many, stops at the same one
        H, g, ev = oracle.lscv_H_min(z, ftol=1e-300, xtol=1e-300, max_evals=k)
        r = minimize(lambda t: oracle.lscv_H(z, H_of(t)), th0, method="Nelder-Mead",
                     options={"initial_simplex": simplex, "maxfev": ev, "xatol": 0.0, "fatol": 0.0,
                              "adaptive": False})
        assert ev >= k and ev == r.nfev, (k, ev, r.nfev)
        assert np.allclose(H, H_of(r.x), rtol=1e-9, atol=0) and g == pytest.approx(r.fun, rel=1e-12)
