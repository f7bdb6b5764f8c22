"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (mixed precision):
  * h_rot, sigma: FP64 on both sides, 1e-12 relative.
  * psi_r, pilot g, plug-in h: 1e-5 relative.
  * g(h): |g_gpu - g_oracle| <= 1e-5 * gscale(h), where gscale is the same
    expression with the two pair sums added (the magnitude g is a difference
    of); |dg|/|g| is reported alongside.
  * raw pair sums s1, s2 (positive terms): 1e-5 relative, plus the FP32 range
    limit of the mixed form (pairs * 2^-126: a term below the smallest normal
    FP32 may flush to zero).
  * chosen grid index: equal to the oracle's argmin of eq. (LSCV-finalH).  A
    case may be named a near tie explicitly (none is); it then passes only if
    g_oracle[k_gpu] - min g_oracle <= 2 max|dg|, and the margin is printed.
FP64 form: 1e-10 on the same quantities.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOL64 = 1e-10


@pytest.fixture(scope="module")
def kde():
    import paper_1505_01998_amd as kde

    return kde


@pytest.fixture(scope="module")
def ctx(kde):
    c = kde.Context(0, "mixed")
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx64(kde):
    c = kde.Context(0, "fp64")
    yield c
    c.close()


def check_curve(g, gs, oc, tol, label=""):
    err = np.abs(g - oc.g) / oc.gscale
    assert np.all(np.isfinite(g)), label
    assert err.max() <= tol, (label, float(err.max()), int(err.argmax()))
    assert np.allclose(gs, oc.gscale, rtol=tol, atol=0), label
    return float(err.max())


def check_argmin(k_gpu, g_gpu, oc, label="", near_tie_ok=False):
    """The GPU selects the oracle's grid index.  Only a case passed with
    near_tie_ok may differ, by a margin within twice the measured error."""
    k_or, _, _ = oracle.argmin(oc.g)
    if k_gpu == k_or:
        return
    dg = float(np.abs(g_gpu - oc.g).max())
    margin = float(oc.g[k_gpu] - oc.g[k_or])
    print(f"{label}: GPU index {k_gpu}, oracle {k_or}, oracle margin {margin:.3e}, max |dg| {dg:.3e}")
    assert near_tie_ok, (label, k_gpu, k_or, margin, dg)
    assert margin <= 2 * dg, (label, k_gpu, k_or, margin, dg)


# ---------------------------------------------------------------- rule of thumb
@pytest.mark.parametrize("family,n,dtype", [
    ("normal", 1000, np.float64), ("mixture", 4097, np.float32), ("lognormal", 2, np.float32),
    ("gamma", 777, np.float64), ("uniform", 65536 + 3, np.float32)])
def test_rot(ctx, family, n, dtype):
    x = workloads.draw(family, n, 77 + n, dtype)
    s, h = oracle.bw_rot(x)
    assert ctx.bw_rot(x) == pytest.approx(h, rel=1e-12)


# ---------------------------------------------------------------- plug-in
@pytest.mark.parametrize("family,n,dtype,stages", [
    ("normal", 1000, np.float64, 2),      # the plain 1k workload
    ("normal", 1000, np.float64, 3),
    ("mixture", 5003, np.float32, 3),
    ("lognormal", 4096, np.float32, 3),
    ("bimodal", 257, np.float32, 2),
    ("uniform", 3, np.float64, 2),
    ("gamma", 12345, np.float32, 3),
])
def test_plugin(ctx, family, n, dtype, stages):
    x = workloads.draw(family, n, 1000 + n + stages, dtype)
    o = oracle.bw_plugin(x, stages)
    h, info = ctx.bw_plugin(x, stages)
    first = 0 if stages == 3 else 1
    for s in range(first, 3):
        assert info.g[s] == pytest.approx(o.g[s], rel=TOL), ("g", s)
        assert info.psi[s] == pytest.approx(o.psi[s], rel=TOL), ("psi", s, info.kappa[s])
        assert info.precision_used[s] in (0, 1)
    assert info.sigma == pytest.approx(o.sigma, rel=1e-12)
    assert h == pytest.approx(o.h, rel=TOL)


def test_plugin_fp64_form(ctx64):
    x = workloads.draw("mixture", 6001, 5, np.float32)
    o = oracle.bw_plugin(x, 3)
    h, info = ctx64.bw_plugin(x, 3)
    for s in range(3):
        assert info.psi[s] == pytest.approx(o.psi[s], rel=TOL64)
        assert info.precision_used[s] == 1
    assert h == pytest.approx(o.h, rel=TOL64)


# ---------------------------------------------------------------- LSCV
def test_lscv_plain_1k(ctx):
    w = workloads.workload("plain-1k")
    x = w.column()
    oc = oracle.lscv_curve(x, w.grid)
    g, gs, grid = ctx.lscv_curve(x, w.grid)
    assert np.array_equal(grid, w.grid)
    err = check_curve(g, gs, oc, TOL, "plain-1k")
    h, k, _ = ctx.bw_lscv(x, w.grid)
    check_argmin(k, g, oc, "plain-1k")
    assert h == w.grid[k]
    print(f"plain-1k max|dg|/gscale = {err:.3e}")


@pytest.mark.parametrize("family,n,dtype", [
    ("mixture", 3001, np.float32), ("lognormal", 10007, np.float32), ("bimodal", 256, np.float64),
    ("gamma", 513, np.float32), ("normal", 2, np.float32), ("uniform", 65, np.float64)])
def test_lscv_curve_and_sums(ctx, family, n, dtype):
    x = workloads.draw(family, n, 31 + n, dtype)
    grid = np.geomspace(0.004, 3.0, 37)
    oc = oracle.lscv_curve(x, grid)
    g, gs, _ = ctx.lscv_curve(x, grid)
    check_curve(g, gs, oc, TOL, family)
    s1, s2 = ctx.lscv_sums(x, grid)
    # FP32 terms: a term below the smallest normal FP32 (2^-126) may flush to zero
    atol = n * (n - 1) / 2 * 2.0**-126
    assert np.allclose(s1, oc.s1, rtol=TOL, atol=atol)
    assert np.allclose(s2, oc.s2, rtol=TOL, atol=atol)
    _, k, _ = ctx.bw_lscv(x, grid)
    check_argmin(k, g, oc, family)


@pytest.mark.parametrize("hc", [8, 16, 32])
@pytest.mark.parametrize("seg", [0, 512, 1536])
def test_lscv_tile_configs_agree(kde, hc, seg):
    """Every tuning configuration meets the oracle bar (n spans several rows and items)."""
    x = workloads.draw("mixture", 4099, 8, np.float32)
    grid = np.geomspace(0.01, 2.0, 41)
    oc = oracle.lscv_curve(x, grid)
    with kde.Context(0) as c:
        c.set_option("lscv_hc", hc)
        c.set_option("seg", seg)
        g, gs, _ = c.lscv_curve(x, grid)
    check_curve(g, gs, oc, TOL, f"hc={hc} seg={seg}")


@pytest.mark.parametrize("family,n", [("mixture", 4099), ("lognormal", 10007), ("bimodal", 65), ("normal", 2),
                                      ("uniform", 300)])
def test_lscv_matrix_core_variant(kde, family, n):
    """The LSCV kernel that forms exponent arguments on the matrix cores meets
    the same bar (including the masked diagonal, ragged tails and n_h not a
    multiple of the 16-bandwidth chunk)."""
    x = workloads.draw(family, n, 70 + n, np.float32)
    grid = np.geomspace(0.004, 3.0, 41)
    oc = oracle.lscv_curve(x, grid)
    with kde.Context(0) as c:
        c.set_option("lscv_mfma", 1)
        g, gs, _ = c.lscv_curve(x, grid)
        s1, s2 = c.lscv_sums(x, grid)
    check_curve(g, gs, oc, TOL, f"mfma {family} {n}")
    atol = n * (n - 1) / 2 * 2.0**-126
    assert np.allclose(s1, oc.s1, rtol=TOL, atol=atol)
    assert np.allclose(s2, oc.s2, rtol=TOL, atol=atol)


def test_lscv_fp64_form(ctx64):
    x = workloads.draw("lognormal", 3333, 12, np.float32)
    grid = np.geomspace(0.003, 2.0, 19)
    oc = oracle.lscv_curve(x, grid)
    g, gs, _ = ctx64.lscv_curve(x, grid)
    check_curve(g, gs, oc, TOL64, "fp64")


def test_lscv_default_grid(ctx):
    x = workloads.draw("gamma", 2500, 4, np.float64)
    og = oracle.default_grid(x, 0)
    g, gs, grid = ctx.lscv_curve(x, None, 0)
    assert grid.size == 150
    assert np.allclose(grid, og, rtol=1e-12)
    oc = oracle.lscv_curve(x, og)
    check_curve(g, gs, oc, TOL, "default grid")


def test_lscv_mixture_100k_sampled(ctx):
    """Full-size mixture workload (n = 100,000, 256 h): the whole curve on the
    GPU, the oracle on sampled grid points (each one by one)."""
    w = workloads.workload("mixture-100k")
    x = w.column()
    g, gs, _ = ctx.lscv_curve(x, w.grid)
    k = int(np.argmin(g))
    idx = sorted({0, 128, 255, max(0, k - 1), k, min(255, k + 1)})
    oc = oracle.lscv_curve(x, w.grid[idx])
    err = np.abs(g[idx] - oc.g) / oc.gscale
    assert err.max() <= TOL, err
    assert oc.g[idx.index(k)] <= oc.g.min() + 2 * np.abs(g[idx] - oc.g).max()
    print(f"mixture-100k sampled max|dg|/gscale = {err.max():.3e}")


GOLDEN_100K = os.path.join(os.path.dirname(__file__), "golden", "mixture_100k_oracle.json")


def _golden_100k():
    if not os.path.exists(GOLDEN_100K):
        return None
    ref = json.load(open(GOLDEN_100K))
    return ref if "lscv" in ref else None


@pytest.mark.skipif(_golden_100k() is None,
                    reason="full-grid oracle values not written yet (tests/golden/make_mixture_100k.py)")
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_mixture_100k_full_grid_against_stored_oracle(kde, precision):
    """The n = 1e5 mixture workload over its whole 256-point grid against the
    FP64 oracle's stored curve: every g(h) within the tolerance of gscale, the
    selected index of eq. (LSCV-finalH) equal to the oracle's over all 256
    points, and the three-stage plug-in chain (Section 4.4.1) within the
    tolerance of the oracle's psi, pilots and h."""
    ref = _golden_100k()
    w = workloads.workload("mixture-100k")
    x = w.column()
    assert np.allclose(w.grid, ref["lscv"]["h"], rtol=0, atol=0)
    with kde.Context(0, precision) as c:
        g, gs, _ = c.lscv_curve(x, w.grid)
        h, k, _ = c.bw_lscv(x, w.grid)
        h_pi, info = c.bw_plugin(x, 3)
    og, ogs = np.array(ref["lscv"]["g"]), np.array(ref["lscv"]["gscale"])
    tol = TOL if precision == "mixed" else TOL64
    err = np.abs(g - og) / ogs
    assert err.max() <= tol, (float(err.max()), int(err.argmax()))
    assert np.allclose(gs, ogs, rtol=tol, atol=0)
    k_or = ref["lscv"]["argmin"]
    assert int(np.argmin(g)) == k_or and k == k_or, (int(np.argmin(g)), k, k_or)
    assert h == w.grid[k_or]
    p = ref["plugin"]
    for s in range(3):
        tol_s = TOL if precision == "mixed" else TOL64 * max(1.0, p["kappa"][s])
        assert info.psi[s] == pytest.approx(p["psi"][s], rel=tol_s), s
        assert info.g[s] == pytest.approx(p["g"][s], rel=tol_s), s
    assert h_pi == pytest.approx(p["h"], rel=TOL if precision == "mixed" else TOL64 * max(p["kappa"]))
    print(f"mixture-100k full grid ({precision}): max |dg|/gscale {err.max():.2e}, k = {k} (oracle {k_or}, "
          f"margin {ref['lscv']['margin']:.2e}), psi rel "
          f"{[abs(info.psi[s] - p['psi'][s]) / abs(p['psi'][s]) for s in range(3)]}")


# ---------------------------------------------------------------- device columns, determinism, errors
def test_device_column_matches_host(ctx):
    import torch

    x = workloads.draw("bimodal", 5000, 2, np.float32)
    grid = np.geomspace(0.02, 1.0, 16)
    g_host, _, _ = ctx.lscv_curve(x, grid)
    xd = torch.from_numpy(x).to("cuda:0")
    torch.cuda.synchronize()
    g_dev, _, _ = ctx.lscv_curve(xd, grid)
    assert np.array_equal(g_host, g_dev)
    assert ctx.bw_plugin(xd, 3)[0] == ctx.bw_plugin(x, 3)[0]


def test_deterministic(ctx):
    x = workloads.draw("lognormal", 7777, 3, np.float32)
    grid = np.geomspace(0.01, 1.0, 23)
    a = ctx.lscv_curve(x, grid)[0]
    b = ctx.lscv_curve(x, grid)[0]
    assert np.array_equal(a, b)
    assert ctx.bw_plugin(x, 3)[1].psi == ctx.bw_plugin(x, 3)[1].psi


def test_error_paths(ctx, kde):
    with pytest.raises(kde.KdeError) as e:
        ctx.bw_rot(np.array([1.0]))
    assert e.value.status == kde.KDE_E_INVAL
    with pytest.raises(kde.KdeError) as e:
        ctx.bw_plugin(np.array([0.0, np.nan, 1.0]), 2)
    assert e.value.status == kde.KDE_E_INVAL
    with pytest.raises(kde.KdeError) as e:
        ctx.bw_plugin(np.full(100, 3.0), 2)
    assert e.value.status == kde.KDE_E_DEGENERATE
    with pytest.raises(kde.KdeError) as e:
        ctx.lscv_curve(np.arange(10.0), [0.5, 0.2])
    assert e.value.status == kde.KDE_E_INVAL
    with pytest.raises(kde.KdeError) as e:
        ctx.lscv_curve(np.arange(10.0), [0.5, -1.0])
    assert e.value.status == kde.KDE_E_INVAL
    with pytest.raises(kde.KdeError) as e:
        ctx.bw_plugin(np.arange(10.0), 4)
    assert e.value.status == kde.KDE_E_INVAL
    # the context still works after errors
    x = workloads.draw("normal", 100, 1, np.float64)
    assert ctx.bw_rot(x) == pytest.approx(oracle.bw_rot(x)[1], rel=1e-12)


def test_duplicates_contribute_kernel_at_zero(ctx):
    x = np.array([0.5, 0.5, 0.5, 2.0], dtype=np.float32)
    grid = np.array([0.1, 0.7])
    s1, s2 = ctx.lscv_sums(x, grid)
    oc = oracle.lscv_curve(x, grid)
    assert np.allclose(s1, oc.s1, rtol=1e-6) and np.allclose(s2, oc.s2, rtol=1e-6)


def test_timing_counters(kde):
    x = workloads.draw("normal", 20000, 9, np.float32)
    grid = np.geomspace(0.01, 1.0, 32)
    with kde.Context(0) as c:
        c.set_timing(True)
        c.lscv_curve(x, grid)
        launches, ms, evals = c.kernel_time("lscv_pairs")
    assert launches >= 1 and ms > 0
    assert evals == pytest.approx(20000 * 19999 / 2 * 32, rel=1e-12)


def test_lscv_lognormal_1m_sampled_items(kde):
    """The bench workload at full size (n = 1,000,000, 512 h) in the bench's
    launch configuration: the GPU's FP64 partial sums of sampled work items
    (blocks of the pair triangle) against the oracle's sums over the same
    blocks, on every 16th grid point."""
    w = workloads.workload("lognormal-1m")
    x = w.column()
    sel = [0, 1, 5000, -2, -1]
    with kde.Context(0) as c:
        n_items, ranges, sums = c.lscv_item_sums(x, w.grid, sel)
    assert n_items > 5000
    hk = np.arange(0, w.grid.size, 16)
    worst = 0.0
    for k, (i0, j0, j1) in enumerate(ranges):
        o1, o2 = oracle.lscv_block_sums(x, int(i0), int(i0) + 256, int(j0), int(j1), w.grid[hk])
        pairs = 256 * (min(int(j1), x.size) - int(j0))
        atol = pairs * 2.0**-126
        g1, g2 = sums[k, hk, 0], sums[k, hk, 1]
        assert np.allclose(g1, o1, rtol=TOL, atol=atol), (k, i0, j0, j1)
        assert np.allclose(g2, o2, rtol=TOL, atol=atol), (k, i0, j0, j1)
        m = o1 > 1e-20
        worst = max(worst, float(np.max(np.abs(g1[m] - o1[m]) / o1[m])))
    print(f"lognormal-1m sampled items: max rel err {worst:.3e} over {len(sel)} items x {hk.size} h")


GOLDEN_1M = os.path.join(os.path.dirname(__file__), "golden", "lognormal_1m_oracle.json")


@pytest.fixture(scope="module")
def lognormal_1m_curve(kde):
    """The mixed form's whole 512-point curve of the n = 1e6 bench column, as
    the bench computes it (one call over the whole grid)."""
    w = workloads.workload("lognormal-1m")
    x = w.column()
    with kde.Context(0) as c:
        g, gs, _ = c.lscv_curve(x, w.grid)
    return g, gs


@pytest.mark.skipif(not os.path.exists(GOLDEN_1M),
                    reason="full-size oracle values not written (tests/golden/make_lognormal_1m.py)")
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_lognormal_1m_full_size_oracle_values(kde, lognormal_1m_curve, precision):
    """The bench column at full size (n = 1,000,000) against the FP64 oracle's
    stored values: the whole three-stage plug-in chain and g(h) at the stored
    grid indices, among them the window k*-2 .. k*+2 around the selected
    index.  The selected index of eq. (LSCV-finalH) must be the oracle's
    minimum over the stored points (both grid ends, two interior points and
    the window), so it is a minimum of the oracle's curve over its +-2
    neighbours and below the other stored points.  The FP64 form's tolerance
    is 1e-10 times the stage's condition number for psi (a sum of terms of
    both signs) and 1e-10 of gscale for g."""
    ref = json.load(open(GOLDEN_1M))
    w = workloads.workload("lognormal-1m")
    x = w.column()
    idx = sorted(int(k) for k in ref.get("lscv", {}))
    with kde.Context(0, precision) as c:
        h, info = c.bw_plugin(x, 3)
        if precision == "mixed":
            g_full, _ = lognormal_1m_curve
            g = g_full[idx]
        elif idx:
            g, _, _ = c.lscv_curve(x, w.grid[idx])
    p = ref["plugin"]
    for s in range(3):
        tol = TOL if precision == "mixed" else TOL64 * max(1.0, p["kappa"][s])
        assert info.psi[s] == pytest.approx(p["psi"][s], rel=tol), s
        assert info.g[s] == pytest.approx(p["g"][s], rel=tol), s
    tol = TOL if precision == "mixed" else TOL64 * max(p["kappa"])
    assert h == pytest.approx(p["h"], rel=tol)
    assert info.sigma == pytest.approx(p["sigma"], rel=1e-12)
    worst = 0.0
    for a, k in enumerate(idx):
        v = ref["lscv"][str(k)]
        err = abs(g[a] - v["g"]) / v["gscale"]
        worst = max(worst, err)
        assert err <= (TOL if precision == "mixed" else TOL64), (k, g[a], v["g"])
    k_sel = int(np.argmin(lognormal_1m_curve[0]))
    win = [k for k in range(k_sel - 2, k_sel + 3) if str(k) in ref["lscv"]]
    o_g = np.array([ref["lscv"][str(k)]["g"] for k in idx])
    if len(win) == 5:
        # the oracle's minimum over the stored points, and the form's own
        assert idx[int(np.argmin(o_g))] == k_sel, (idx, k_sel)
        assert idx[int(np.argmin(g))] == k_sel, (idx, k_sel)
    print(f"lognormal-1m full size ({precision}): psi rel "
          f"{[abs(info.psi[s] - p['psi'][s]) / abs(p['psi'][s]) for s in range(3)]}, "
          f"h rel {abs(h - p['h']) / p['h']:.2e}, max |dg|/gscale {worst:.2e} over {len(idx)} h, "
          f"selected {k_sel}, oracle window {win}")


@pytest.mark.parametrize("family,n", [("bimodal", 4099), ("lognormal", 20011)])
def test_invariances_on_the_gpu(kde, ctx, family, n):
    """Shift, reflection and permutation leave sigma, psi_r and g(h) unchanged;
    scaling by a multiplies h_rot and h_PI by |a|, psi_r at the scaled pilot by
    |a|^-(r+1), and g_{ax}(|a| h) = g_x(h) / |a| (Section 4.4 definitions
    depend on the samples only through X_i - X_j).  Within the mixed form's
    tolerance; the power-of-two scale and shift keep the FP32 inputs exact."""
    x = workloads.draw(family, n, 77, np.float64)
    grid = np.geomspace(0.02, 2.0, 48)
    rng = np.random.Generator(np.random.PCG64(5))
    h0, i0 = ctx.bw_plugin(x, 3)
    g0, gs0, _ = ctx.lscv_curve(x, grid)
    for y in (x + 4.0, -x, x[rng.permutation(n)]):
        h1, i1 = ctx.bw_plugin(y, 3)
        g1, _, _ = ctx.lscv_curve(y, grid)
        assert i1.sigma == pytest.approx(i0.sigma, rel=1e-12)
        assert h1 == pytest.approx(h0, rel=TOL)
        for s in range(3):
            assert i1.psi[s] == pytest.approx(i0.psi[s], rel=TOL)
        assert np.all(np.abs(g1 - g0) <= TOL * gs0)
    a = -2.0
    h2, i2 = ctx.bw_plugin(a * x, 3)
    g2, _, _ = ctx.lscv_curve(a * x, abs(a) * grid)
    assert i2.h_rot == pytest.approx(abs(a) * i0.h_rot, rel=1e-12)
    assert h2 == pytest.approx(abs(a) * h0, rel=TOL)
    for s, r in enumerate((8, 6, 4)):
        assert i2.psi[s] == pytest.approx(i0.psi[s] * abs(a) ** -(r + 1), rel=TOL)
    assert np.all(np.abs(g2 - g0 / abs(a)) <= TOL * gs0 / abs(a))
    assert int(np.argmin(g2)) == int(np.argmin(g0))


def test_lognormal_1m_argmin_mixed_equals_fp64(kde, lognormal_1m_curve):
    """The bench column at full size: the mixed form's chosen grid index over
    all 512 h is the all-FP64 form's argmin over the chosen index +-6, and the
    two forms agree on that window to far below the tolerance."""
    w = workloads.workload("lognormal-1m")
    x = w.column()
    g, gs = lognormal_1m_curve
    k = int(np.argmin(g))
    win = np.arange(max(0, k - 6), min(w.grid.size, k + 7))
    with kde.Context(0, "fp64") as c64:
        g64, gs64, _ = c64.lscv_curve(x, w.grid[win])
    assert win[int(np.argmin(g64))] == k
    err = np.abs(g[win] - g64) / gs64
    print(f"lognormal-1m: k = {k}, max |g_mixed - g_fp64| / gscale on k+-6: {err.max():.2e}")
    assert err.max() <= TOL
