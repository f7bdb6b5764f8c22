"""LSCV_H at full bandwidth matrices (kde_lscv_H_eval) and its Nelder-Mead
search (kde_bw_lscv_H) against the oracle.  Tolerances as the univariate
pass: |dg| <= 1e-5 of the scale of the terms (mixed), 1e-10 (FP64).  The
search is compared on the value it reaches; in FP64 both sides take the same
steps from the same start, so the matrix itself must agree too."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kde():
    import paper_1505_01998_amd as kde

    return kde


def _sample(n, d, seed, dtype=np.float64):
    """A two-component Gaussian mixture with correlated coordinates."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.standard_normal((d, d)) + 2 * np.eye(d)
    comp = rng.random(n) < 0.35
    z = rng.standard_normal((n, d)) @ A.T
    z[comp] = 0.4 * z[comp] + 3.0
    return np.ascontiguousarray(z.astype(dtype))


def _matrices(x, k, seed):
    """k positive definite matrices around the rule-of-thumb s^2 Sigma:
    itself, its diagonal, and random rescaled and sheared versions.  The
    shear's size shrinks with d so that the matrices stay well conditioned
    (both sides lose about cond(H) * 1e-16 of g in FP64)."""
    n, d = x.shape
    S = np.atleast_2d(np.cov(x.astype(np.float64), rowvar=False))
    s = (4.0 / (d + 2)) ** (1.0 / (d + 4)) * n ** (-1.0 / (d + 4))
    H0 = s * s * S
    out = [H0, np.diag(np.diag(H0))]
    rng = np.random.Generator(np.random.PCG64(seed))
    while len(out) < k:
        B = np.eye(d) + 0.3 * np.sqrt(2.0 / max(d, 2)) * rng.standard_normal((d, d))
        out.append(np.exp(0.7 * rng.standard_normal()) * B @ H0 @ B.T)
    return np.stack(out[:k])


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 8, 12, 16])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_H_eval_matches_oracle(kde, d, precision):
    """Seven matrices a call, d = 1 ... 16."""
    n = 2003 if d <= 8 else 1201
    x = _sample(n, d, 20 + d, np.float32 if precision == "mixed" else np.float64)
    Hs = _matrices(x, 7, 5 + d)
    with kde.Context(0, precision) as c:
        g, gs = c.lscv_H_eval(x, Hs)
    o = np.array([oracle.lscv_H(x, H) for H in Hs])
    tol = 1e-5 if precision == "mixed" else 1e-10
    err = np.abs(g - o) / gs
    assert err.max() <= tol, err.max()
    assert np.all(gs >= np.abs(g))
    print(f"d={d} {precision}: max |dg|/gscale {err.max():.2e}")


@pytest.mark.parametrize("d", [2, 3, 6])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_H_eval_does_not_depend_on_the_batch(kde, d, precision):
    """One matrix a call, two, seven, and 67 (two passes of the 64-matrix
    limit) give the same g for the same matrix, bitwise."""
    x = _sample(1501, d, 3, np.float32 if precision == "mixed" else np.float64)
    Hs = _matrices(x, 67, 11)
    with kde.Context(0, precision) as c:
        g_all, _ = c.lscv_H_eval(x, Hs)
        g_one = np.array([c.lscv_H_eval(x, H)[0][0] for H in Hs[:7]])
        g_two = np.concatenate([c.lscv_H_eval(x, Hs[k:k + 2])[0] for k in range(0, 6, 2)])
        g_sev, _ = c.lscv_H_eval(x, Hs[:7])
    # every matrix is whitened for and swept on its own: bitwise the same
    assert np.array_equal(g_one, g_all[:7])
    assert np.array_equal(g_two, g_all[:6])
    assert np.array_equal(g_sev, g_all[:7])
    o = np.array([oracle.lscv_H(x, H) for H in Hs[60:]])
    with kde.Context(0, precision) as c:
        _, gs = c.lscv_H_eval(x, Hs[60:])
    assert np.all(np.abs(g_all[60:] - o) <= (1e-5 if precision == "mixed" else 1e-10) * gs)


def test_H_reductions_and_invariance(kde):
    """d = 1 with H = h^2 is the univariate objective; H = h^2 Sigma is the
    sphered LSCV_h at h; an affine map of the samples with H mapped alike
    divides g by |det A|."""
    x1 = _sample(3001, 1, 7)[:, 0]
    hs = np.array([0.05, 0.2, 0.7])
    z = _sample(2000, 3, 8)
    S = np.cov(z, rowvar=False)
    A = np.array([[2.0, 0.3, 0.0], [-0.5, 1.0, 0.7], [0.1, 0.0, -1.5]])
    Hs = _matrices(z, 5, 2)
    with kde.Context(0, "fp64") as c:
        gH, _ = c.lscv_H_eval(x1[:, None], (hs * hs)[:, None, None])
        g1, _, _ = c.lscv_curve(x1, hs)
        assert np.allclose(gH, g1, rtol=1e-10)
        gS, _ = c.lscv_H_eval(z, (hs * hs)[:, None, None] * S)
        gm, _, _ = c.lscv_md_curve(z, hs)
        assert np.allclose(gS, gm, rtol=1e-10)
        g0, _ = c.lscv_H_eval(z, Hs)
        ga, _ = c.lscv_H_eval(z @ A.T + [5.0, -3.0, 100.0], A @ Hs @ A.T)
        assert np.allclose(ga, g0 / abs(np.linalg.det(A)), rtol=1e-9)
    with kde.Context(0) as c:
        gH, gs = c.lscv_H_eval(x1[:, None].astype(np.float32), (hs * hs)[:, None, None])
        g1, gs1, _ = c.lscv_curve(x1.astype(np.float32), hs)
        assert np.all(np.abs(gH - g1) <= 1e-5 * gs1)


def test_H_eval_larger_column_against_oracle(kde):
    """n = 40,000 (many items a row, a ragged last tile): three matrices."""
    x = _sample(40_000, 2, 31, np.float32)
    Hs = _matrices(x, 3, 4)
    with kde.Context(0) as c:
        g, gs = c.lscv_H_eval(x, Hs)
    o = np.array([oracle.lscv_H(x, H) for H in Hs])
    err = np.abs(g - o) / gs
    assert err.max() <= 1e-5, err.max()
    print(f"n=40000 d=2: max |dg|/gscale {err.max():.2e}")


def test_H_eval_inputs_and_errors(kde):
    import torch

    x = _sample(1200, 2, 9, np.float32)
    Hs = _matrices(x, 3, 1)
    with kde.Context(0) as c:
        g, gs = c.lscv_H_eval(x, Hs)
        gd, _ = c.lscv_H_eval(torch.from_numpy(x).to("cuda:0"), Hs)
        assert np.array_equal(gd, g)
        # only the lower triangle is read
        Hu = Hs.copy()
        Hu[:, 0, 1] = 123.0
        assert np.array_equal(c.lscv_H_eval(x, Hu)[0], g)
        # a matrix that is not positive definite: +inf, scale 0; the others unchanged
        bad = np.array([[1.0, 2.0], [2.0, 1.0]])
        gb, gsb = c.lscv_H_eval(x, np.stack([Hs[0], bad, Hs[1]]))
        assert gb[1] == np.inf and gsb[1] == 0.0 and gb[0] == g[0] and gb[2] == g[1]
        for args in ((x, np.full((1, 2, 2), np.nan)), (_sample(100, 17, 1), np.eye(17)[None])):
            with pytest.raises(kde.KdeError) as e:
                c.lscv_H_eval(*args)
            assert e.value.status == kde.KDE_E_INVAL
        xn = x.copy()
        xn[7, 1] = np.nan
        with pytest.raises(kde.KdeError) as e:
            c.lscv_H_eval(xn, Hs)
        assert e.value.status == kde.KDE_E_INVAL
        col = np.stack([x[:, 0], 2 * x[:, 0] + 1], axis=1)
        with pytest.raises(kde.KdeError) as e:
            c.lscv_H_eval(col, Hs)
        assert e.value.status == kde.KDE_E_DEGENERATE
        with pytest.raises(kde.KdeError) as e:
            c.bw_lscv_H(x, ftol=0.0)
        assert e.value.status == kde.KDE_E_INVAL
        # the context is usable after the errors
        assert np.array_equal(c.lscv_H_eval(x, Hs)[0], g)


@pytest.mark.parametrize("d,n", [(1, 1500), (2, 1200), (3, 700), (4, 600), (5, 300)])
def test_search_fp64_follows_the_oracle(kde, d, n):
    x = _sample(n, d, 50 + d)
    with kde.Context(0, "fp64") as c:
        H, info = c.bw_lscv_H(x, max_evals=8000)
    Ho, go, evo = oracle.lscv_H_min(x, max_evals=8000)
    assert info.converged == 1
    assert abs(info.g - go) <= 1e-9 * abs(go), (info.g, go)
    assert np.linalg.norm(H - Ho) <= 1e-3 * np.linalg.norm(Ho), (H, Ho)
    assert abs(oracle.lscv_H(x, H) - info.g) <= 1e-10 * abs(go)
    print(f"d={d}: g {info.g:.12e} (oracle {go:.12e}), evals {info.evals} (oracle {evo}), passes {info.passes}")


def test_search_budget_stop_matches_the_oracle(kde):
    x = _sample(1000, 2, 77)
    with kde.Context(0, "fp64") as c:
        H, info = c.bw_lscv_H(x, max_evals=9)
    Ho, go, evo = oracle.lscv_H_min(x, max_evals=9)
    assert info.converged == 0 and info.evals == evo
    assert np.allclose(H, Ho, rtol=1e-9, atol=0) and info.g == pytest.approx(go, rel=1e-10)


@pytest.mark.parametrize("d", [2, 3])
def test_search_mixed_reaches_the_oracle_minimum(kde, d):
    x = _sample(2000, d, 90 + d, np.float32)
    with kde.Context(0) as c:
        H, info = c.bw_lscv_H(x, ftol=1e-7, xtol=1e-4)
    Ho, go, _ = oracle.lscv_H_min(x)
    g_at = oracle.lscv_H(x, H)
    assert info.converged == 1
    assert g_at - go <= 1e-6 * abs(go), (g_at, go)
    assert np.linalg.norm(H - Ho) <= 2e-2 * np.linalg.norm(Ho)
    print(f"d={d} mixed: oracle g at the found H {g_at:.10e}, oracle minimum {go:.10e}, evals {info.evals}")


@pytest.mark.parametrize("d", [2, 3, 4, 8])
def test_H_throughput(kde, d):
    """n = 1e5: one call with 64 matrices, then 16 calls with one matrix each
    (the search's usual step, staging included): (pair, matrix) evaluations
    per second."""
    import time

    n = 100_000
    x = _sample(n, d, 10, np.float32)
    Hs = _matrices(x, 64, 3)
    pairs = n * (n - 1) / 2
    with kde.Context(0) as c:
        c.lscv_H_eval(x, Hs[:4])
        t = time.perf_counter()
        g, _ = c.lscv_H_eval(x, Hs)
        t64 = time.perf_counter() - t
        t = time.perf_counter()
        for H in Hs[:16]:
            c.lscv_H_eval(x, H)
        t1 = (time.perf_counter() - t) / 16
    assert np.all(np.isfinite(g))
    print(f"d={d}: n=1e5, 64 matrices in one pass {t64:.3f} s, {pairs * 64 / t64:.3e} evals/s; "
          f"one matrix a call {t1 * 1e3:.2f} ms, {pairs / t1:.3e} evals/s")


@pytest.mark.parametrize("d,m", [(2, 11), (3, 5), (6, 3)])
def test_md_kernel_timing_counts_every_evaluation(kde, d, m):
    """With timing on, the d-dimensional pair launches report exactly
    m n(n-1)/2 (pair, matrix) evaluations for an m-matrix call (partial
    chunks included), and the LSCV_h curve n(n-1)/2 per bandwidth."""
    n = 3001
    x = _sample(n, d, 12, np.float32)
    Hs = _matrices(x, m, 3)
    with kde.Context(0) as c:
        c.set_timing(True)
        c.lscv_H_eval(x, Hs)
        launches, ms, evals = c.kernel_time("md_pairs")
        assert launches >= 1 and ms > 0 and evals == n * (n - 1) / 2 * m
        c.set_timing(True)
        c.lscv_md_curve(x, np.geomspace(0.05, 2.0, 37))
        assert c.kernel_time("md_pairs")[2] == n * (n - 1) / 2 * 37


@pytest.mark.parametrize("d", [2, 5])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_prepared_sample_equals_eval(kde, d, precision):
    """A prepared sample gives kde_lscv_H_eval's g bitwise, over several
    passes of matrices and between other calls on the context; it owns a copy
    of the samples (a device column may be freed after prepare); a later
    change of the context's precision is refused."""
    import torch

    x = _sample(6000, d, 80 + d, np.float32)
    H = _matrices(x, 70, 3 + d)
    other = _sample(3000, d, 90 + d, np.float32)
    with kde.Context(0, precision) as c:
        g_ref, gs_ref = c.lscv_H_eval(x, H)
        xd = torch.from_numpy(x).to("cuda:0")
        with c.lscv_H_prepare(xd) as prep:
            del xd
            torch.cuda.synchronize()
            g1, gs1 = prep.eval(H)
            c.lscv_H_eval(other, H[:5])  # reuses the context's workspace
            c.density_H(other, H[0], other[:10].astype(np.float64))
            g2, _ = prep.eval(H[3])
            g3, gs3 = kde.kde_lscv_H_eval_prepared(prep, H[::-1])
            c.set_precision("fp64" if precision == "mixed" else "mixed")
            with pytest.raises(kde.KdeError) as e:
                prep.eval(H[0])
            assert e.value.status == kde.KDE_E_INVAL
    assert np.array_equal(g1, g_ref) and np.array_equal(gs1, gs_ref)
    assert g2[0] == g_ref[3]
    assert np.array_equal(g3, g_ref[::-1]) and np.array_equal(gs3, gs_ref[::-1])
    with kde.Context(0) as c:
        with pytest.raises(kde.KdeError) as e:
            c.lscv_H_prepare(_sample(50, 17, 1))
        assert e.value.status == kde.KDE_E_INVAL
        with c.lscv_H_prepare(x) as prep:
            for bad in (np.full((d, d), np.nan), np.zeros((0, d, d))):
                with pytest.raises(kde.KdeError) as e:
                    prep.eval(bad)
                assert e.value.status == kde.KDE_E_INVAL


def test_context_close_releases_prepared_samples_and_jobs(kde):
    """Closing a context releases the prepared samples and resumable jobs
    created on it; closing those handles afterwards (explicitly, or when they
    are collected) does nothing."""
    import gc

    x = workloads.draw_matrix(3000, 2, 5, np.float32)
    col = workloads.draw("normal", 4000, 6, np.float32)
    c = kde.Context(0)
    prep = c.lscv_H_prepare(x)
    g0, _ = prep.eval(np.eye(2) * 0.2)
    job = kde.Job(c, kde.Request(col, kde.KDE_METHOD_ROT | kde.KDE_METHOD_LSCV, 3, ("log_rot", 0.25, 4.0, 16)))
    extra = c.lscv_H_prepare(x)
    c.close()
    assert prep.handle is None and extra.handle is None and job.job is None
    prep.close()
    job.close()
    del extra
    gc.collect()
    # a fresh context still works and gives the same value
    with kde.Context(0) as c2:
        with c2.lscv_H_prepare(x) as p2:
            g1, _ = p2.eval(np.eye(2) * 0.2)
    assert np.array_equal(g0, g1)
