"""Tile pruning on sorted samples (option "prune"): the LSCV sums may drop only
tiles whose total is provably below 2^-34 of every sum, so results must agree
with the dense form far inside the tolerance and with the oracle to it; the
chosen grid index must not move; the evaluation count must shrink where
samples are spread, and be exact (performed + skipped = dense)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5
EPS = 2.0**-34


@pytest.fixture(scope="module")
def kde():
    import paper_1505_01998_amd as kde

    return kde


def _pair(kde, reqs):
    with kde.Context(0) as dense, kde.Context(0) as pr:
        pr.set_option("prune", 1)
        a = dense.batch(reqs)
        b = pr.batch(reqs)
    return a, b


@pytest.mark.parametrize("family,n,grid", [
    ("lognormal", 20011, np.geomspace(0.002, 0.6, 96)),
    ("bimodal", 4099, np.geomspace(0.01, 2.0, 40)),
    ("uniform", 257, np.geomspace(0.001, 0.3, 17)),
    ("mixture", 100_000, np.geomspace(0.005, 2.0, 256)),
])
def test_pruned_equals_dense_and_oracle(kde, family, n, grid):
    x = workloads.draw(family, n, 41, np.float32)
    req = kde.Request(x, kde.KDE_METHOD_LSCV | kde.KDE_METHOD_PLUGIN, 3, grid)
    (a,), (b,) = _pair(kde, [req])
    assert a.status == b.status == kde.KDE_OK
    # plug-in passes are not pruned: bitwise equal
    assert a.h_plugin == b.h_plugin and a.plugin.psi == b.plugin.psi
    # dense vs pruned: summation order differs (sorted samples) and at most
    # 2^-34 of each sum is dropped
    d = np.abs(a.g - b.g) / a.gscale
    assert d.max() <= 1e-7, d.max()
    assert b.k_lscv == a.k_lscv
    assert a.lscv_evals == a.lscv_evals_dense == pytest.approx(n * (n - 1) / 2 * grid.size, rel=1e-15)
    assert b.lscv_evals_dense == a.lscv_evals_dense and 0 < b.lscv_evals <= b.lscv_evals_dense
    if n <= 20011:
        o = oracle.lscv_curve(x, grid)
        assert np.all(np.abs(b.g - o.g) <= TOL * o.gscale)
        assert b.k_lscv == int(np.argmin(o.g)) or o.g[b.k_lscv] - o.g.min() <= 2 * np.abs(b.g - o.g).max()
    print(f"{family} n={n}: performed {b.lscv_evals / b.lscv_evals_dense:.3f} of the dense evaluations, "
          f"max |g_pruned - g_dense| / gscale {d.max():.2e}")


def test_pruning_skips_far_tiles_and_counts_exactly(kde):
    """Two far-apart clusters: every pair across them is negligible at small
    h, so about half the dense evaluations are skipped; the raw sums stay
    within the bound of the dense ones."""
    rng = np.random.Generator(np.random.PCG64(3))
    n = 30000
    x = np.concatenate([rng.normal(0.0, 1.0, n // 2), rng.normal(1000.0, 1.0, n - n // 2)]).astype(np.float32)
    rng.shuffle(x)
    grid = np.geomspace(0.01, 1.0, 32)
    (a,), (b,) = _pair(kde, [kde.Request(x, kde.KDE_METHOD_LSCV, 2, grid)])
    frac = b.lscv_evals / b.lscv_evals_dense
    assert frac < 0.6, frac
    assert b.lscv_evals == int(b.lscv_evals)  # an exact count
    with kde.Context(0) as dense, kde.Context(0) as pr:
        pr.set_option("prune", 1)
        s_d = dense.lscv_sums(x, grid)
        s_p = pr.lscv_sums(x, grid)
    for sd, sp in zip(s_d, s_p):
        assert np.all(sp <= sd * (1 + 1e-6)) and np.all(sd - sp <= 1e-6 * sd + EPS * sd)
    print(f"two clusters: performed {frac:.3f} of the dense evaluations")


def test_pruned_batch_results_equal_pruned_alone(kde):
    A = kde.KDE_METHOD_ROT | kde.KDE_METHOD_PLUGIN | kde.KDE_METHOD_LSCV
    reqs = [kde.Request(workloads.draw(f, 3000 + 1999 * k, 60 + k, np.float32), A, 3, workloads.BATCH_GRID)
            for k, f in enumerate(workloads.BATCH_FAMILIES)]
    with kde.Context(0) as pr:
        pr.set_option("prune", 1)
        batch = pr.batch(reqs)
        alone = [pr.batch([r])[0] for r in reqs]
    for a, b in zip(batch, alone):
        assert a.status == b.status == kde.KDE_OK
        assert np.array_equal(a.g, b.g) and a.k_lscv == b.k_lscv and a.lscv_evals == b.lscv_evals


def _same_result(r, a):
    assert r.status == a.status == 0
    assert [r.h_rot, r.h_plugin, r.h_lscv, r.k_lscv] == [a.h_rot, a.h_plugin, a.h_lscv, a.k_lscv]
    assert np.array_equal(r.g, a.g) and np.array_equal(r.gscale, a.gscale)
    assert r.lscv_evals == a.lscv_evals and r.lscv_evals_dense == a.lscv_evals_dense


def test_pruned_served_and_job_results_equal_pruned_batch(kde):
    """With the prune option the sort, near tiles and cuts of a column run in
    the server iteration (or job slice) where its LSCV work starts, and its
    pruned sweep is split over later ones: results and the count of
    evaluations performed are bitwise those of the pruned batch.  A pruned
    job's checkpoint resumes in another pruned job, not in a dense one."""
    A = kde.KDE_METHOD_ROT | kde.KDE_METHOD_PLUGIN | kde.KDE_METHOD_LSCV
    reqs = [kde.Request(workloads.draw(f, 20000 + 9001 * k, 80 + k, np.float32), A, 3, workloads.BATCH_GRID)
            for k, f in enumerate(workloads.BATCH_FAMILIES)]
    with kde.Context(0) as pr, kde.Context(0) as srv:
        pr.set_option("prune", 1)
        alone = [pr.batch([r])[0] for r in reqs]
        srv.set_option("prune", 1)
        srv.set_option("serve_iter_evals", 1_000_000_000)
        srv.set_option("serve_iter_ms", 20)  # budgets adapt between iterations; results may not
        srv.server_start(8 << 30, 4)
        tickets = [srv.submit(r) for r in reqs]
        served = [srv.wait(t, timeout_s=120) for t in tickets]
        srv.server_stop()
        sliced = []
        for r in reqs[:2]:
            with kde.Job(pr, r) as job:
                _, total, _ = job.progress()
                slices = 0
                while not job.run(total / 9):
                    slices += 1
                assert slices >= 5
                sliced.append(job.result())
        with kde.Job(pr, reqs[2]) as job:
            _, total, _ = job.progress()
            job.run(0.6 * total)
            assert not job.progress()[2]
            ck = job.checkpoint()
        with kde.Job(srv, reqs[2]) as job2:
            job2.resume(ck)
            resumed = job2.run_to_end(total / 4)
    with kde.Context(0) as dense:
        with kde.Job(dense, reqs[2]) as j3:
            with pytest.raises(kde.KdeError) as e:
                j3.resume(ck)
            assert e.value.status == kde.KDE_E_INVAL
    assert any(a.lscv_evals < 0.9 * a.lscv_evals_dense for a in alone)
    for r, a in zip(served, alone):
        _same_result(r, a)
    for r, a in zip(sliced, alone[:2]):
        _same_result(r, a)
    _same_result(resumed, alone[2])
    print("performed fractions: " + ", ".join(f"{a.lscv_evals / a.lscv_evals_dense:.3f}" for a in alone))


def test_search_with_pruning_per_step(kde):
    """The k-section search runs every step through the planner, so with the
    prune option each step's pass is pruned.  Near the minimum neighbouring g
    values differ by less than the pruning bound, so the two searches may
    take different brackets there (measured: 0.16% apart in h); both end at
    the same minimum value of g."""
    x = workloads.draw("mixture", 200_000, 44, np.float32)
    with kde.Context(0) as dense, kde.Context(0) as pr:
        pr.set_option("prune", 1)
        hd, infod = dense.bw_lscv_min(x, 1e-3, 1.0, 1e-4, 16)
        hp, infop = pr.bw_lscv_min(x, 1e-3, 1.0, 1e-4, 16)
    assert abs(infop["g"] - infod["g"]) <= 1e-7 * abs(infod["g"])
    assert abs(hp / hd - 1.0) <= 1e-2
    assert abs(infop["iterations"] - infod["iterations"]) <= 2


def test_pruned_degenerate_and_smallest_columns(kde):
    """With pruning on, a column of zero spread ends DEGENERATE and a
    two-sample column finishes, alone, in a batch, served and as a job."""
    L = kde.KDE_METHOD_LSCV
    reqs = [kde.Request(np.full(5000, 2.5, np.float32), L, 3, workloads.BATCH_GRID),
            kde.Request(np.array([0.0, 1.0], np.float32), L, 3, np.geomspace(0.1, 2.0, 8)),
            kde.Request(workloads.draw("bimodal", 7001, 90, np.float32), L, 3, workloads.BATCH_GRID)]
    with kde.Context(0) as pr:
        pr.set_option("prune", 1)
        alone = [pr.batch([r])[0] for r in reqs]
        batch = pr.batch(reqs)
        jobs = []
        for r in reqs:
            with kde.Job(pr, r) as job:
                jobs.append(job.run_to_end(1e8))
        pr.server_start(1 << 30, 4)
        served = [pr.wait(pr.submit(r), timeout_s=60) for r in reqs]
        pr.server_stop()
    assert [a.status for a in alone] == [kde.KDE_E_DEGENERATE, kde.KDE_OK, kde.KDE_OK]
    for got in (batch, jobs, served):
        assert [g.status for g in got] == [a.status for a in alone]
        for g, a in zip(got[1:], alone[1:]):
            assert np.array_equal(g.g, a.g) and g.k_lscv == a.k_lscv and g.lscv_evals == a.lscv_evals
