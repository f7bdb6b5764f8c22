"""LSCV bandwidth by search (kde_bw_lscv_min): the GPU's k-section search
against the oracle's same search.  The search's decisions compare g values,
so where two candidates are closer than the mixed form's error the paths may
part; the check is the continuous form of the near-tie rule: the oracle's g at
the GPU's bandwidth exceeds its own minimum by at most twice the GPU's measured
error there, and both lie inside the oracle's last bracket's neighbourhood."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def kde():
    import paper_1505_01998_amd as kde

    return kde


@pytest.mark.parametrize("family,n,lo,hi", [
    ("normal", 3001, 0.01, 2.0),
    ("bimodal", 5003, 0.005, 3.0),
    ("lognormal", 4097, 0.002, 1.0),
])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_search_matches_oracle(kde, family, n, lo, hi, precision):
    x = workloads.draw(family, n, 23, np.float32)
    tol, m = 1e-6, 16
    with kde.Context(0, precision) as c:
        h, info = c.bw_lscv_min(x, lo, hi, tol, m)
        g_gpu_at_h = c.lscv_curve(x, np.array([h]))[0][0]
    ho, go, steps, (a, b) = oracle.lscv_min(x, lo, hi, tol, m)
    o_h = oracle.lscv_curve(x, np.array([h]))  # one point per call: the grid must ascend
    o_ho = oracle.lscv_curve(x, np.array([ho]))
    err = abs(g_gpu_at_h - o_h.g[0]) / o_h.gscale[0]
    assert err <= TOL
    assert info["g"] == pytest.approx(g_gpu_at_h, rel=1e-12, abs=1e-15)
    # the GPU's bandwidth is as good as the oracle's up to twice the measured error
    assert o_h.g[0] - o_ho.g[0] <= 2 * max(err, 1e-15) * o_h.gscale[0] + 1e-15
    assert info["bracket"][1] / info["bracket"][0] - 1 <= tol
    assert info["evaluated"] == info["iterations"] * m
    if precision == "fp64":
        assert h == pytest.approx(ho, rel=1e-4) and info["iterations"] == steps
    print(f"{family} n={n} {precision}: h={h:.8f} oracle {ho:.8f}, rel {abs(h - ho) / ho:.1e}, "
          f"{info['iterations']} steps, {info['evaluated']} h evaluated")


def test_search_errors(kde):
    x = workloads.draw("gamma", 500, 1, np.float32)
    with kde.Context(0) as c:
        for bad in ((0.0, 1.0, 1e-3, 8), (1.0, 0.5, 1e-3, 8), (0.1, 1.0, 0.0, 8), (0.1, 1.0, 1e-3, 3),
                    (0.1, float("inf"), 1e-3, 8)):
            with pytest.raises(kde.KdeError) as e:
                c.bw_lscv_min(x, *bad)
            assert e.value.status == kde.KDE_E_INVAL


def test_search_on_the_bench_column(kde):
    """n = 1e6 lognormal: the search over the bench grid's range finds a
    bandwidth whose g is below every point of the 512-point grid (or ties
    within the error), with far fewer bandwidths evaluated."""
    w = workloads.workload("lognormal-1m")
    x = w.column()
    with kde.Context(0) as c:
        h, info = c.bw_lscv_min(x, w.grid[0], w.grid[-1], 1e-5, 16)
        g_grid, gs_grid, _ = c.lscv_curve(x, w.grid)
    k = int(np.argmin(g_grid))
    assert info["g"] <= g_grid[k] + 1e-8 * gs_grid[k]
    assert abs(np.log(h / w.grid[k])) <= np.log(w.grid[1] / w.grid[0])
    assert info["evaluated"] < w.grid.size / 3
    print(f"lognormal-1m search: h={h:.7f} (grid {w.grid[k]:.7f}), {info['iterations']} steps, "
          f"{info['evaluated']} h evaluated vs 512")
