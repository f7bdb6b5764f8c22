"""The estimate's consumers on the GPU (Section 3.2): density at query points
and range COUNT/SUM/AVG, against the oracle.

Tolerances: the density's mixed form sums FP32 terms (relative error of a
term ~ |u^2/2| 2^-23 for exponent u^2/2, random in sign) in compensated runs,
so 1e-5 relative plus 1e-12 of the peak density absolute (points far in the
tails); the FP64 form 1e-10.  Range aggregates are FP64 on both sides; they
differ in summation order and in how the difference of Phi is taken (tails on
the GPU), so 1e-9 relative plus 1e-9 of n absolute."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kde():
    import paper_1505_01998_amd as kde

    return kde


CASES = [("normal", 2, 0.5), ("bimodal", 4099, 0.2), ("lognormal", 20011, 0.05), ("mixture", 100_000, 0.07)]


@pytest.mark.parametrize("family,n,h", CASES)
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_density(kde, family, n, h, dtype, precision):
    x = workloads.draw(family, n, 31, dtype)
    pts = np.concatenate([np.linspace(float(x.min()) - 3, float(x.max()) + 3, 1500), np.asarray(x[:37], np.float64)])
    with kde.Context(0, precision) as c:
        f = c.density(x, h, pts)
    xe = np.asarray(x, np.float64)
    if precision == "mixed" and dtype == np.float64:
        # the mixed form keeps float64 samples as FP32 offsets from their mean
        m = float(np.mean(xe))
        xe = np.asarray(np.float32(xe - m), np.float64) + m
    o = oracle.density(xe, h, pts)
    rtol = 1e-5 if precision == "mixed" else 1e-10
    atol = 1e-12 * o.max()
    assert np.allclose(f, o, rtol=rtol, atol=atol), np.max(np.abs(f - o) / (np.abs(o) + atol))


@pytest.mark.parametrize("family,n,h", CASES)
def test_range_aggregates(kde, family, n, h):
    x = workloads.draw(family, n, 32, np.float32)
    xs = np.sort(np.asarray(x, np.float64))
    rng = np.random.Generator(np.random.PCG64(4))
    a = rng.choice(xs, 60) - rng.uniform(0, 2, 60)
    b = a + rng.exponential(1.0, 60)
    lo = np.concatenate([[-np.inf, xs[0] - 50, 3.0, -np.inf], a])
    hi = np.concatenate([[np.inf, xs[0] - 40, 3.0, float(np.median(xs))], b])
    with kde.Context(0) as c:
        cnt, sm, avg = c.range_aggregates(x, h, lo, hi)
    oc, osm = oracle.range_aggregates(x, h, lo, hi)
    assert np.allclose(cnt, oc, rtol=1e-9, atol=1e-9 * n)
    assert np.allclose(sm, osm, rtol=1e-9, atol=1e-9 * n * max(1.0, float(np.abs(xs).max())))
    assert cnt[0] == pytest.approx(n, rel=1e-12) and sm[0] == pytest.approx(float(xs.sum()), rel=1e-10)
    assert cnt[2] == 0.0 and np.isnan(avg[2])
    ok = oc > 1e-6 * n
    assert np.allclose(avg[ok], osm[ok] / oc[ok], rtol=1e-8)
    # a range below every sample: far-tail counts keep their digits
    assert cnt[1] == pytest.approx(oc[1], rel=1e-6, abs=1e-300)


def test_consumer_errors(kde):
    x = workloads.draw("gamma", 300, 1, np.float32)
    with kde.Context(0) as c:
        for call in (lambda: c.density(x, 0.0, [1.0]), lambda: c.density(x, 0.5, [np.nan]),
                     lambda: c.density(np.array([1.0, np.inf]), 0.5, [1.0]),
                     lambda: c.range_aggregates(x, 0.5, [2.0], [1.0]),
                     lambda: c.range_aggregates(x, -1.0, [0.0], [1.0])):
            with pytest.raises(kde.KdeError) as e:
                call()
            assert e.value.status == kde.KDE_E_INVAL
        # a column of zero spread still has a density
        f = c.density(np.full(10, 2.0, np.float32), 0.5, [2.0])
        assert f[0] == pytest.approx(1 / (0.5 * np.sqrt(2 * np.pi)), rel=1e-6)


def test_aqp_on_the_bench_column(kde):
    """n = 1e6 at the LSCV bandwidth: 4096 density points and 1024 ranges,
    against the oracle on sampled points and ranges."""
    import time

    w = workloads.workload("lognormal-1m")
    x = w.column()
    h = 0.0142678
    pts = np.linspace(0.0, 10.0, 4096)
    rng = np.random.Generator(np.random.PCG64(5))
    lo = rng.uniform(0, 8, 1024)
    hi = lo + rng.exponential(0.5, 1024)
    with kde.Context(0) as c:
        c.density(x, h, pts[:8])
        t0 = time.perf_counter()
        f = c.density(x, h, pts)
        t1 = time.perf_counter()
        cnt, sm, avg = c.range_aggregates(x, h, lo, hi)
        t2 = time.perf_counter()
    sel = np.arange(0, 4096, 128)
    o = oracle.density(x, h, pts[sel])
    assert np.allclose(f[sel], o, rtol=1e-5, atol=1e-12 * o.max())
    rs = np.arange(0, 1024, 64)
    oc, osm = oracle.range_aggregates(x, h, lo[rs], hi[rs])
    assert np.allclose(cnt[rs], oc, rtol=1e-9, atol=1e-3)
    assert np.allclose(sm[rs], osm, rtol=1e-9, atol=1e-2)
    print(f"n=1e6: density at 4096 points {1e3 * (t1 - t0):.1f} ms ({4096e6 / (t1 - t0):.3e} pair-terms/s), "
          f"1024 range aggregates {1e3 * (t2 - t1):.1f} ms")
