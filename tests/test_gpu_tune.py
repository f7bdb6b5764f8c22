"""The tile autotuner of the LSCV pass: every variant it chooses between gives
bitwise the same sums, its decision is cached per shape, and a context that
tunes returns the same results as one that does not."""
import time

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kde():
    import paper_1505_01998_amd as kde

    return kde


def test_variants_bitwise_equal(kde):
    x = workloads.draw("gamma", 20011, 17, np.float32)
    grid = np.geomspace(0.01, 3.0, 100)  # not a multiple of 8, 16 or 32: padded last chunks
    out = {}
    with kde.Context(0) as c:
        for hc in (8, 16, 32):
            c.set_option("lscv_hc", hc)
            out[hc] = c.lscv_sums(x, grid)
        c.set_option("lscv_hc", 16)
        for tj in (256, 1024):
            c.set_option("lscv_tj", tj)
            out[(16, tj)] = c.lscv_sums(x, grid)
        with pytest.raises(kde.KdeError) as e:
            c.set_option("lscv_tj", 768)
        assert e.value.status == kde.KDE_E_INVAL
    for v in (8, 32, (16, 256), (16, 1024)):
        assert np.array_equal(out[v][0], out[16][0]) and np.array_equal(out[v][1], out[16][1]), v
    o = oracle.lscv_curve(x, grid)
    assert np.allclose(out[16][0], o.s1, rtol=1e-5) and np.allclose(out[16][1], o.s2, rtol=1e-5)


def test_autotune_choice_and_cache(kde):
    """Every variant of the persistent sweep runs and passes the tuner's
    bitwise parity gate; the choice is the default (16, 512) unless another
    variant is 3% faster; a second call for the same shape, or for a column in
    the same quarter octave of n, returns the cached decision at once."""
    with kde.Context(0) as c:
        t0 = time.perf_counter()
        choice, rates, parity = c.autotune(200_000, 128)
        t1 = time.perf_counter()
        again = c.autotune(200_000, 128)
        t2 = time.perf_counter()
        near = c.autotune(205_000, 128)
    print(f"autotune n=2e5 n_h=128: {choice} rates={ {k: f'{v:.3e}' for k, v in rates.items()} } "
          f"parity={parity} first {t1 - t0:.3f} s, cached {t2 - t1:.6f} s")
    assert choice in kde.TUNE_VARIANTS
    assert set(rates) == set(kde.TUNE_VARIANTS)
    assert all(v > 1e11 for v in rates.values())
    assert all(parity.values())
    # the default is kept unless another variant is 3% faster
    assert rates[choice] >= rates[(16, 512)]
    if choice != (16, 512):
        assert rates[choice] > 1.03 * rates[(16, 512)]
    assert again == (choice, rates, parity) and near == (choice, rates, parity)
    assert t2 - t1 < 0.05


def test_autotune_errors(kde):
    with kde.Context(0) as c:
        for n, nh in ((1, 10), (1000, 0), (1000, 70000)):
            with pytest.raises(kde.KdeError) as e:
                c.autotune(n, nh)
            assert e.value.status == kde.KDE_E_INVAL
    with kde.Context(0, "fp64") as c:
        with pytest.raises(kde.KdeError) as e:
            c.autotune(1000, 10)
        assert e.value.status == kde.KDE_E_INVAL


def test_autotuned_jobs_equal_default(kde):
    """A job large enough to be tuned (>= 1e13 pair-term evaluations) and a
    small one: the tuning context's results are bitwise the default's."""
    big = workloads.draw("bimodal", 400_000, 5, np.float32)
    grid = np.geomspace(0.002, 1.0, 128)
    small = [kde.Request(workloads.draw(f, 3000 + 7 * k, k, np.float32),
                         kde.KDE_METHOD_PLUGIN | kde.KDE_METHOD_LSCV, 3, workloads.BATCH_GRID)
             for k, f in enumerate(workloads.BATCH_FAMILIES)]
    with kde.Context(0) as tuned, kde.Context(0) as plain:
        tuned.set_option("autotune", 1)
        g_t, gs_t, _ = tuned.lscv_curve(big, grid)
        g_p, gs_p, _ = plain.lscv_curve(big, grid)
        r_t = tuned.batch(small)
        r_p = plain.batch(small)
        choice, _, _ = tuned.autotune(big.size, grid.size)  # cached by the first call
    assert np.array_equal(g_t, g_p) and np.array_equal(gs_t, gs_p)
    for a, b in zip(r_t, r_p):
        assert a.status == b.status == kde.KDE_OK
        assert a.h_lscv == b.h_lscv and a.h_plugin == b.h_plugin
        assert np.array_equal(a.g, b.g)
    assert choice in kde.TUNE_VARIANTS


def test_inner_loop_ceiling(kde):
    """The inner loop run from one LDS tile bounds the sweep: a full sweep of
    a column is no faster than it, within noise.  The tuner's steady-state
    trial runs the same loop (the same compiled instructions) on short rows
    of an evenly spread column and keeps the better of two rounds; it ranks
    variants against each other and is not an absolute rate, and it measures
    3-4% above the ceiling's launch on the part, so it is only checked to be
    the same rate within 10%."""
    import time

    x = workloads.draw("lognormal", 200_000, 9, np.float32)
    grid = np.geomspace(0.002, 0.6, 64)
    with kde.Context(0) as c:
        ceil16 = c.lscv_ceiling(16)
        ceil8 = c.lscv_ceiling(8)
        _, rates, _ = c.autotune(x.size, grid.size)
        c.lscv_curve(x, grid)
        t = time.perf_counter()
        c.lscv_curve(x, grid)
        dt = time.perf_counter() - t
        for bad in (0, 12, 64):
            with pytest.raises(kde.KdeError) as e:
                c.lscv_ceiling(bad)
            assert e.value.status == kde.KDE_E_INVAL
    sweep = x.size * (x.size - 1) / 2 * grid.size / dt
    assert ceil16 > 1e12 and ceil8 > 1e12
    assert sweep <= 1.05 * ceil16
    assert 0.9 * ceil16 <= rates[(16, 512)] <= 1.10 * ceil16
    print(f"inner-loop ceiling {ceil16:.3e} (hc 16), {ceil8:.3e} (hc 8); steady state {rates[(16, 512)]:.3e}; "
          f"sweep n=2e5 {sweep:.3e} evals/s")
