"""kde_lscv_curve_noalloc against kde_lscv_curve, through the C ABI.

The allocation-free entry point runs the same job in the library's fixed
device scratch, so its g(h) and gscale(h) must equal kde_lscv_curve's on the
same context options bit for bit (a stricter bar than the 1e-5 * gscale the
path owes the FP64 oracle, which the oracle check below also applies).  Two
calls in a row, the second on a smaller column, check that a call does not
depend on what an earlier one left in the shared scratch; a request larger
than the scratch is refused before anything is enqueued."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kde():
    import paper_1505_01998_amd as kde

    return kde


def _curve_pair(kde, ctx, x, grid):
    g0, gs0, _ = ctx.lscv_curve(x, grid)
    g1, gs1 = ctx.lscv_curve_noalloc(x, grid)
    return g0, gs0, g1, gs1


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_noalloc_equals_lscv_curve_two_calls_second_smaller(kde, prec):
    import torch

    big = workloads.draw("bimodal", 70_001, 71, np.float32)
    small = workloads.draw("gamma", 5_003, 72, np.float32)
    grid_big = np.geomspace(0.004, 1.5, 200)
    grid_small = np.geomspace(0.01, 2.0, 37)
    with kde.Context(0, prec) as ctx:
        # first call: the larger column, on the device
        xd = torch.from_numpy(big).to("cuda:0")
        torch.cuda.synchronize()
        print(f"noalloc {prec}: n={big.size} n_h={grid_big.size} (device column)", flush=True)
        g0, gs0, g1, gs1 = _curve_pair(kde, ctx, xd, grid_big)
        assert np.array_equal(g0, g1) and np.array_equal(gs0, gs1)
        # second call: a smaller column from host memory, smaller grid
        print(f"noalloc {prec}: n={small.size} n_h={grid_small.size} (host column)", flush=True)
        g0s, gs0s, g1s, gs1s = _curve_pair(kde, ctx, small, grid_small)
        assert np.array_equal(g0s, g1s) and np.array_equal(gs0s, gs1s)
        # and the no-alloc result of the small column holds the oracle's bar
        oc = oracle.lscv_curve(small, grid_small)
        tol = 1e-5 if prec == "mixed" else 1e-10
        assert np.max(np.abs(g1s - oc.g) / oc.gscale) <= tol
        assert int(np.argmin(g1s)) == oracle.argmin(oc.g)[0]


def test_noalloc_default_grid_and_repeat(kde):
    x = workloads.draw("normal", 3_001, 73, np.float64)
    with kde.Context(0) as ctx:
        g0, gs0, _ = ctx.lscv_curve(x, None, 64)
        for _ in range(2):
            g1, gs1 = ctx.lscv_curve_noalloc(x, None, 64)
            assert np.array_equal(g0, g1) and np.array_equal(gs0, gs1)


def test_noalloc_holds_device_memory_steady(kde):
    import torch

    x = workloads.draw("uniform", 40_000, 74, np.float32)
    y = workloads.draw("normal", 9_000, 75, np.float32)
    grid = np.geomspace(0.002, 0.5, 96)
    with kde.Context(0) as ctx:
        ctx.lscv_curve_noalloc(x, grid)  # warm: code objects, runtime staging
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info(0)
        ctx.lscv_curve_noalloc(y, grid[:40])
        ctx.lscv_curve_noalloc(x, grid)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info(0)
    assert free0 - free1 <= 1 << 20, (free0, free1)


def test_noalloc_rejects_beyond_scratch_and_bad_arguments(kde):
    x = workloads.draw("normal", 400_000, 76, np.float32)
    grid = np.geomspace(0.001, 1.0, 512)
    with kde.Context(0) as ctx:
        with pytest.raises(kde.KdeError) as e:
            ctx.lscv_curve_noalloc(x, grid)
        assert e.value.status == kde.KDE_E_NOMEM
        assert "scratch" in str(e.value)
        with pytest.raises(kde.KdeError) as e:
            ctx.lscv_curve_noalloc(x[:1], grid)
        assert e.value.status == kde.KDE_E_INVAL
        with pytest.raises(kde.KdeError) as e:
            ctx.lscv_curve_noalloc(x[:100], grid[::-1].copy())
        assert e.value.status == kde.KDE_E_INVAL
        # the context still works normally afterwards, with its own buffers
        small = x[:2000].copy()
        g0, _, _ = ctx.lscv_curve(small, grid[:16])
        g1, _ = ctx.lscv_curve_noalloc(small, grid[:16])
        assert np.array_equal(g0, g1)
        ctx.set_option("autotune", 1)
        with pytest.raises(kde.KdeError) as e:
            ctx.lscv_curve_noalloc(small, grid[:16])
        assert e.value.status == kde.KDE_E_INVAL
