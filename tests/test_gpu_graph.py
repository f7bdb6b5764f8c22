"""The graph option: a job's kernel launches are captured into a HIP graph
once and replayed by later jobs of the same signature.  Every replay is
checked bitwise against the same job run eagerly in another context, with
eager work and synchronisations between the replays; new samples, grid
values and device column addresses must reach a replay."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kde():
    import paper_1505_01998_amd as kde

    return kde


def _same(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return a.shape == b.shape and np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(a[~np.isnan(a)],
                                                                                               b[~np.isnan(b)])


def test_single_column_replays(kde):
    import torch

    grid = np.geomspace(0.02, 2.0, 40)
    with kde.Context(0) as g, kde.Context(0) as e:
        g.set_option("graph", 1)
        for rep in range(4):
            x = workloads.draw(workloads.BATCH_FAMILIES[rep], 5003, 100 + rep, np.float32)
            gg, gs, gh = g.lscv_curve(x, grid)
            ge, gse, ghe = e.lscv_curve(x, grid)
            assert _same(gg, ge) and _same(gs, gse) and _same(gh, ghe), rep
            # eager work between replays: torch kernels and another context
            y = torch.randn(1 << 20, device="cuda:0")
            (y * y).sum().item()
            e.bw_rot(x)
            torch.cuda.synchronize()
        captures, replays = g.graph_stats()
    assert (captures, replays) == (1, 3)
    o = oracle.lscv_curve(x, grid)
    assert np.all(np.abs(gg - o.g) <= 1e-5 * o.gscale)


def test_new_grid_values_and_device_addresses(kde):
    import torch

    keep = []
    with kde.Context(0) as g, kde.Context(0) as e:
        g.set_option("graph", 1)
        for rep in range(3):  # device columns at new addresses
            keep.append(torch.empty(1000 * (rep + 1), device="cuda:0"))  # moves the next allocation
            x = torch.from_numpy(workloads.draw("gamma", 12345, 7 + rep, np.float32)).to("cuda:0")
            keep.append(x)
            torch.cuda.synchronize()
            h1, info1 = g.bw_plugin(x, 3)
            h2, info2 = e.bw_plugin(x, 3)
            assert h1 == h2 and _same(info1.psi, info2.psi) and _same(info1.kappa, info2.kappa), rep
        assert g.graph_stats() == (1, 2)
        for rep in range(3):  # new grid values of the same size, alternating with a plug-in job
            g.bw_plugin(workloads.draw("normal", 777, rep, np.float32), 2)
            x = workloads.draw("bimodal", 12345, 30 + rep, np.float32)
            grid = np.geomspace(0.01 * (rep + 1), 3.0, 64)
            s1 = g.lscv_sums(x, grid)
            s2 = e.lscv_sums(x, grid)
            assert _same(s1[0], s2[0]) and _same(s1[1], s2[1]), rep
        # the LSCV job: one capture, then replays; the small plug-in job is
        # captured once more only if the first LSCV job grew the device buffers
        captures, replays = g.graph_stats()
        assert captures + replays == 9 and replays >= 4 and captures <= 4
    o = oracle.lscv_curve(x, grid)
    assert np.allclose(s1[0], o.s1, rtol=1e-5) and np.allclose(s1[1], o.s2, rtol=1e-5)


def test_batch_replays_and_signature_changes(kde):
    A = kde.KDE_METHOD_ROT | kde.KDE_METHOD_PLUGIN | kde.KDE_METHOD_LSCV

    def reqs(seed, n0=3000):
        out = []
        for k, f in enumerate(workloads.BATCH_FAMILIES):
            x = workloads.draw(f, n0 + 997 * k, seed + k, np.float32 if k % 2 else np.float64)
            out.append(kde.Request(x, A, 3, workloads.BATCH_GRID))
        out.append(kde.Request(np.array([1.0]), A, 3, workloads.BATCH_GRID))  # invalid: n < 2
        out.append(kde.Request(workloads.draw("normal", 4000, seed, np.float32), kde.KDE_METHOD_LSCV, 2,
                               np.geomspace(0.05, 1.0, 33)))
        return out

    with kde.Context(0) as g, kde.Context(0) as e:
        g.set_option("graph", 1)
        for rep, (seed, n0) in enumerate([(1, 3000), (2, 3000), (3, 3000), (4, 3100), (5, 3100)]):
            rg = g.batch(reqs(seed, n0))
            re_ = e.batch(reqs(seed, n0))
            for a, b in zip(rg, re_):
                assert a.status == b.status
                assert _same([a.h_rot, a.h_plugin, a.h_lscv], [b.h_rot, b.h_plugin, b.h_lscv])
                assert _same(a.plugin.psi, b.plugin.psi) and a.k_lscv == b.k_lscv
                if b.g is not None:
                    assert _same(a.g, b.g) and _same(a.gscale, b.gscale)
            assert rg[4].status == kde.KDE_E_INVAL
        captures, replays = g.graph_stats()
        # timing on: eager launches, no graph use
        g.set_timing(True)
        g.batch(reqs(9, 3100))
        assert g.graph_stats() == (captures, replays)
    # n0 changes the shapes once: two captures, three replays
    assert (captures, replays) == (2, 3)


def test_pruned_jobs_replay(kde):
    """With tile pruning the job's column sorts are kernels of the library, so
    a pruned job is captured and replayed like a dense one; every replay is
    bitwise the eager pruned job, evaluation counts included."""
    import torch

    grid = np.geomspace(0.002, 1.0, 64)
    A = kde.KDE_METHOD_ROT | kde.KDE_METHOD_PLUGIN | kde.KDE_METHOD_LSCV
    with kde.Context(0) as g, kde.Context(0) as e:
        for c in (g, e):
            c.set_option("prune", 1)
        g.set_option("graph", 1)
        for rep in range(3):
            cols = [workloads.draw(f, 6000 + 17 * k, 300 + 10 * rep + k, np.float32)
                    for k, f in enumerate(workloads.BATCH_FAMILIES)]
            reqs = [kde.Request(x, A, 3, grid) for x in cols]
            rg = g.batch(reqs)
            re_ = e.batch(reqs)
            for a, b in zip(rg, re_):
                assert a.status == b.status == kde.KDE_OK
                assert _same(a.g, b.g) and a.h_lscv == b.h_lscv and a.h_plugin == b.h_plugin, rep
                assert a.lscv_evals == b.lscv_evals < a.lscv_evals_dense
            y = torch.randn(1 << 18, device="cuda:0")
            (y * y).sum().item()
            torch.cuda.synchronize()
        captures, replays = g.graph_stats()
    assert (captures, replays) == (1, 2)
