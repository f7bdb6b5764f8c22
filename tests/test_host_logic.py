"""Host logic of the library on the CPU (no device touched): the planner's
cut of the i < j triangle into work items, the device footprint that the
server's admission compares with its budget, and the loud failure of a
context on a machine without a GPU."""
import numpy as np
import pytest

import paper_1505_01998_amd as kde


def _covered(n, seg, n_h=128):
    i0, jb, je, pr = kde.kde_plan_items(n, n_h, seg)
    count = np.zeros((n, n), np.int32)
    for a, b, e, p in zip(i0, jb, je, pr):
        assert a % 256 == 0 and (b - a) % 512 == 0 and (e - a) % 512 == 0 and b < e
        sub = 0
        for i in range(a, min(a + 256, n)):
            lo, hi = max(b, i + 1), min(e, n)
            if hi > lo:
                count[i, lo:hi] += 1
                sub += hi - lo
        assert sub == p
    assert np.all(np.diff(pr) <= 0), "items are not ordered longest first"
    return count, pr


@pytest.mark.parametrize("n", [2, 3, 255, 256, 257, 511, 512, 513, 1000, 3001])
@pytest.mark.parametrize("seg", [-1, 0, 512, 700, 1536])
@pytest.mark.parametrize("n_h", [0, 128])
def test_items_cover_the_triangle_exactly_once(n, seg, n_h):
    count, pr = _covered(n, seg, n_h)
    iu = np.triu_indices(n, 1)
    assert np.all(count[iu] == 1)
    assert count.sum() == n * (n - 1) // 2 == pr.sum()


@pytest.mark.parametrize("n,n_h", [(1_000_000, 512), (2_000_000, 128), (123_457, 256), (1_000_000, 0)])
def test_items_at_full_size(n, n_h):
    i0, jb, je, pr = kde.kde_plan_items(n, n_h, -1)
    assert pr.sum() == n * (n - 1) / 2
    assert np.all(pr > 0) and np.all(np.diff(pr) <= 0)
    assert i0.max() < n and jb.min() >= 0
    # the j-ranges of a row tile the row's span without overlap
    order = np.lexsort((jb, i0))
    a, b, e = i0[order], jb[order], je[order]
    same = a[1:] == a[:-1]
    assert np.all(b[1:][same] == e[:-1][same])
    rows = np.unique(a)
    assert rows.size == (n + 255) // 256


def test_plan_items_errors():
    for n, n_h in ((1, 10), (0, 10), (-5, 10), ((1 << 30) + 1, 10), (1000, -1), (1000, 65537)):
        with pytest.raises(kde.KdeError) as e:
            kde.kde_plan_items(n, n_h)
        assert e.value.status == kde.KDE_E_INVAL


def test_unit_count_is_bounded_for_very_large_columns():
    """The automatic cut lengthens items so that a pass holds at most 2^24
    units (items x 16-bandwidth chunks); at the workloads' sizes it does not
    act (the n = 1e6 cut is the launch-size rule's)."""
    m = kde.kde_plan_items(20_000_000, 512)[0].size
    assert m * 32 <= 1 << 24
    assert kde.kde_plan_items(20_000_000, 0)[0].size <= 1 << 24
    a = kde.kde_plan_items(1_000_000, 512)[2]
    b = kde.kde_plan_items(1_000_000, 16)[2]
    assert np.array_equal(a, b)


def test_footprint_grows_with_the_request():
    A = kde.KDE_METHOD_ROT | kde.KDE_METHOD_PLUGIN | kde.KDE_METHOD_LSCV

    def fp(n, methods=A, grid=("log_rot", 1 / 64, 4.0, 128), dtype=np.float32):
        return kde.kde_request_footprint(kde.Request(np.zeros(n, dtype), methods, 3, grid))

    sizes = [fp(n) for n in (1000, 10_000, 100_000, 1_000_000)]
    assert all(b > a for a, b in zip(sizes, sizes[1:]))
    assert fp(10_000, grid=("log_rot", 1 / 64, 4.0, 256)) > fp(10_000)
    assert fp(10_000, methods=kde.KDE_METHOD_ROT) < fp(10_000)
    assert fp(10_000, dtype=np.float64) > fp(10_000)
    # at least the padded FP32 copy and the FP64 partial slab of the LSCV pass
    n, n_h = 1_000_000, 128
    items = kde.kde_plan_items(n, n_h)[0].size
    assert fp(n) >= 4 * (n + 768) + 16 * n_h * items
    assert fp(n) % 256 == 0


def test_footprint_rejects_invalid_requests():
    bad = [
        kde.Request(np.zeros(1, np.float32), kde.KDE_METHOD_ROT),
        kde.Request(np.zeros(100, np.float32), kde.KDE_METHOD_PLUGIN, 4),
        kde.Request(np.zeros(100, np.float32), kde.KDE_METHOD_LSCV, 2, np.array([0.2, 0.1])),
        kde.Request(np.zeros(100, np.float32), kde.KDE_METHOD_LSCV, 2, ("log_rot", 2.0, 1.0, 10)),
    ]
    for r in bad:
        with pytest.raises(kde.KdeError) as e:
            kde.kde_request_footprint(r)
        assert e.value.status == kde.KDE_E_INVAL


def test_context_without_gpu_fails_loudly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(kde.KdeError) as e:
        kde.Context(0)
    assert e.value.status == kde.KDE_E_DEVICE
