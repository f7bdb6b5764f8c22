"""The continuous-batching server: results equal the same request run alone
(bitwise), admission respects slots and the HBM budget, stop cancels the
queue, and the synchronous calls refuse to run beside a server."""
import threading
import time

import numpy as np
import pytest

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


def _mix(kde, count=24, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    A = kde.KDE_METHOD_ROT | kde.KDE_METHOD_PLUGIN | kde.KDE_METHOD_LSCV
    reqs = []
    for k in range(count):
        n = int(np.exp(rng.uniform(np.log(300), np.log(60000))))
        fam = workloads.BATCH_FAMILIES[k % 4]
        x = workloads.draw(fam, n, 500 + k, np.float32 if k % 3 else np.float64)
        kind = k % 4
        if kind == 0:
            reqs.append(kde.Request(x, A, 3, workloads.BATCH_GRID))
        elif kind == 1:
            reqs.append(kde.Request(x, A, 2, np.geomspace(0.01, 2.0, 40)))
        elif kind == 2:
            reqs.append(kde.Request(x, kde.KDE_METHOD_LSCV, 3, ("paper", 64)))
        else:
            reqs.append(kde.Request(x, kde.KDE_METHOD_PLUGIN, 3))
    return reqs


def _check_same(r, a):
    assert r.status == a.status
    assert _same([r.h_rot, r.h_plugin, r.h_lscv], [a.h_rot, a.h_plugin, a.h_lscv])
    assert _same(r.plugin.psi, a.plugin.psi) and r.k_lscv == a.k_lscv
    if a.g is not None:
        assert _same(r.g, a.g) and _same(r.gscale, a.gscale)


def test_served_results_equal_alone_bitwise(kde):
    import torch

    reqs = _mix(kde)
    # a few device-resident columns as well
    reqs[5] = kde.Request(torch.from_numpy(np.asarray(reqs[5].x)).to("cuda:0"), reqs[5].methods, reqs[5].stages,
                          reqs[5].grid)
    torch.cuda.synchronize()
    with kde.Context(0) as srv, kde.Context(0) as ref:
        # a small iteration budget splits plug-in stages and LSCV passes of the
        # larger requests over many iterations
        srv.set_option("serve_iter_evals", 3_000_000_000)
        srv.server_start(8 << 30, 16)
        tickets = []
        for k, r in enumerate(reqs):  # staggered arrivals so requests join running iterations
            tickets.append(srv.submit(r))
            if k % 5 == 4:
                time.sleep(0.01)
        got = [srv.wait(t, timeout_s=120) for t in tickets]
        srv.server_stop()
        alone = [ref.batch([r])[0] for r in reqs]
    for r, a in zip(got, alone):
        assert r is not None
        assert r.status == kde.KDE_OK
        _check_same(r, a)
        assert r.t_queue_s >= 0 and r.t_service_s > 0


def test_submit_from_threads(kde):
    reqs = _mix(kde, count=12, seed=9)
    results = {}
    with kde.Context(0) as srv:
        srv.server_start(4 << 30, 8)
        lock = threading.Lock()

        def client(k):
            with lock:
                t = srv.submit(reqs[k])
            r = srv.wait(t, timeout_s=120)
            results[k] = r

        th = [threading.Thread(target=client, args=(k,)) for k in range(len(reqs))]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=180)
        srv.server_stop()
    assert len(results) == len(reqs) and all(r is not None and r.status == kde.KDE_OK for r in results.values())


def test_admission_budget_slots_and_nomem(kde):
    big = kde.Request(workloads.draw("normal", 200_000, 1, np.float32), kde.KDE_METHOD_LSCV, 3,
                      workloads.BATCH_GRID)
    small = [kde.Request(workloads.draw("gamma", 2000 + 10 * k, k, np.float32),
                         kde.KDE_METHOD_PLUGIN | kde.KDE_METHOD_LSCV, 3, workloads.BATCH_GRID) for k in range(6)]
    with kde.Context(0) as srv:
        srv.server_start(3 << 20, 1)  # 3 MB and one slot: small requests one at a time, big one too large
        tb = srv.submit(big)
        ts = [srv.submit(r) for r in small]
        rb = srv.wait(tb, timeout_s=60)
        rs = [srv.wait(t, timeout_s=60) for t in ts]
        srv.server_stop()
    assert rb.status == kde.KDE_E_NOMEM
    assert all(r.status == kde.KDE_OK for r in rs)
    # one slot: each later request waited for the earlier ones
    assert rs[-1].t_queue_s > rs[0].t_queue_s


def test_stop_cancels_queued_and_sync_calls_are_refused(kde):
    reqs = _mix(kde, count=10, seed=21)
    with kde.Context(0) as srv:
        srv.server_start(8 << 30, 1)
        ts = [srv.submit(r) for r in reqs]
        with pytest.raises(kde.KdeError) as e:
            srv.bw_rot(np.arange(10.0))
        assert e.value.status == kde.KDE_E_BUSY
        with pytest.raises(kde.KdeError) as e:
            srv.submit(kde.Request(np.array([1.0]), kde.KDE_METHOD_ROT))
        assert e.value.status == kde.KDE_E_INVAL
        srv.server_stop()
        out = [srv.wait(t, timeout_s=10) for t in ts]
        # after stop the synchronous calls work again
        assert srv.bw_rot(np.arange(10.0)) > 0
    st = [r.status for r in out]
    assert all(s in (kde.KDE_OK, kde.KDE_E_CANCELLED) for s in st)
    assert kde.KDE_E_CANCELLED in st
    with pytest.raises(kde.KdeError):
        srv.poll(ts[0])  # collected (and the context is closed)


def test_admission_uses_the_request_footprint(kde):
    """A request whose footprint equals the budget is served; one byte less
    and it completes with KDE_E_NOMEM."""
    r = kde.Request(workloads.draw("gamma", 5000, 11, np.float32), kde.KDE_METHOD_PLUGIN | kde.KDE_METHOD_LSCV, 3,
                    workloads.BATCH_GRID)
    with kde.Context(0) as srv:
        fp = srv.footprint(r)
        assert fp == kde.kde_request_footprint(r)  # default options
        srv.server_start(fp, 1)
        ok = srv.wait(srv.submit(r), timeout_s=60)
        srv.server_stop()
        srv.server_start(fp - 1, 1)
        no = srv.wait(srv.submit(r), timeout_s=60)
        srv.server_stop()
    assert ok.status == kde.KDE_OK and no.status == kde.KDE_E_NOMEM


def test_cancel_queued_and_admitted_requests(kde):
    """A queued request leaves the queue at once; an admitted one leaves at the
    end of the running iteration and frees its slot; the others complete with
    the results they have alone; a collected ticket cannot be cancelled."""
    long = kde.Request(workloads.draw("normal", 400_000, 2, np.float32), kde.KDE_METHOD_LSCV, 3,
                       workloads.BATCH_GRID)
    small = [kde.Request(workloads.draw("gamma", 3000 + 7 * k, 40 + k, np.float32),
                         kde.KDE_METHOD_PLUGIN | kde.KDE_METHOD_LSCV, 3, workloads.BATCH_GRID) for k in range(4)]
    with kde.Context(0) as srv, kde.Context(0) as ref:
        srv.set_option("serve_iter_evals", 1_000_000_000)
        srv.server_start(8 << 30, 1)  # one slot: the small requests queue behind the long one
        tl = srv.submit(long)
        ts = [srv.submit(r) for r in small]
        srv.cancel(ts[1])  # still queued
        time.sleep(0.3)
        srv.cancel(tl)  # admitted (about 1e13 evaluations, over a second of work)
        rl = srv.wait(tl, timeout_s=60)
        rs = [srv.wait(t, timeout_s=60) for t in ts]
        with pytest.raises(kde.KdeError) as e:
            srv.cancel(ts[0])
        assert e.value.status == kde.KDE_E_INVAL
        srv.server_stop()
        alone = [ref.batch([r])[0] for r in small]
    assert rl.status == kde.KDE_E_CANCELLED and 0 < rl.t_service_s < 1.0, (rl.status, rl.t_service_s)
    assert rs[1].status == kde.KDE_E_CANCELLED and rs[1].t_service_s == 0
    for k in (0, 2, 3):
        assert rs[k].status == kde.KDE_OK
        _check_same(rs[k], alone[k])


def test_failure_hook_fails_one_request_and_the_rest_complete(kde):
    """The host-forced failure hook: the named request ends with KDE_E_DEVICE,
    the requests that shared its launches complete with their results
    alone, its slot is released and the server keeps serving."""
    reqs = _mix(kde, count=6, seed=31)
    with kde.Context(0) as srv, kde.Context(0) as ref:
        srv.set_option("serve_fail_ticket", 3)
        srv.server_start(8 << 30, 8)
        ts = [srv.submit(r) for r in reqs]
        got = [srv.wait(t, timeout_s=120) for t in ts]
        again = srv.wait(srv.submit(reqs[2]), timeout_s=120)
        srv.server_stop()
        srv.set_option("serve_fail_ticket", 1)
        srv.server_start(8 << 30, 1)  # one slot: the second request needs the failed one's slot
        first = srv.wait(srv.submit(reqs[0]), timeout_s=120)
        second = srv.wait(srv.submit(reqs[1]), timeout_s=120)
        srv.server_stop()
        alone = [ref.batch([r])[0] for r in reqs]
    assert ts[2] == 3 and got[2].status == kde.KDE_E_DEVICE
    for k in (0, 1, 3, 4, 5):
        _check_same(got[k], alone[k])
    _check_same(again, alone[2])
    assert first.status == kde.KDE_E_DEVICE
    _check_same(second, alone[1])
