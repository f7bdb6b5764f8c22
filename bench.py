"""Throughput of the exact bandwidth-selection pair sums on one MI355X.

One step = the whole selector path on one resident sample column: moments and
rule of thumb, the three-stage plug-in chain (pairwise psi_8, psi_6, psi_4)
and the LSCV objective over the workload's bandwidth grid, with the argmin.
The metric counts pair-term evaluations: n(n-1)/2 per psi stage plus
n(n-1)/2 per LSCV grid point.

Prints one JSON line.  `roofline` reports the LSCV pair kernel (the dominant
kernel) against the issue-rate bound of its instruction mix, measured live with
HIP events around every launch of it; `cpu_baseline` times the FP64 oracle on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

T_START = time.perf_counter()

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402

# MI355X: 256 CUs at 2.4 GHz.  The published FP32 vector peak, 157.3 TFLOP/s
# counting an FMA as 2, is 128 FP32 lanes of add/mul/fma per CU and clock,
# reached with packed (two-wide) instructions; unpacked instructions retire
# half that, 64 lanes, and v_exp_f32 retires 32 lanes.  The library's
# issue-rate probe (kde_issue_rates, run in every default line) measures the
# unpacked and exp2 rates on the part (62.7 and 31.0 lanes per clock and CU).
# One LSCV (pair, h) term is 1 mul + 1 exp2 + 1 add + 1 fma.  The peak the
# roofline reports is the chip's bound for that mix at its published FP32
# rate, with the exponential not overlapping plain issue:
#   R = 1 / (3 / (CUS * 128 * f) + 1 / (CUS * 32 * f)) = 11.23e12 terms/s.
# This build compiles without packed FP32 instructions, so the ceiling it can
# reach is the same mix at the unpacked rate, R_unpacked = 7.86e12 terms/s;
# the line reports the kernel against both.
CUS, CLOCK_HZ = 256, 2.4e9
VALU_LANES, TRANS_LANES = 128, 32
UNPACKED_LANES = 64
LSCV_PEAK = 1.0 / (3.0 / (CUS * VALU_LANES * CLOCK_HZ) + 1.0 / (CUS * TRANS_LANES * CLOCK_HZ))  # 11.23e12/s
LSCV_PEAK_UNPACKED = 1.0 / (3.0 / (CUS * UNPACKED_LANES * CLOCK_HZ) + 1.0 / (CUS * TRANS_LANES * CLOCK_HZ))
# The psi pass at the same issue model.  With the samples pre-scaled by 1/g
# (one O(n) pass per stage) a pair needs sub, mul (w = u^2), mul (exp2
# argument), r/2 Horner ops for He_r in w and two fma (the term and its
# absolute value): 5 + r/2 plain FP32 instructions (PSI_PLAIN, r = 8, 6, 4)
# and one exp2.  Three stages of equal pair count, so the bound of the pass
# is their harmonic mean (6.55e12 pairs/s).
PSI_PLAIN = (9, 8, 7)
PSI_PEAK = 3.0 / sum(p / (CUS * VALU_LANES * CLOCK_HZ) + 1.0 / (CUS * TRANS_LANES * CLOCK_HZ) for p in PSI_PLAIN)
PSI_PEAK_UNPACKED = 3.0 / sum(p / (CUS * UNPACKED_LANES * CLOCK_HZ) + 1.0 / (CUS * TRANS_LANES * CLOCK_HZ)
                              for p in PSI_PLAIN)
FP32_PEAK_TFLOPS = 157.3
LSCV_FLOP_PER_EVAL = 5.0                  # mul + exp + add + fma(2)

# HBM bytes per LSCV launch of this workload from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes, each scaled by the ratio the same counter shows for a
# plain 1 GiB copy (fetch x2.0, write x1.0).  Valid only for the sources they
# were taken on; reported as null once those change.  The kernels, their
# shared header and the runtime (the planner sizes the units, and so the
# partial-sum writes; the persistent pass's grouping decides which die reads
# which part of the column) decide the traffic.  One launch is one whole
# LSCV pass of the step (the persistent form).
TRAFFIC_SOURCES = ("kde_internal.h", "kde_kernels.hip", "kde_runtime.hip")
MEASURED_TRAFFIC = {
    "workload": "lognormal-1m",
    "kernel": "k_lscv_units_f32_queue<16, 512>",
    "sources_sha256": "331fd9f42e6a0e5f0ee7c45868e630c3797f1e1b5cea1f62cb8610dc8401afd6",
    "fetch_bytes": 1.71920e+08,
    "write_bytes": 1.14624e+09,
}


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of the dominant kernel from the committed counter
    passes, or None when the workload, the kernel or its source has changed."""
    import hashlib

    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1505_01998_amd", "csrc", f), "rb").read())
    sha = h.hexdigest()
    t = MEASURED_TRAFFIC
    if sha != t["sources_sha256"] or workload != t["workload"] or kernel != t["kernel"]:
        return None
    return t["fetch_bytes"] + t["write_bytes"]


GOLDEN = {"lognormal-1m": os.path.join(ROOT, "tests", "golden", "lognormal_1m_oracle.json")}


def _rel(a, b):
    return abs(a - b) / abs(b)


def accuracy(kde, xd, w, h_pi, info, g, gs):
    """Error of the mixed form (outside the timed region): against the
    all-FP64 GPU form on the same column (the whole plug-in chain and g(h) at
    both grid ends, two interior indices and the chosen index +-6), and against
    the FP64 oracle's stored full-size values where they exist."""
    m = w.grid.size
    k = int(np.argmin(g))
    win = [j for j in range(k - 6, k + 7) if 0 <= j < m]
    idx = sorted({0, m // 8, m // 2, m - 1, *win})
    log(f"accuracy: FP64 GPU form, plug-in and g(h) at {len(idx)} grid points")
    with kde.Context(0, "fp64") as c64:
        t = time.perf_counter()
        h64, info64 = c64.bw_plugin(xd, w.stages)
        g64, gs64, _ = c64.lscv_curve(xd, w.grid[idx])
        t64 = time.perf_counter() - t
    g64_win = [g64[idx.index(j)] for j in win]
    stages = range(3 - w.stages, 3)
    out = {
        "vs_fp64_gpu": {
            "psi_order": [8, 6, 4][3 - w.stages:],
            "psi_rel": [_rel(info.psi[s], info64.psi[s]) for s in stages],
            "h_plugin_rel": _rel(h_pi, h64),
            "g_indices": idx,
            "g_err_over_gscale_max": max(abs(g[j] - g64[a]) / gs64[a] for a, j in enumerate(idx)),
            "argmin_in_window_same": win[int(np.argmin(g64_win))] == k,
            "window": win,
            "window_g_minus_min_over_gscale": [(g[j] - g[k]) / gs[k] for j in win],
            "window_fp64_g_minus_min_over_gscale": [(v - min(g64_win)) / gs64[idx.index(k)] for v in g64_win],
            "fp64_seconds": t64,
        },
        "vs_oracle": None,
    }
    path = GOLDEN.get(w.name)
    if path and os.path.exists(path):
        ref = json.load(open(path))
        o = {}
        if "plugin" in ref:
            o["psi_rel"] = [_rel(info.psi[s], ref["plugin"]["psi"][s]) for s in stages]
            o["h_plugin_rel"] = _rel(h_pi, ref["plugin"]["h"])
            o["fp64_gpu_psi_rel"] = [_rel(info64.psi[s], ref["plugin"]["psi"][s]) for s in stages]
        pts = {int(j): v for j, v in ref.get("lscv", {}).items() if int(j) in idx}
        if pts:
            o["g_indices"] = sorted(pts)
            o["g_err_over_gscale_max"] = max(abs(g[j] - v["g"]) / v["gscale"] for j, v in pts.items())
            o["fp64_gpu_g_err_over_gscale_max"] = max(abs(g64[idx.index(j)] - v["g"]) / v["gscale"]
                                                      for j, v in pts.items())
        out["vs_oracle"] = o
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, x, budget_s: float):
    """The FP64 oracle on the leading samples of the same column, full grid."""
    import oracle

    oracle.build(force=False)
    n_s = 2048
    t0 = time.perf_counter()
    oracle.lscv_curve(x[:n_s], w.grid)
    dt = time.perf_counter() - t0
    rate = n_s * (n_s - 1) / 2 * w.grid.size / dt
    # grow the sample so the timed oracle run takes about budget_s
    n_s = int(min(x.size, max(n_s, np.sqrt(2 * budget_s * rate / w.grid.size))))
    t0 = time.perf_counter()
    oracle.lscv_curve(x[:n_s], w.grid)
    dt = time.perf_counter() - t0
    evals = n_s * (n_s - 1) / 2 * w.grid.size
    return {
        "value": evals / dt,
        "unit": "pair-evals/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"LSCV g(h) over the full {w.grid.size}-point grid on the first {n_s} samples "
                  f"of the {w.name} column ({evals:.3e} evals, {dt:.1f} s)",
        "plain_1k": plain_1k_oracle_times(),
    }


def plain_1k_oracle_times(reps: int = 3):
    """The whole method on the CPU-sized workload (n = 1,000: rule of thumb,
    two-stage plug-in, LSCV over 100 h and its argmin) by the oracle, on one
    core and on all of them (mean seconds of `reps` runs)."""
    import oracle

    w = workloads.workload("plain-1k")
    x = w.column()

    def run():
        oracle.bw_rot(x)
        oracle.bw_plugin(x, w.stages)
        oracle.argmin(oracle.lscv_curve(x, w.grid).g)

    all_cores = oracle.num_threads()
    out = {}
    try:
        for tag, t in (("one_core_s", 1), ("all_cores_s", all_cores)):
            oracle.set_threads(t)
            run()
            t0 = time.perf_counter()
            for _ in range(reps):
                run()
            out[tag] = (time.perf_counter() - t0) / reps
    finally:
        oracle.set_threads(all_cores)
    out["cores"] = all_cores
    return out


def _requests_of(kde, cols, grid=None, stages=None):
    A = kde.KDE_METHOD_ROT | kde.KDE_METHOD_PLUGIN | kde.KDE_METHOD_LSCV
    return [kde.Request(x, A, stages or workloads.BATCH_STAGES, grid or workloads.BATCH_GRID) for x in cols]


def _apply_options(ctx, args):
    if args.hc > 0:
        ctx.set_option("lscv_hc", args.hc)
    if getattr(args, "tj", -1) > 0:
        ctx.set_option("lscv_tj", args.tj)
    if args.seg >= 0:
        ctx.set_option("seg", args.seg)
    if args.mfma >= 0:
        ctx.set_option("lscv_mfma", args.mfma)
    if args.autotune >= 0:
        ctx.set_option("autotune", args.autotune)
    if args.graph >= 0:
        ctx.set_option("graph", args.graph)
    if getattr(args, "persistent", -1) >= 0:
        ctx.set_option("persistent", args.persistent)
    if getattr(args, "prune", -1) >= 0:
        ctx.set_option("prune", args.prune)
    if getattr(args, "aging_ms", 0) > 0:
        ctx.set_option("serve_aging_ms", args.aging_ms)
    if getattr(args, "iter_evals", 0) > 0:
        ctx.set_option("serve_iter_evals", int(args.iter_evals))
    if getattr(args, "iter_ms", 0) > 0:
        ctx.set_option("serve_iter_ms", args.iter_ms)


def _lscv_kernel(ctx, args, n, n_h):
    """Name of the LSCV kernel the runs used (the autotuner's cached choice for
    the job's largest column when tuning is on)."""
    if args.precision != "mixed":
        return "k_lscv_units_f64<8>"
    if args.prune > 0:
        hc = ctx.autotune(n, n_h)[0][0] if args.autotune > 0 else (args.hc if args.hc > 0 else 16)
        return f"k_lscv_units_prune<{hc}>"
    if args.autotune > 0:
        hc, tj = ctx.autotune(n, n_h)[0]
        return f"k_lscv_units_f32_queue<{hc}, {tj}>"
    if args.mfma > 0:
        return "k_lscv_units_mfma"
    hc = args.hc if args.hc > 0 else 16
    tj = args.tj if getattr(args, "tj", -1) > 0 else 512
    # the dense pass runs as one persistent launch unless switched off
    return f"k_lscv_units_f32<{hc}>" if getattr(args, "persistent", -1) == 0 else f"k_lscv_units_f32_queue<{hc}, {tj}>"


def batch_bench(args):
    """512 uneven columns as one kde_batch job vs one call per column."""
    import torch

    import paper_1505_01998_amd as kde

    specs = workloads.batch_columns()
    cols = [torch.from_numpy(s.column()).to("cuda:0") for s in specs]
    torch.cuda.synchronize()
    reqs = _requests_of(kde, cols)
    n_h = workloads.BATCH_GRID[3]
    evals = sum(s.n * (s.n - 1) / 2 * (n_h + workloads.BATCH_STAGES) for s in specs)
    ctx = kde.Context(0, args.precision)
    _apply_options(ctx, args)
    for i in range(args.warmup):
        log(f"warmup {i + 1}/{args.warmup}")
        ctx.batch(reqs)
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = ctx.batch(reqs)
        log(f"batched step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    launches, ms, evals_k = ctx.kernel_time("lscv_pairs")
    assert all(r.status == kde.KDE_OK for r in out)
    t0 = time.perf_counter()
    for k, r in enumerate(reqs):
        ctx.batch([r])
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    log(f"plain per-column calls done in {t_plain:.1f} s")
    kernel = _lscv_kernel(ctx, args, max(s.n for s in specs), n_h)
    ctx.close()
    achieved = evals_k / (ms * 1e-3)
    return {
        "metric": "pair-kernel evals/s (batched 512 uneven columns)",
        "value": evals / t_batch,
        "unit": "pair-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_batch * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": "batch-512", "columns": len(specs), "n_range": [1000, 200000], "n_h": n_h,
                   "plugin_stages": workloads.BATCH_STAGES, "precision": args.precision,
                   "autotune": args.autotune > 0, "persistent": args.persistent != 0},
        "columns_per_s": len(specs) / t_batch,
        "plain": {"columns_per_s": len(specs) / t_plain, "value": evals / t_plain, "seconds": t_plain},
        "speedup_vs_plain": t_plain / t_batch,
        # plug-in stages whose pair sum was re-taken in FP64 (condition number
        # above the fp64_kappa threshold), of columns x stages
        "psi_fp64_reruns": {"stages": sum(1 for r in out for p in r.plugin.precision_used if p == kde.KDE_PREC_FP64),
                            "columns": sum(1 for r in out if kde.KDE_PREC_FP64 in r.plugin.precision_used),
                            "of_stages": len(out) * workloads.BATCH_STAGES, "of_columns": len(out)},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": LSCV_PEAK / 1e12, "unit": "Teval/s",
                     "frac": achieved / LSCV_PEAK, "traffic": None, "kernel": kernel,
                     "launches": launches, "avg_launch_ms": ms / max(launches, 1)},
    }


# Instruction-mix roofline of the LSCV_H sweep kernel at d = 2 (plain VALU at
# 128 lanes/clk/CU, exp2 at 32, not overlapped): per pair 2 differences, the
# squared norm (mul + fma), the two accumulations (add + fma) and one exp2.
LSCV_H_PEAK_D2 = 1.0 / (6.0 / (256 * 128 * 2.4e9) + 1.0 / (256 * 32 * 2.4e9))


def lscv_H_bench(args):
    """The LSCV_H search (Nelder-Mead over full 2x2 bandwidth matrices, one
    sweep of the pair kernel per evaluated matrix) on n = 1e5 two-dimensional
    samples; a step is one whole search from the rule-of-thumb start."""
    import torch

    import paper_1505_01998_amd as kde

    n, d = 100_000, 2
    x = workloads.draw_matrix(n, d, 1998010, np.float32)
    xd = torch.from_numpy(x).to("cuda:0")
    torch.cuda.synchronize()
    ctx = kde.Context(0, args.precision)
    opts = dict(ftol=1e-7, xtol=1e-4, max_evals=400)
    for i in range(args.warmup):
        log(f"warmup search {i + 1}/{args.warmup}")
        ctx.bw_lscv_H(xd, **opts)
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        H, info = ctx.bw_lscv_H(xd, **opts)
        log(f"timed search {i + 1}/{args.steps} done ({info.evals} evaluations)")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    launches, ms, evals_k = ctx.kernel_time("md_pairs")
    ctx.close()
    pairs = n * (n - 1) / 2
    peak = LSCV_H_PEAK_D2
    achieved = evals_k / (ms * 1e-3)
    out = {
        "metric": "(pair, matrix) evals/s (LSCV_H Nelder-Mead search, n=1e5, d=2)",
        "value": info.evals * pairs / dt,
        "unit": "pair-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": "lscv-H", "n": n, "d": d, "precision": args.precision, **opts},
        "search": {"evals": info.evals, "passes": info.passes, "converged": info.converged, "g": info.g,
                   "H": np.asarray(H).tolist()},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "Teval/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "k_HZ_units_f32<2>" if args.precision == "mixed" else "k_HZ_units_f64<2>",
                     "launches": launches, "avg_launch_ms": ms / max(launches, 1),
                     "evals_per_launch": evals_k / max(launches, 1)},
    }
    if args.cpu_budget > 0:
        import oracle

        oracle.build(force=False)
        Hs = np.asarray(H)
        n_s = 4000
        t0 = time.perf_counter()
        oracle.lscv_H(x[:n_s], Hs)
        rate = n_s * (n_s - 1) / 2 / (time.perf_counter() - t0)
        n_s = int(min(n, max(n_s, np.sqrt(2 * min(args.cpu_budget, 10.0) * rate))))
        t0 = time.perf_counter()
        oracle.lscv_H(x[:n_s], Hs)
        dt_o = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n_s * (n_s - 1) / 2 / dt_o, "unit": "pair-evals/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"g(H) at the found H on the first {n_s} samples ({dt_o:.1f} s)"}
    return out


def served_prefix(n_max: int, budget_s: float, evals_per_s: float, n_lo: float = 2e3, n_hi: float = 2e6,
                  rate: float = 200.0):
    """The longest prefix (at most n_max, at least 4 requests) of the seeded
    served stream whose four runs (plain and served, at the stream's arrival
    times and load-matched) are expected to fit budget_s at the measured pair
    throughput; the load-matched runs stretch the arrivals to 0.7x capacity.
    Measured on the part, the stream's requests (128 h, three plug-in stages,
    many small columns) run at about 0.9 of the single-column rate, and a
    load-matched run ends some seconds after its last arrival."""
    stream = workloads.served_stream(n_max, rate=rate, n_lo=n_lo, n_hi=n_hi)
    work = np.cumsum([a.spec.n * (a.spec.n - 1) / 2 * (workloads.BATCH_GRID[3] + workloads.BATCH_STAGES)
                      for a in stream]) / (0.87 * evals_per_s)
    est = work * (2.0 + 2.0 / 0.7) + 0.05 * np.arange(1, len(stream) + 1) + 10.0
    fit = int(np.searchsorted(est, budget_s, side="right"))
    return stream[:max(4, min(fit, len(stream)))]


def served_block(kde, args, stream, n_lo: float = 2e3, n_hi: float = 2e6):
    """Served form (continuous batching) vs plain per-request calls on a
    prefix of the seeded served stream (Poisson arrivals at args.rate, n
    log-uniform in [n_lo, n_hi], the four batch families; plug-in with three
    stages and LSCV over 128 h each): first at the stream's own arrival
    times, then load-matched at 0.7 x the plain form's measured capacity.
    Every served result is compared with the plain one."""
    import threading

    cols = [a.spec.column() for a in stream]
    reqs = _requests_of(kde, cols)
    n_h = workloads.BATCH_GRID[3]
    evals = sum(a.spec.n * (a.spec.n - 1) / 2 * (n_h + workloads.BATCH_STAGES) for a in stream)
    log(f"{elapsed():.0f} s: served: {len(reqs)} requests, {evals:.3e} pair-evals, "
        f"arrivals over {stream[-1].t:.2f} s")

    def pct(v, q):
        return float(np.percentile(np.asarray(v), q))

    def progress(tag, k, t_start):
        if k == len(reqs) or (k % max(1, len(reqs) // 8)) == 0:
            log(f"{elapsed():.0f} s: served: {tag} {k}/{len(reqs)} done ({time.perf_counter() - t_start:.1f} s)")

    def run_plain(ctx, times, tag):
        lat, res_all, t_start = [], [], time.perf_counter()
        for k, (r, t) in enumerate(zip(reqs, times)):
            now = time.perf_counter() - t_start
            if now < t:
                time.sleep(t - now)
            res = ctx.batch([r])[0]
            assert res.status == kde.KDE_OK
            res_all.append(res)
            lat.append(time.perf_counter() - t_start - t)
            progress(tag, k + 1, t_start)
        span = time.perf_counter() - t_start - times[0]
        return lat, span, res_all

    def run_served(ctx, times, tag):
        ctx.server_start(args.hbm_budget_gb << 30, args.slots)
        tickets = [None] * len(reqs)
        t_start = time.perf_counter()

        def feeder():
            for k, (r, t) in enumerate(zip(reqs, times)):
                now = time.perf_counter() - t_start
                if now < t:
                    time.sleep(t - now)
                tickets[k] = ctx.submit(r)

        th = threading.Thread(target=feeder)
        th.start()
        lat, done_at, res_all = [], [], []
        for k in range(len(reqs)):
            while tickets[k] is None:
                time.sleep(0.0005)
            res = ctx.wait(tickets[k])
            assert res.status == kde.KDE_OK, res.status
            res_all.append(res)
            lat.append(res.t_queue_s + res.t_service_s)
            done_at.append(time.perf_counter() - t_start)
            progress(tag, k + 1, t_start)
        th.join()
        ctx.server_stop()
        return lat, max(done_at) - times[0], res_all

    def summary(lat, span, _res):
        return {"req_per_s": len(lat) / span, "p50_s": pct(lat, 50), "p99_s": pct(lat, 99),
                "mean_s": float(np.mean(lat)), "makespan_s": span}

    def same(a, b):
        return all(x.h_lscv == y.h_lscv and x.h_plugin == y.h_plugin and np.array_equal(x.g, y.g)
                   for x, y in zip(a, b))

    out = {}
    ctx = kde.Context(0, args.precision)
    _apply_options(ctx, args)
    ctx.batch(reqs[:1])  # warm-up: code objects, allocations
    arrivals = [a.t for a in stream]
    lm_only = getattr(args, "lm_rate", 0.0) > 0
    if lm_only:
        # load-matched runs only, at a rate the caller states (0.7 x a plain
        # capacity measured elsewhere)
        lm_rate = args.lm_rate
    else:
        plain = run_plain(ctx, arrivals, "plain at arrival times")
        out["plain"] = summary(*plain)
        served = run_served(ctx, arrivals, "served at arrival times")
        out["served"] = summary(*served)
        lm_rate = 0.7 * out["plain"]["req_per_s"]
    scale = args.rate / lm_rate
    matched = [t * scale for t in arrivals]
    log(f"{elapsed():.0f} s: served: load-matched at {lm_rate:.3f} req/s")
    plain_lm = run_plain(ctx, matched, "plain load-matched")
    out["plain_load_matched"] = summary(*plain_lm)
    served_lm = run_served(ctx, matched, "served load-matched")
    out["served_load_matched"] = summary(*served_lm)
    ctx.close()
    ns = [a.spec.n for a in stream]
    res = {
        "requests": len(reqs),
        "stream": f"first {len(reqs)} requests of the seeded served stream (seed 1998005, Poisson {args.rate:g} "
                  f"req/s over 60 s, n log-uniform in [{n_lo:g}, {n_hi:g}]; this prefix has n from {min(ns)} to "
                  f"{max(ns)})",
        "pair_evals": evals,
        "load_matched_rate_req_s": lm_rate,
        **out,
        "speedup_req_s_load_matched": out["served_load_matched"]["req_per_s"] /
                                      out["plain_load_matched"]["req_per_s"],
        "results_bitwise_equal_plain": same(plain_lm[2], served_lm[2]) and
                                       (lm_only or same(plain[2], served[2])),
        "p99_note": f"p99 over {len(reqs)} latencies (linear interpolation between the two largest)"
                    if len(reqs) < 100 else f"p99 over {len(reqs)} latencies",
    }
    if not lm_only:
        res["speedup_req_s"] = out["served"]["req_per_s"] / out["plain"]["req_per_s"]
    return res


def served_bench(args):
    """The served block alone, as its own line."""
    import paper_1505_01998_amd as kde

    n_lo, n_hi = (2e3, 2e6) if args.workload == "served" else (2e3, 6e4)
    stream = workloads.served_stream(args.requests, rate=args.rate, n_lo=n_lo, n_hi=n_hi)
    blk = served_block(kde, args, stream, n_lo, n_hi)
    head = blk["served"] if "served" in blk else blk["served_load_matched"]
    return {
        "metric": "served req/s + p99 latency vs plain",
        "value": head["req_per_s"],
        "unit": "req/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": head["makespan_s"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": args.workload, "requests": blk["requests"], "rate_req_s": args.rate,
                   "n_range": [n_lo, n_hi], "n_h": workloads.BATCH_GRID[3], "plugin_stages": workloads.BATCH_STAGES,
                   "hbm_budget_gb": args.hbm_budget_gb, "slots": args.slots, "aging_ms": args.aging_ms,
                   "prune": args.prune > 0, "iter_evals": args.iter_evals or None, "iter_ms": args.iter_ms or None},
        "served": blk,
    }


def elapsed():
    return time.perf_counter() - T_START


def issue_probe(kde):
    """The device's measured issue rates (per clock and CU) next to the ones
    the roofline assumes."""
    with kde.Context(0) as c:
        r = c.issue_rates()
    return {**{k: r[k] for k in ("clock_hz", "cus")},
            "lanes_per_clk_cu": {k: r[k] for k in ("add_f32", "mul_f32", "fma_f32", "exp_f32")},
            "lscv_terms_per_clk_cu": {"spread": r["lscv_mix"], "zero": r["lscv_mix_zero"]},
            "assumed_lanes_per_clk_cu": {"plain_f32_packed": VALU_LANES, "plain_f32_unpacked": UNPACKED_LANES,
                                         "exp_f32": TRANS_LANES}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--budget-s", type=float, default=465.0,
                    help="wall-clock budget of the whole run from process start (s): warm-up stops after one step "
                         "longer than 10 s, and the timed steps are cut to what fits before the legs after them")
    ap.add_argument("--workload", default="lognormal-1m",
                    choices=workloads.WORKLOADS + ("batch-512", "served", "served-small", "lscv-H"))
    ap.add_argument("--requests", type=int, default=32, help="served workloads: requests taken from the stream")
    ap.add_argument("--served-requests", type=int, default=100,
                    help="single-column workloads: most requests of the served block carried in the same line "
                         "(0 = none); the prefix actually run is the longest that fits --served-budget-s")
    ap.add_argument("--served-budget-s", type=float, default=230.0,
                    help="single-column workloads: seconds of the budget reserved for the served block")
    ap.add_argument("--rate", type=float, default=200.0, help="served: arrival rate of the stream (req/s)")
    ap.add_argument("--lm-rate", type=float, default=0.0,
                    help="served workloads: run only the load-matched pair, at this rate (req/s; 0 = measure the "
                         "plain capacity first and run all four)")
    ap.add_argument("--hbm-budget-gb", type=int, default=64)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--aging-ms", type=int, default=0, help="served: aging time constant of the SRPT order (0 = off)")
    ap.add_argument("--ceiling", type=int, default=1,
                    help="after the timed steps, measure the LSCV kernel's steady-state rate, the ceiling of its "
                         "inner loop and the device's issue rates (0 = skip, e.g. under counter collection)")
    ap.add_argument("--iter-ms", type=int, default=0,
                    help="served: target duration of a server iteration in ms (0 = size by evaluations only)")
    ap.add_argument("--iter-evals", type=float, default=0,
                    help="served: pair-term evaluations per server iteration (0 = the library's default)")
    ap.add_argument("--precision", default="mixed", choices=("mixed", "fp64"))
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time (0 = skip)")
    ap.add_argument("--accuracy", type=int, default=1,
                    help="compare the mixed form with the all-FP64 GPU form after the timed steps (1/0)")
    ap.add_argument("--hc", type=int, default=-1, help="bandwidths per LSCV pass (8, 16, 32; -1 = default)")
    ap.add_argument("--tj", type=int, default=-1,
                    help="samples per LDS tile of the persistent LSCV sweep (256, 512, 1024; -1 = default)")
    ap.add_argument("--seg", type=int, default=-1, help="j-range per work item (-1 = automatic, 0 = whole rows)")
    ap.add_argument("--mfma", type=int, default=-1, help="LSCV arguments on the matrix cores (1/0; -1 = default)")
    ap.add_argument("--prune", type=int, default=-1,
                    help="LSCV tile pruning on sorted samples (1/0; -1 = default, off)")
    ap.add_argument("--graph", type=int, default=-1,
                    help="replay captured HIP graphs of repeated jobs (1/0; -1 = default, off)")
    ap.add_argument("--persistent", type=int, default=-1,
                    help="dense LSCV pass as one persistent launch over a device work queue (1/0; -1 = default, on)")
    ap.add_argument("--autotune", type=int, default=-1,
                    help="pick the LSCV variant with the tile autotuner (1/0; -1 = default, off)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        import torch

        a = torch.empty(args.copy_calibration // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; the path is not sharded across GPUs",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload == "batch-512":
        print(json.dumps(batch_bench(args)), flush=True)
        return
    if args.workload in ("served", "served-small"):
        print(json.dumps(served_bench(args)), flush=True)
        return
    if args.workload == "lscv-H":
        print(json.dumps(lscv_H_bench(args)), flush=True)
        return

    import torch

    import paper_1505_01998_amd as kde

    w = workloads.workload(args.workload)
    x = w.column()
    n, n_h = x.size, w.grid.size
    pairs = n * (n - 1) / 2
    evals_step = pairs * (n_h + w.stages)
    xd = torch.from_numpy(x).to("cuda:0")
    torch.cuda.synchronize()
    ctx = kde.Context(0, args.precision)
    _apply_options(ctx, args)
    log(f"{elapsed():.0f} s: set up {w.name}")

    skipped = []

    def step():
        if args.prune > 0:
            # one job for both selectors, so the performed LSCV evaluations come back
            r = ctx.batch([kde.Request(xd, kde.KDE_METHOD_PLUGIN | kde.KDE_METHOD_LSCV, w.stages, w.grid)])[0]
            assert r.status == kde.KDE_OK, r.status
            skipped.append((r.lscv_evals_dense - r.lscv_evals, r.lscv_evals / r.lscv_evals_dense))
            return r.h_plugin, r.plugin, r.g, r.gscale
        h_pi, info = ctx.bw_plugin(xd, w.stages)
        g, gs, _ = ctx.lscv_curve(xd, w.grid)
        return h_pi, info, g, gs

    # Reserve for the legs after the timed region (accuracy, served block,
    # CPU baseline, probes), scaled from the step time where it matters.
    t_step = None
    warm = 0
    for i in range(max(args.warmup, 0)):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        t_step = time.perf_counter() - t
        warm += 1
        log(f"{elapsed():.0f} s: warmup step {i + 1}/{args.warmup} took {t_step:.1f} s")
        if t_step > 10.0:
            break
    reserve = (15.0 if args.accuracy else 0.0) + (args.cpu_budget + 10.0 if args.cpu_budget > 0 else 0.0) + \
              (args.served_budget_s if args.served_requests > 0 else 0.0) + (15.0 if args.ceiling else 0.0)
    steps = args.steps
    if t_step is not None:
        fit = int((args.budget_s - elapsed() - reserve) // max(t_step, 1e-3))
        steps = max(1, min(args.steps, fit))
    if steps < args.steps:
        log(f"{elapsed():.0f} s: timing {steps} of the {args.steps} requested steps to stay within "
            f"{args.budget_s:.0f} s (step {t_step:.1f} s, {reserve:.0f} s reserved for the later legs)")
    # kernel timing brackets every launch with events, which the graph option
    # does not capture; with graphs the kernels are timed on one extra
    # (eager) step after the timed region
    use_graph = args.graph > 0
    if not use_graph:
        ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        h_pi, info, g, gs = step()
        if steps <= 20 or (i + 1) % 50 == 0:
            log(f"{elapsed():.0f} s: timed step {i + 1}/{steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    graph_stats = ctx.graph_stats()
    timed_skipped = sum(s for s, _ in skipped[-steps:]) if skipped else 0.0
    if use_graph:
        ctx.set_timing(True)
        step()
        torch.cuda.synchronize()
        timed_skipped = skipped[-1][0] if skipped else 0.0
    launches, ms, evals_k = ctx.kernel_time("lscv_pairs")
    p_launches, p_ms, p_evals = ctx.kernel_time("psi_pairs")
    kernel = _lscv_kernel(ctx, args, n, n_h)
    steady = ceiling = probe = None
    if args.ceiling and args.precision == "mixed" and args.prune <= 0 and args.mfma <= 0 and args.autotune <= 0:
        # outside the timed region: the same kernel's steady-state rate (the
        # tuner's trial: launches of B and 2B identical units, differenced),
        # the ceiling of its inner loop run from one LDS tile, and the issue
        # rates of the part
        hc = args.hc if args.hc > 0 else 16
        steady = ctx.autotune(n, n_h)[1][(hc, 512)]
        ceiling = ctx.lscv_ceiling(hc)
        probe = issue_probe(kde)
    ctx.close()
    log(f"{elapsed():.0f} s: timed region done ({steps} steps, {dt:.1f} s)")

    ms_step = dt * 1e3 / steps
    value = evals_step / (ms_step * 1e-3)
    # under pruning the kernel is credited only with the evaluations it performed
    performed_k = evals_k - timed_skipped
    achieved = performed_k / (ms * 1e-3)
    out = {
        "metric": "pair-kernel evals/s (LSCV+plug-in, n=1M)" if n == 1_000_000 else
                  f"pair-kernel evals/s (LSCV+plug-in, n={n})",
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": steps,
        "steps_requested": args.steps,
        "warmup": warm,
        "warmup_requested": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "family": w.family, "n": n, "n_h": n_h, "plugin_stages": w.stages,
                   "precision": args.precision, "input_dtype": str(np.dtype(w.dtype)), "autotune": args.autotune > 0,
                   "graph": use_graph, "graph_captures_replays": list(graph_stats), "prune": args.prune > 0,
                   "persistent": args.persistent != 0},
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": LSCV_PEAK / 1e12,
            "unit": "Teval/s",
            "frac": achieved / LSCV_PEAK,
            "traffic": measured_traffic(w.name, kernel),
            "traffic_unit": "bytes per launch",
            "kernel": kernel,
            "launches": launches,
            "avg_launch_ms": ms / max(launches, 1),
            "evals_per_launch": performed_k / max(launches, 1),
            "fp32_flop_frac": achieved * LSCV_FLOP_PER_EVAL / (FP32_PEAK_TFLOPS * 1e12),
            "peak_unpacked": LSCV_PEAK_UNPACKED / 1e12,
            "frac_of_peak_unpacked": achieved / LSCV_PEAK_UNPACKED,
            "steady_state": None if steady is None else steady / 1e12,
            "inner_loop_ceiling": None if ceiling is None else ceiling / 1e12,
            "frac_of_inner_loop_ceiling": None if ceiling is None else achieved / ceiling,
            "issue_probe": probe,
        },
        "psi_kernel": {"launches": p_launches, "ms": p_ms, "evals": p_evals,
                       "achieved": p_evals / (p_ms * 1e-3) / 1e12 if p_ms > 0 else None, "peak": PSI_PEAK / 1e12,
                       "unit": "Tpair/s", "frac": p_evals / (p_ms * 1e-3) / PSI_PEAK if p_ms > 0 else None,
                       "peak_unpacked": PSI_PEAK_UNPACKED / 1e12,
                       "frac_of_peak_unpacked": p_evals / (p_ms * 1e-3) / PSI_PEAK_UNPACKED if p_ms > 0 else None},
        "result": {"h_plugin": h_pi, "h_lscv": float(w.grid[int(np.argmin(g))]), "k_lscv": int(np.argmin(g))},
        "prune": None if args.prune <= 0 else {
            "performed_frac": skipped[-1][1],
            "performed_evals_per_s": (pairs * n_h * skipped[-1][1] + pairs * w.stages) / (ms_step * 1e-3),
            "note": "value counts the dense method's evaluations; roofline.achieved counts the evaluations the "
                    "pruned sweep performed (every skipped tile's total is below 2^-34 of every sum)"},
    }
    if args.accuracy and args.precision == "mixed":
        out["accuracy"] = accuracy(kde, xd, w, h_pi, info, g, gs)
        log(f"{elapsed():.0f} s: accuracy leg done")
    del xd
    torch.cuda.empty_cache()
    if args.served_requests > 0:
        # the longest stream prefix whose four runs fit the served block's
        # share of the budget at the throughput just measured
        left = args.budget_s - elapsed() - (args.cpu_budget + 10.0 if args.cpu_budget > 0 else 0.0)
        stream = served_prefix(args.served_requests, max(20.0, min(args.served_budget_s, left)), value)
        out["served"] = served_block(kde, args, stream)
        log(f"{elapsed():.0f} s: served block done")
    if args.cpu_budget > 0:
        # at least 10 s of oracle work (or all of --cpu-budget, if smaller),
        # even when the legs before ran over their share
        left = args.budget_s - elapsed() - 10.0
        out["cpu_baseline"] = cpu_baseline(w, x, max(min(10.0, args.cpu_budget), min(args.cpu_budget, left / 2)))
        log(f"{elapsed():.0f} s: cpu baseline done")
    out["wall_s"] = elapsed()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
