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

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402

# MI355X: 256 CUs at 2.4 GHz.  Per CU and clock the vector units retire 128
# FP32 lanes of add/mul/fma (157.3 TFLOP/s counting an FMA as 2) and 32 lanes
# of v_exp_f32.  Microbenchmarks on gfx950 show the two do not overlap: an
# exp occupies issue like ~3 plain FP32 ops.  One LSCV (pair, h) term is
# 1 mul + 1 exp + 1 add + 1 fma, so the term rate is bounded by
#   1 / (3 / (CUS * 128 * f) + 1 / (CUS * 32 * f)).
CUS, CLOCK_HZ = 256, 2.4e9
VALU_LANES, TRANS_LANES = 128, 32
LSCV_PEAK = 1.0 / (3.0 / (CUS * VALU_LANES * CLOCK_HZ) + 1.0 / (CUS * TRANS_LANES * CLOCK_HZ))  # 11.23e12/s
FP32_PEAK_TFLOPS = 157.3
LSCV_FLOP_PER_EVAL = 5.0                  # mul + exp + add + fma(2)

# HBM bytes per LSCV launch of this workload from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes, each scaled by the ratio the same counter shows for a
# plain 1 GiB copy (fetch x2.0, write x1.0).  Valid only for the kernel
# source they were taken on; reported as null once that source changes.
MEASURED_TRAFFIC = {
    "workload": "lognormal-1m",
    "kernels_sha256": "15e425ddff1f835919f6ed65dfd1992272f796e9c7fbe7784d404a3687a72d85",
    "fetch_bytes": 1.5053e7,
    "write_bytes": 3.2968e6,
}


def measured_traffic(workload: str):
    import hashlib

    src = os.path.join(ROOT, "paper_1505_01998_amd", "csrc", "kde_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    t = MEASURED_TRAFFIC
    if sha != t["kernels_sha256"] or workload != t["workload"]:
        return None
    return t["fetch_bytes"] + t["write_bytes"]


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
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lognormal-1m", choices=workloads.WORKLOADS)
    ap.add_argument("--precision", default="mixed", choices=("mixed", "fp64"))
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time (0 = skip)")
    ap.add_argument("--hc", type=int, default=-1, help="bandwidths per LSCV pass (8, 16, 32; -1 = default)")
    ap.add_argument("--seg", type=int, default=-1, help="j-range per work item (-1 = automatic, 0 = whole rows)")
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
    if args.hc > 0:
        ctx.set_option("lscv_hc", args.hc)
    if args.seg >= 0:
        ctx.set_option("seg", args.seg)

    def step():
        h_pi, info = ctx.bw_plugin(xd, w.stages)
        g, gs, _ = ctx.lscv_curve(xd, w.grid)
        return h_pi, info, g

    for i in range(args.warmup):
        log(f"warmup step {i + 1}/{args.warmup}")
        step()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        h_pi, info, g = step()
        log(f"timed step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, ms, evals_k = ctx.kernel_time("lscv_pairs")
    p_launches, p_ms, p_evals = ctx.kernel_time("psi_pairs")
    ctx.close()

    ms_step = dt * 1e3 / args.steps
    value = evals_step / (ms_step * 1e-3)
    achieved = evals_k / (ms * 1e-3)
    out = {
        "metric": "pair-kernel evals/s (LSCV+plug-in, n=1M)",
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "family": w.family, "n": n, "n_h": n_h, "plugin_stages": w.stages,
                   "precision": args.precision, "input_dtype": str(np.dtype(w.dtype))},
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": LSCV_PEAK / 1e12,
            "unit": "Teval/s",
            "frac": achieved / LSCV_PEAK,
            "traffic": measured_traffic(w.name),
            "traffic_unit": "bytes per launch",
            "kernel": "k_lscv_pairs_f32" if args.precision == "mixed" else "k_lscv_pairs_f64",
            "launches": launches,
            "avg_launch_ms": ms / max(launches, 1),
            "evals_per_launch": evals_k / max(launches, 1),
            "fp32_flop_frac": achieved * LSCV_FLOP_PER_EVAL / (FP32_PEAK_TFLOPS * 1e12),
        },
        "psi_kernel": {"launches": p_launches, "ms": p_ms, "evals": p_evals},
        "result": {"h_plugin": h_pi, "h_lscv": float(w.grid[int(np.argmin(g))]), "k_lscv": int(np.argmin(g))},
    }
    if args.cpu_budget > 0:
        out["cpu_baseline"] = cpu_baseline(w, x, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
