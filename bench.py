"""Throughput of the exact bandwidth-selection pair sums on one MI355X.

One step = the whole selector path on one resident sample column: moments and
rule of thumb, the three-stage plug-in chain (pairwise psi_8, psi_6, psi_4)
and the LSCV objective over the workload's bandwidth grid, with the argmin.
The metric counts pair-term evaluations: n(n-1)/2 per psi stage plus
n(n-1)/2 per LSCV grid point.

Prints one JSON line.  `roofline` reports the LSCV pair kernel (the dominant
kernel) against the transcendental issue rate of the chip, measured live with
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

# MI355X: 256 CUs at 2.4 GHz.  v_exp_f32 issues at a quarter of the 64-lane
# VALU rate: 16 lanes per clock per CU.  One LSCV (pair, h) term needs one exp.
CUS, CLOCK_HZ = 256, 2.4e9
EXP_PEAK = CUS * 16 * CLOCK_HZ            # 9.83e12 exp/s
FP32_PEAK_TFLOPS = 157.3                  # dense FP32 vector, packed issue
LSCV_FLOP_PER_EVAL = 5.0                  # mul + exp + add + fma(2)


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
    args = ap.parse_args()
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
            "peak": EXP_PEAK / 1e12,
            "unit": "Teval/s",
            "frac": achieved / EXP_PEAK,
            "traffic": None,
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
