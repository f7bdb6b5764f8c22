"""Write the FP64 oracle's values for the small columns of the 512-column batch.

Runs only the CPU oracle on every column of the batched workload with
n <= 20,000 (about 290 of the 512): rule-of-thumb h and sigma, the
three-stage plug-in chain (Section 4.4.1) and the LSCV objective g(h)
(Section 4.4.2) over the request's grid, 128 points log-spaced over
h_ROT * [1/64, 4].  The whole curve is computed; the file keeps its argmin,
the margin to the second-best point, and g, gscale at every 8th grid point
and at the argmin +-2.

Usage:  python tests/golden/make_batch_512.py [out.npz]     (about an hour on 8 cores)
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402

N_MAX = 20_000
FIXED = list(range(0, 128, 8)) + [127]


def main(out: str) -> None:
    lo, hi, n_h = workloads.BATCH_GRID[1:]
    specs = workloads.batch_columns()
    picks = [k for k, s in enumerate(specs) if s.n <= N_MAX]
    rows = {key: [] for key in ("col", "n", "sigma", "h_rot", "psi", "g_pilot", "h_plugin", "k_star", "margin",
                                "idx", "g", "gscale")}
    t0 = time.time()
    for m, k in enumerate(picks):
        x = specs[k].column()
        sigma, h_rot = oracle.bw_rot(x)
        p = oracle.bw_plugin(x, workloads.BATCH_STAGES)
        grid = h_rot * np.geomspace(lo, hi, n_h)
        c = oracle.lscv_curve(x, grid)
        ks, _, margin = oracle.argmin(c.g)
        idx = FIXED + [min(max(ks + d, 0), n_h - 1) for d in (-2, -1, 0, 1, 2)]
        for key, v in (("col", k), ("n", x.size), ("sigma", sigma), ("h_rot", h_rot), ("psi", p.psi),
                       ("g_pilot", p.g), ("h_plugin", p.h), ("k_star", ks), ("margin", margin), ("idx", idx),
                       ("g", c.g[idx]), ("gscale", c.gscale[idx])):
            rows[key].append(v)
        if (m + 1) % 20 == 0:
            print(f"{m + 1}/{len(picks)} columns, {time.time() - t0:.0f} s", flush=True)
    arrays = {key: np.asarray(v) for key, v in rows.items()}
    tmp = out + ".tmp.npz"
    np.savez_compressed(tmp, **arrays)
    os.replace(tmp, out)
    print(f"wrote {out}: {len(picks)} columns in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "batch_512_small_oracle.npz"))
