"""Write the FP64 oracle's values for a seeded 1% sample of the served
stream's small requests.

The served workload is the seeded Poisson stream of bandwidth-selection
requests (200 per second over 60 s, n log-uniform in [2e3, 2e6], the four
batch families).  Of its requests with n <= 20,000, a seeded 1% sample is
taken; for each, only the CPU oracle runs: rule-of-thumb h and sigma, the
three-stage plug-in chain (Section 4.4.1) and the LSCV objective g(h)
(Section 4.4.2) over the request's grid, 128 points log-spaced over
h_ROT * [1/64, 4].  The file keeps the whole curve (g and gscale), its argmin
and the margin to the second-best point.

Usage:  python tests/golden/make_served_sample.py [out.npz]     (about 10 min on 8 cores)
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
SAMPLE_SEED = 1998006  # the sample's own seed, apart from the stream's


def sample_indices(stream) -> list[int]:
    """Stream positions of the seeded 1% sample of the requests with n <= N_MAX."""
    small = [k for k, a in enumerate(stream) if a.spec.n <= N_MAX]
    m = max(1, int(np.ceil(0.01 * len(small))))
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    return sorted(int(k) for k in rng.choice(small, size=m, replace=False))


def main(out: str) -> None:
    lo, hi, n_h = workloads.BATCH_GRID[1:]
    stream = workloads.served_stream()
    picks = sample_indices(stream)
    print(f"{len(stream)} requests, {len(picks)} sampled", flush=True)
    rows = {key: [] for key in ("pos", "n", "sigma", "h_rot", "psi", "g_pilot", "h_plugin", "k_star", "margin",
                                "g", "gscale")}
    t0 = time.time()
    for m, k in enumerate(picks):
        x = stream[k].spec.column()
        sigma, h_rot = oracle.bw_rot(x)
        p = oracle.bw_plugin(x, workloads.BATCH_STAGES)
        grid = h_rot * np.geomspace(lo, hi, n_h)
        c = oracle.lscv_curve(x, grid)
        ks, _, margin = oracle.argmin(c.g)
        for key, v in (("pos", k), ("n", x.size), ("sigma", sigma), ("h_rot", h_rot), ("psi", p.psi),
                       ("g_pilot", p.g), ("h_plugin", p.h), ("k_star", ks), ("margin", margin), ("g", c.g),
                       ("gscale", c.gscale)):
            rows[key].append(v)
        if (m + 1) % 10 == 0:
            print(f"{m + 1}/{len(picks)} requests, {time.time() - t0:.0f} s", flush=True)
    arrays = {key: np.asarray(v) for key, v in rows.items()}
    tmp = out + ".tmp.npz"
    np.savez_compressed(tmp, **arrays)
    os.replace(tmp, out)
    print(f"wrote {out}: {len(picks)} requests in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "served_sample_oracle.npz"))
