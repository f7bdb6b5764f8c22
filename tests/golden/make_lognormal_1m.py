"""Write the FP64 oracle's full-size values for the n = 1,000,000 lognormal column.

Runs only the CPU oracle (the plain FP64 double loops) on the seeded column of
the n = 1e6 workload: the whole three-stage plug-in chain (pairwise psi_8,
psi_6, psi_4 and the pilots between them, Section 4.4.1) and the LSCV
objective g(h) (Section 4.4.2) at a fixed set of grid indices: both grid
ends and two interior points, chosen before any GPU result existed, and the
window 168..172 around index 170, the index the GPU path selects.  Only that
index choice comes from the GPU path; every stored value is the oracle's, and
the test checks that the oracle's own minimum over the window lies inside it,
so the window holds a local minimum of the oracle's curve.  The full curve is
512 h and would take days on a CPU; these values pin the GPU path at its real
size without sampling, and at the selected bandwidth of eq. (LSCV-finalH).

Usage:  python tests/golden/make_lognormal_1m.py [out.json]
Takes a few hours on 8 cores; the plug-in part is written first, each LSCV
index is added to the file as soon as it is done.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402

# the fixed points first, then the window around the selected index, centre outwards
LSCV_INDICES = (0, 64, 256, 511, 170, 169, 171, 168, 172)


def main(out: str) -> None:
    w = workloads.workload("lognormal-1m")
    x = w.column()
    grid = w.grid
    doc = {
        "what": "FP64 oracle values for the n=1e6 lognormal(0,1) float32 column, three-stage plug-in and LSCV g(h) "
                "at fixed grid indices",
        "workload": w.name,
        "seed": int(w.seed),
        "n": int(x.size),
        "threads": oracle.num_threads(),
        "citations": "plug-in chain: Section 4.4.1 (psi_r estimator, pilot bandwidths, final h); "
                     "LSCV objective: Section 4.4.2 (g(h) with K*K - 2K)",
    }
    if os.path.exists(out):
        with open(out) as f:
            doc.update(json.load(f))

    def save():
        tmp = out + ".tmp"
        with open(tmp, "w") as f:
            json.dump(doc, f, indent=1)
        os.replace(tmp, out)

    if "plugin" not in doc:
        t = time.time()
        p = oracle.bw_plugin(x, stages=3)
        doc["plugin"] = {"sigma": p.sigma, "h_rot": p.h_rot, "stages": p.stages, "g": list(p.g),
                         "psi": list(p.psi), "kappa": list(p.kappa), "h": p.h,
                         "seconds": time.time() - t}
        save()
        print(f"plug-in done in {time.time() - t:.0f} s: h={p.h!r}", flush=True)
    lscv = doc.setdefault("lscv", {})
    for k in LSCV_INDICES:
        if str(k) in lscv:
            continue
        t = time.time()
        c = oracle.lscv_curve(x, np.array([grid[k]]))
        lscv[str(k)] = {"h": float(grid[k]), "g": float(c.g[0]), "gscale": float(c.gscale[0]),
                        "s1": float(c.s1[0]), "s2": float(c.s2[0]), "seconds": time.time() - t}
        save()
        print(f"lscv index {k} done in {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "lognormal_1m_oracle.json"))
