"""Write the FP64 oracle's values for the whole n = 100,000 mixture workload.

Runs only the CPU oracle (the plain FP64 double loops) on the seeded column of
the n = 1e5 workload: the three-stage plug-in chain (pairwise psi_8, psi_6,
psi_4 and the pilots between them, Section 4.4.1) and the LSCV objective g(h)
(Section 4.4.2) at every one of the 256 grid points, with the argmin of
eq. (LSCV-finalH) over the whole grid.  Nothing here reads a GPU result.

Usage:  python tests/golden/make_mixture_100k.py [out.json]
About 35 minutes on 8 cores (1.28e12 pair-bandwidth terms, two FP64
exponentials each).
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

CHUNK = 16


def main(out: str) -> None:
    w = workloads.workload("mixture-100k")
    x = w.column()
    grid = w.grid
    doc = {
        "what": "FP64 oracle values for the n=1e5 mixture 0.5N(-2,0.5^2)+0.5N(1,1) float32 column: three-stage "
                "plug-in and LSCV g(h) over the whole 256-point grid",
        "workload": w.name,
        "seed": int(w.seed),
        "n": int(x.size),
        "threads": oracle.num_threads(),
        "citations": "plug-in chain: Section 4.4.1 (psi_r estimator, pilot bandwidths, final h); "
                     "LSCV objective and its argmin: Section 4.4.2 (g(h) with K*K - 2K, eq. LSCV-finalH)",
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
    # g(h) at each grid point is a sum of its own: the grid is run in chunks,
    # each added to the file when done, so an interrupted run resumes.
    parts = doc.setdefault("lscv_parts", {})
    for k0 in range(0, grid.size, CHUNK):
        if str(k0) in parts:
            continue
        t = time.time()
        c = oracle.lscv_curve(x, grid[k0:k0 + CHUNK])
        parts[str(k0)] = {"g": [float(v) for v in c.g], "gscale": [float(v) for v in c.gscale],
                          "s1": [float(v) for v in c.s1], "s2": [float(v) for v in c.s2],
                          "seconds": time.time() - t}
        save()
        print(f"lscv grid {k0}..{min(k0 + CHUNK, grid.size) - 1} done in {time.time() - t:.0f} s", flush=True)
    if "lscv" not in doc:
        keys = sorted(parts, key=int)
        cat = {f: [v for key in keys for v in parts[key][f]] for f in ("g", "gscale", "s1", "s2")}
        k, at_edge, margin = oracle.argmin(np.array(cat["g"]))
        doc["lscv"] = {"h": [float(v) for v in grid], **cat, "argmin": int(k), "at_edge": bool(at_edge),
                       "margin": float(margin), "seconds": sum(parts[key]["seconds"] for key in keys)}
        del doc["lscv_parts"]
        save()
        print(f"lscv over {grid.size} h: k*={k}", flush=True)

if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "mixture_100k_oracle.json"))
