"""Build the gfx950 shared library libkde_bw.so in-tree with hipcc.

Each HIP source is compiled to its own object (in parallel, under _build/)
and the objects are linked into one shared library."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libkde_bw.so")
OBJ_DIR = os.path.join(ROOT, "_build")
SOURCES = ["kde_kernels.hip", "kde_runtime.hip", "kde_server.hip", "kde_tune.hip", "kde_sort.hip", "kde_query.hip",
           "kde_md.hip", "kde_lscv_H.hip", "kde_query_md.hip", "kde_job.hip", "kde_probe.hip",
           "kde_noalloc.hip"]

# Packed FP32 VALU instructions are disabled for all device code; the kernels
# are written for scalar FP32/FP64 issue.
HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core results straight into VGPRs (no AGPR round trip before exp2)
    "-mllvm", "-amdgpu-mfma-vgpr-form=true",
    "-Wno-unused-result",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libkde_bw.so; always recompiles."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = [os.path.join(OBJ_DIR, s.replace(".hip", ".o")) for s in SOURCES]
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)), 16))
    with ThreadPoolExecutor(jobs) as pool:
        futs = [pool.submit(_run, [hipcc(), *HIPCC_FLAGS, *inc, "-c", "-o", o, os.path.join(CSRC, s)], verbose)
                for s, o in zip(SOURCES, objs)]
        for f in futs:
            f.result()
    tmp = LIB + ".tmp"
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
