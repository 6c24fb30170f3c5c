"""Build librobostep.so (HIP, gfx950) in-tree with hipcc.

Each translation unit is compiled to an object in parallel, then the objects
are linked into the shared library.

    python -m paper_2505_06771_amd.build                  # librobostep.so
    python -m paper_2505_06771_amd.build --phase-timers   # librobostep_timers.so

The second form defines RS_PHASE_TIMERS: a diagnostic library whose fused
rollout records per-wavefront phase cycles (rs_phase_cycles); the product
library never carries that code.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "librobostep.so")
LIB_TIMERS = os.path.join(PKG, "librobostep_timers.so")
OBJ_DIR = os.path.join(PKG, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]
# Per-file additions. The fused rollout runs two wavefronts per SIMD and is
# bound by instruction latency: the backend's max-ILP scheduling strategy
# interleaves its independent dependency chains better there (it shortened
# launches by about 1% in same-box comparisons; on env_run it does not help).
FILE_FLAGS = {
    "rs_rollout.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
}
# the host pass does not know the packed-fp32 feature; that warning is noise
_NOISE = ("packed-fp32-ops",)


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if not any(n in l for n in _NOISE))
    return res.returncode, err


def build(verbose: bool = False, phase_timers: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    obj_dir = OBJ_DIR + ("_timers" if phase_timers else "")
    lib = LIB_TIMERS if phase_timers else LIB
    os.makedirs(obj_dir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    defs = ["-DRS_PHASE_TIMERS"] if phase_timers else []
    jobs = []
    for src in sources():
        obj = os.path.join(obj_dir, os.path.basename(src)[:-4] + ".o")
        extra = FILE_FLAGS.get(os.path.basename(src), [])
        jobs.append((obj, [hipcc, *HIPCC_FLAGS, *extra, *defs, *inc, "-c", src, "-o", obj]))
    if verbose:
        for _, cmd in jobs:
            print(" ".join(cmd), flush=True)
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda j: _run(j[1]), jobs))
    for (obj, _), (rc, err) in zip(jobs, results):
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {os.path.basename(obj)} ({rc}):\n{err}")
        if verbose and err.strip():
            print(err, file=sys.stderr)
    tmp = lib + ".tmp"
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for o, _ in jobs], "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    rc, err = _run(link)
    if rc != 0:
        raise RuntimeError(f"hipcc link failed ({rc}):\n{err}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, phase_timers="--phase-timers" in sys.argv[1:]))
