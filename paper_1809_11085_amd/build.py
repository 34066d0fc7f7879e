"""Build libscqr.so (HIP, gfx950 only) in-tree with hipcc.

    python -m paper_1809_11085_amd.build          # or build() from Python

Every .hip file under csrc/ is compiled for gfx950 into one shared library next to this file.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libscqr.so")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off in every kernel (scalar / float2 code only)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = [l for l in (res.stdout + res.stderr).splitlines()
             if l.strip() and "packed-fp32-ops" not in l and "ignoring feature" not in l]
    return res.returncode, noise


def build(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 (one hipcc per source, in parallel) and link
    libscqr.so (always recompiles)."""
    from concurrent.futures import ThreadPoolExecutor

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(objdir, os.path.basename(f)[:-4] + ".o") for f in srcs]
    cflags = [f for f in FLAGS if f != "-shared"]
    jobs = [[hipcc, *cflags, *inc, "-c", f, "-o", o] for f, o in zip(srcs, objs)]
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda c: _run(c, verbose), jobs))
    failed = False
    for (rc, noise), f in zip(results, srcs):
        if rc != 0 or (verbose and noise):
            sys.stderr.write("\n".join(noise) + "\n")
        failed |= rc != 0
    if failed:
        raise RuntimeError("hipcc failed building libscqr.so")
    tmp = LIB + ".tmp"
    rc, noise = _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp], verbose)
    if rc != 0:
        sys.stderr.write("\n".join(noise) + "\n")
        raise RuntimeError("hipcc failed linking libscqr.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
