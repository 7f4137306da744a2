"""Build the HIP library libpbe.so (gfx950) in-tree with hipcc.

Each .hip source is compiled to its own object in parallel (kernels and their
launchers live in the same translation unit, so no relocatable device code is
needed), then the objects are linked into one shared library.
"""
from __future__ import annotations

import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpbe.so")
OBJ_DIR = os.path.join(ROOT, "_build", "obj")
ARCH = os.environ.get("PBE_OFFLOAD_ARCH", "gfx950")

# -packed-fp32-ops: never emit packed FP32 VALU instructions
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def _stale(obj, src, headers):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [src] + headers)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental=True: only objects older than their source or any header)."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    incs = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    headers = glob.glob(os.path.join(HERE, "csrc", "*.h")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    jobs = []
    objs = []
    for src in sources():
        obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
        objs.append(obj)
        if incremental and not _stale(obj, src, headers):
            continue
        jobs.append(["hipcc"] + FLAGS + incs + ["-c", src, "-o", obj])
    workers = max(1, min(max(len(jobs), 1), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda c: _run(c, verbose), jobs))
    tmp = LIB + ".tmp"
    _run(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}"] + objs + ["-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose=True, incremental="--incremental" in sys.argv))
