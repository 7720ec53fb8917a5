"""Build libhperm.so (HIP kernels for gfx950 + host C++) in-tree with hipcc.

    python paper_1112_6072_amd/build.py   (runs without importing the package)
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libhperm.so")
SOURCES = ["kernels.hip", "split.hip", "dexpand.hip", "noalloc.hip", "expand.cpp", "api.cpp", "serve.cpp",
           "dexpand_host.cpp", "tune.cpp", "sched.cpp", "poly.cpp"]
HIP_HOST_SOURCES = {"api.cpp", "serve.cpp", "dexpand_host.cpp", "tune.cpp"}   # host code that calls the HIP runtime
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# gfx950 only; packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-I" + os.path.join(HERE, "..", "include")]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    lines = [l for l in r.stdout.splitlines()
             if "packed-fp32-ops" not in l and "not a recognized feature" not in l]
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + "\n".join(lines))
    return lines


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link libhperm.so; always rebuilds."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = []
    for src in SOURCES:
        parts = [0, 1, 2, 3] if src == "kernels.hip" else [None]
        for part in parts:
            stem = os.path.splitext(src)[0] + ("" if part is None else f"_p{part}")
            obj = os.path.join(OUT_DIR, stem + ".o")
            if src.endswith(".cpp") and src not in HIP_HOST_SOURCES:
                # plain host C++ (no HIP runtime calls): native popcount for the expansion
                cmd = [HIPCC, *COMMON, "-mpopcnt", "-x", "c++"]
            else:
                cmd = [HIPCC, *COMMON, *DEVICE_FLAGS, "-x", "hip"]
            if part is not None:
                cmd.append(f"-DHP_PART={part}")
            cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
            jobs.append((cmd, obj))
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        outs = list(ex.map(lambda j: _run(j[0]), jobs))
    if verbose:
        for out in outs:
            print("\n".join(out))
    objs = [o for _, o in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
