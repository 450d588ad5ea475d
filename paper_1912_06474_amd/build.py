"""Build libsdd.so (HIP, gfx950) in-tree: python -m paper_1912_06474_amd.build"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsdd.so")
SOURCES = ["api.cpp", "bvh_build.cpp", "kernels.hip", "bvh_device.hip", "bvh_wide.hip", "nrc.hip"]

# gfx950 only; packed FP32 instructions disabled for all device code
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-fno-hip-fp32-correctly-rounded-divide-sqrt",
            # matrix-core results in ordinary VGPRs (no copies out of accumulation registers)
            "-mllvm", "-amdgpu-mfma-vgpr-form=1",
            "-Wall", "-Wno-unused-result"]


# The FP32-path-state measurement build: the same sources with the per-path
# ray state and shading geometry in FP32 (it states what FP64 state buys in
# accuracy and costs in time); loaded only when SDD_PATH_STATE=f32.
VARIANTS = {"": [], "_f32state": ["-DSDD_PATH_STATE_F32"]}


def build(verbose: bool = False, jobs: int = 3) -> str:
    """Build libsdd.so and the measurement build; returns the library's path."""
    for suffix, defs in VARIANTS.items():
        _build_one(suffix, defs, verbose)
    return LIB


def _build_one(suffix: str, defs: list, verbose: bool) -> str:
    objdir = os.path.join(HERE, "_build" + suffix)
    lib = os.path.join(HERE, "libsdd" + suffix + ".so")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = ["hipcc", *HIPFLAGS, *defs, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = False
    for cmd, p in procs:
        out, _ = p.communicate()
        out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
        if out.strip():
            print(out, file=sys.stderr)
        if p.returncode != 0:
            failed = True
    if failed:
        raise RuntimeError("HIP compilation failed")
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", lib + ".tmp"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
