"""Build libce.so (HIP, gfx950) in-tree next to this file.

    python -m paper_0712_0813_amd.build
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libce.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # only explicit fma() calls fuse, so every kernel rounds identically
    "-ffp-contract=off",
    # packed FP32 instructions stay disabled in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


# kernel families compiled once per model of the potential (quartic,
# polynomial): the source is built twice with CE_UNIT_MODEL set
MODEL_UNITS = ("ce_kernels.hip", "ce_step2d.hip", "ce_step3d.hip")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def compile_units():
    """(source, extra flags, object name) of every object of the library."""
    out = []
    for src in sources():
        base = os.path.basename(src)
        if base in MODEL_UNITS:
            for m in (0, 1):
                out.append((src, [f"-DCE_UNIT_MODEL={m}"], f"{base}.m{m}.o"))
        else:
            out.append((src, ["-DCE_UNIT_MODEL=0"], f"{base}.o"))
    return out


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "hipcc")
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds, objs = [], []
    for src, extra, name in compile_units():
        obj = os.path.join(objdir, name)
        cmds.append([hipcc, *HIPCC_FLAGS, *extra, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj])
        objs.append(obj)
    # one compiler process per source, at most as many as there are cores
    jobs = max(1, min(len(cmds), os.cpu_count() or 1, 16))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
        for fut in [ex.submit(subprocess.check_call, cmd) for cmd in cmds]:
            fut.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
