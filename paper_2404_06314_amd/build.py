"""Build libqtm.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libqtm.so"
SOURCES = ["api.hip", "plain.hip", "fused.hip", "multi.hip", "circuit.cpp", "schedule.cpp"]

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 (v_pk_*_f32) instructions in any kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep SimplifyCFG from merging the per-register-bit switch cases into
    # pointer phis, which would force the 16-amplitude register arrays into
    # scratch memory
    "-mllvm", "-simplifycfg-sink-common=false",
    "-I" + str(ROOT / "include"),
]


def build(verbose: bool = False) -> Path:
    objdir = PKG / "_build"
    objdir.mkdir(exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = objdir / (src + ".o")
        cmd = ["hipcc", *HIP_FLAGS, "-c", str(CSRC / src), "-o", str(obj)]
        if src.endswith(".cpp"):
            cmd = ["hipcc", "-O2", "-std=c++17", "-fPIC", "-I" + str(ROOT / "include"),
                   "-c", str(CSRC / src), "-o", str(obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    bad = [p.wait() for p in procs]
    if any(bad):
        raise RuntimeError("hipcc failed")
    tmp = LIB.with_suffix(".so.tmp")
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
