"""Build the gfx950 shared library liblbmpcm.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbmpcm.so")
SOURCES = [os.path.join(CSRC, "lbm_kernels.hip"), os.path.join(CSRC, "lbm_api.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # never let the compiler form packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no FMA contraction: every operation rounds on its own, so every launch
    # shape (template instantiation) gives bit-identical populations
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, extra_flags=(), out: str = LIB) -> str:
    """Compile every source to an object in parallel, then link.  extra_flags
    (e.g. -DLBM_NT_LOADS=0) and out build variants of the library."""
    objs, procs = [], []
    objdir = CSRC if out == LIB else os.path.dirname(os.path.abspath(out))
    tag = "" if out == LIB else "." + os.path.basename(out)
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.basename(src) + tag + ".o")
        cmd = [HIPCC] + [f for f in FLAGS if f != "-shared"] + list(extra_flags) + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
