"""Build the HIP library ``liblbm_solid.so`` for gfx950 in-tree.

Every HIP source is compiled with packed FP32 instructions disabled; the
library is plain C ABI (include/lbm_solid.h) with no torch dependency.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", f) for f in ("lbm_solid.hip", "lbm_batch.hip")]
LIB = os.path.join(HERE, "liblbm_solid.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


INST = os.path.join(HERE, "csrc", "instantiate.hip")
PRECISIONS = ["PrecF64", "PrecF32", "PrecF32U64", "PrecF16", "PrecBF16"]


def build(verbose: bool = False) -> str:
    """Compile the runtime sources and one object per precision (in
    parallel), then link the library."""
    jobs = [(src, [], os.path.join(HERE, "csrc", os.path.basename(src) + ".o")) for src in SRCS]
    jobs += [(INST, [f"-DLBM_PREC={pr}"], os.path.join(HERE, "csrc", f"inst_{pr}.o")) for pr in PRECISIONS]
    objs = [o for _, _, o in jobs]
    procs = []
    for src, defs, obj in jobs:
        cmd = ["hipcc", *HIPCC_FLAGS, *defs, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    rcs = [p.wait() for p in procs]
    if any(rcs):
        raise subprocess.CalledProcessError(max(rcs), "hipcc -c")
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
