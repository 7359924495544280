"""Build step: compile the HIP sources for gfx950 into the in-tree shared library."""
from __future__ import annotations

import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkerrhip.so")
SOURCES = ["kerrhip.hip", "mlp.hip", "fixed.hip"]

# -packed-fp32-ops: keep the compiler from forming packed FP32 instructions.
# -ffp-contract=on: fuse multiply-adds per source expression, so every inlined
# copy of the right-hand side rounds identically (bitwise resume and
# launch-shape independence rely on it).
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# Per-source additions.  The integrator kernels keep many per-lane
# loop-invariant values; machine-level LICM hoists constant materialisations
# out of the attempt loop into scalar registers, which then spill into vector
# lanes and are read back with v_readlane inside the loop (measured: 102 scalar
# spills and 245 lane reads with it, 52 and 101 without).
SOURCE_FLAGS = {"kerrhip.hip": ["-mllvm", "-disable-machine-licm"]}


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    inc = ["-I", os.path.join(ROOT, "include")]
    with tempfile.TemporaryDirectory() as d:
        objs = []
        for src in SOURCES:
            obj = os.path.join(d, src + ".o")
            _run([hipcc, *HIPCC_FLAGS, *SOURCE_FLAGS.get(src, []), *inc, "-c", "-o", obj, os.path.join(CSRC, src)],
                 verbose)
            objs.append(obj)
        _run([hipcc, "--offload-arch=gfx950", "-fPIC", "-shared", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
