"""Build step of the HIP library: hipcc for gfx950 into an in-tree shared object."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libugkwp.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "api.hip", "mlp.hip")]

# -ffp-contract=off: every product and sum rounds on its own, in source order.
# The target-feature switch keeps the compiler from forming packed FP32 ops.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(quiet: bool = True) -> str:
    cmd = ["hipcc", *HIPCC_FLAGS, "-o", LIB + ".tmp", *SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout[-4000:] + r.stderr[-4000:])
    if not quiet:
        print(" ".join(cmd))
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(quiet=False))
