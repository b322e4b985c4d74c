"""Build the HIP library ``liblbwake.so`` for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "lbwake.hip")
SRCS = [SRC, os.path.join(HERE, "csrc", "lbw_batch.hip")]
DEPS = [*SRCS, os.path.join(HERE, "csrc", "lbw_kernels.hpp"), os.path.join(HERE, "csrc", "lbw_device.hpp"),
        os.path.join(HERE, "csrc", "lbw_adjoint.hpp"), os.path.join(HERE, "csrc", "lbwake.map"),
        os.path.join(ROOT, "include", "lbwake.h")]
SO = os.path.join(HERE, "liblbwake.so")
ARCH = os.environ.get("LBW_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # multiply-adds are fused per source expression only, so that the same
    # expression rounds the same way in every kernel that inlines it
    "-ffp-contract=on",
    # packed FP32 instructions stay off (they have given wrong results on this hardware)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-lambda-capture",
    # only the C ABI of include/lbwake.h is exported (kernel handles included
    # in the hidden part by the version script)
    "-fvisibility=hidden",
    "-Wl,--version-script=" + os.path.join(HERE, "csrc", "lbwake.map"),
]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile the HIP sources under ``csrc/`` into ``liblbwake.so``; always recompiles when force."""
    if not force and os.path.exists(SO) and all(os.path.getmtime(SO) >= os.path.getmtime(d) for d in DEPS):
        return SO
    tmp = SO + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, *SRCS, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    build(verbose=True)
    print(SO)
    sys.exit(0)
