"""Build the HIP library libnshe.so in-tree for gfx950.

Usage: python -m paper_2602_24271_amd.build

Each source compiles to its own object (in parallel), then one link; the
kernels are launched from the file that defines them, so no relocatable
device code is needed.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/ntt.hip", "csrc/rns.hip", "csrc/api.hip", "csrc/probe.hip"]
LIB = os.path.join(HERE, "libnshe.so")

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # packed-FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _run(cmd) -> None:
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))


def build(verbose: bool = False) -> str:
    # objects in a fixed directory (paths end up in the library, so a fixed
    # one keeps the build reproducible: the same sources give the same bytes)
    tmp = os.path.join(HERE, "_build")
    os.makedirs(tmp, exist_ok=True)
    objs = [os.path.join(tmp, os.path.basename(s) + ".o") for s in SOURCES]
    cmds = [[hipcc(), *FLAGS, "-c", "-o", o, os.path.join(HERE, s)]
            for s, o in zip(SOURCES, objs)]
    with ThreadPoolExecutor(len(cmds)) as ex:
        for f in [ex.submit(_run, c) for c in cmds]:
            f.result()
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-o", LIB + ".tmp", *objs])
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        sys.stderr.write(f"built {LIB}\n")
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
