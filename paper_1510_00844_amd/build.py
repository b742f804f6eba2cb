"""Build the HIP library libspgemm.so for gfx950 with hipcc (in-tree)."""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libspgemm.so")
ARCH = os.environ.get("SPG_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return [
        "--offload-arch=" + ARCH,
        "-O3", "-std=c++17", "-fPIC", "-shared",
        "-fno-strict-aliasing",
        "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
        # no packed FP32 instructions anywhere in the device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I" + os.path.join(os.path.dirname(HERE), "include"),
    ]


def build(verbose: bool = False) -> str:
    src = os.path.join(CSRC, "spgemm.hip")
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + flags() + ["-o", tmp, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for %s" % src)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
