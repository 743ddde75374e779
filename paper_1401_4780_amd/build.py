"""Build the HIP library libasyrk.so for gfx950, in tree.

    python -m paper_1401_4780_amd.build

Host setup code (validation, row weights, alias table, packing) is compiled
by g++ with -ffp-contract=off; kernels and the C ABI by hipcc for gfx950.
"""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
OUT = PKG / "_build"
LIB = PKG / "_build" / "libasyrk.so"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
    # packed FP32 instructions are disabled for every kernel in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(str(c) for c in cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[0]} {cmd[-1]}")
    noise = [ln for ln in (r.stderr or "").splitlines()
             if ln.strip() and "packed-fp32-ops" not in ln and "warning generated" not in ln]
    if verbose and noise:
        sys.stderr.write("\n".join(noise) + "\n")


def build(verbose: bool = False) -> Path:
    """Compile every source and link libasyrk.so (always rebuilds)."""
    OUT.mkdir(exist_ok=True)
    objs = []
    o = OUT / "setup.o"
    _run(["g++", *HOST_FLAGS, "-c", str(CSRC / "setup.cpp"), "-o", str(o)], verbose)
    objs.append(o)
    for src in ("kernels.hip", "setup_dev.hip", "api.hip", "server.hip"):
        o = OUT / (src.replace(".hip", ".o"))
        _run([HIPCC, *HIP_FLAGS, "-c", str(CSRC / src), "-o", str(o)], verbose)
        objs.append(o)
    tmp = OUT / f"libasyrk.so.tmp{os.getpid()}"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *map(str, objs), "-o", str(tmp)], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
