"""Compile the HIP library libgmg.so in-tree for gfx950 with hipcc.

    python paper_1812_08606_amd/build.py

(run as a script: importing the package loads the library, which may be
missing or built from older sources).
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgmg.so")
SOURCES = [os.path.join(HERE, "csrc", "gmg.hip")]
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-pthread",
]


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def command(out):
    return [hipcc(), *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", out, *SOURCES]


def build(verbose=False):
    """Always recompiles; returns the path of the library."""
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError(f"hipcc failed with status {proc.returncode}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
