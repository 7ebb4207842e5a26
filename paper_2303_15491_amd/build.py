"""Builds libplmss.so (hipcc, gfx950) next to this file."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libplmss.so")
SRC = os.path.join(HERE, "csrc", "plmss.hip")
ARCH = "gfx950"


def sources():
    return [SRC] + sorted(glob.glob(os.path.join(HERE, "csrc", "*.h"))) + [os.path.join(ROOT, "include", "plmss.h")]


def command(out: str):
    return ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result",
            "-I", os.path.join(ROOT, "include"), "-o", out, SRC]


def build(force: bool = True) -> str:
    """Compile the library (always when force, else only if a source is newer)."""
    if not force and os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(s) <= t for s in sources()):
            return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(command(tmp))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
