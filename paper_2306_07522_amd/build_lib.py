"""Build the HIP library libheom.so in-tree for gfx950 (hipcc)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libheom.so")

SOURCES = ["abi.cpp", "host_hierarchy.cpp", "device_tables.cpp", "apply.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-command-line-argument",
]


def extra_sources():
    return [s for s in sorted(os.listdir(CSRC)) if s.endswith((".hip", ".cpp")) and s not in SOURCES]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES + extra_sources()]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    tmp = OUT + ".tmp"
    cmd = ["/opt/rocm/bin/hipcc", *HIPCC_FLAGS, *inc, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libheom.so")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
