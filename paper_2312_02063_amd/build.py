"""Build the gfx950 shared library ``libgpfc.so`` in-tree with hipcc.

Usage: ``python -m paper_2312_02063_amd.build`` (or ``build()`` from Python).
Always recompiles.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgpfc.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("gpfc_api.hip", "gpfc_kernels.hip", "gpfc_cnn.hip", "gpfc_reduce.hip", "gpfc_roof.hip", "gpfc_pnet.hip", "gpfc_detrend.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",          # every FP op rounds where written; fma only where spelled out
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libgpfc.so")
    if verbose:
        noise = "is not a recognized feature for this target"
        out = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if noise not in l)
        if out.strip():
            sys.stderr.write(out + "\n")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
