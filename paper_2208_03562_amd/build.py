"""Build the HIP library ``libprc.so`` in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libprc.so")
SOURCES = [os.path.join(CSRC, f) for f in ("prc_lib.hip", "prc_batch.hip", "prc_serve.hip")]
HEADERS = [os.path.join(CSRC, h) for h in ("prc_coef.hpp", "prc_device.hpp", "prc_collide.hpp",
                                         "prc_sweep.hpp", "prc_host.hpp", "prc_reduce.hpp",
                                         "prc_batch.hpp", "prc_sweep2.hpp")] + [
    os.path.join(ROOT, "include", "prc.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # multiply-adds are fused only within one source expression, so a node's
    # arithmetic is fixed by the source alone: the single-problem and the
    # batched sweeps, which inline the same code into different kernels,
    # give the same bits
    "-ffp-contract=on",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    """Compile ``libprc.so`` (always recompiles; a few tens of seconds)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))


def source_hash() -> str:
    """Hash of the library's code (identifies the kernels a profile was taken
    on): the sources and headers with comments and blank space removed, so
    that editing a comment does not orphan the committed counter data."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in sorted(SOURCES + HEADERS):
        text = open(f, encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]
