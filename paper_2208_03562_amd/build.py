"""Build the HIP library ``libprc.so`` in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libprc.so")
SOURCES = [os.path.join(CSRC, f) for f in ("prc_lib.hip", "prc_batch.hip", "prc_serve.hip",
                                              "prc_resident.hip")]
# compiled on its own with WIDE_FLAGS added: the two-step sweep on 1024-thread tiles
WIDE = os.path.join(CSRC, "prc_wide.hip")
HEADERS = [os.path.join(CSRC, h) for h in ("prc_coef.hpp", "prc_device.hpp", "prc_collide.hpp",
                                         "prc_sweep.hpp", "prc_host.hpp", "prc_reduce.hpp",
                                         "prc_batch.hpp", "prc_sweep2.hpp", "prc_launch.hpp",
                                         "prc_resident.hpp")] + [
    os.path.join(ROOT, "include", "prc.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # multiply-adds are fused only within one source expression, so a node's
    # arithmetic is fixed by the source alone: the single-problem and the
    # batched sweeps, which inline the same code into different kernels,
    # give the same bits
    "-ffp-contract=on",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
# instruction scheduling for the 1024-thread two-step workgroups: the
# strategy that favours instruction-level parallelism (measured faster for
# them, slower for the other shapes; it reorders, it does not change results)
WIDE_FLAGS = ["-mllvm", "--amdgpu-sched-strategy=max-ilp"]


def build(verbose: bool = False) -> str:
    """Compile ``libprc.so`` (always recompiles; the sources compile in
    parallel, a minute or so)."""
    tmp = LIB + ".tmp"
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, procs = [], []
    try:
        for src in SOURCES + [WIDE]:
            obj = os.path.join(PKG, "_" + os.path.basename(src) + ".o")
            extra = WIDE_FLAGS if src == WIDE else []
            cmd = [HIPCC, *FLAGS, *extra, *inc, "-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((subprocess.Popen(cmd), cmd))
            objs.append(obj)
        for proc, cmd in procs:
            if proc.wait() != 0:
                raise subprocess.CalledProcessError(proc.returncode, cmd)
        cmd = [HIPCC, "--offload-arch=gfx950", "-fPIC", "-shared", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    finally:
        for proc, _ in procs:
            if proc.poll() is None:
                proc.kill()
                proc.wait()
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
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
    for f in sorted(SOURCES + [WIDE] + HEADERS):
        text = open(f, encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    h.update(" ".join(FLAGS + WIDE_FLAGS).encode())
    return h.hexdigest()[:16]
