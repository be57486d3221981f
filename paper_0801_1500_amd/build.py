"""Build libtr.so (the HIP library behind include/tr.h) for gfx950.

Each translation unit is compiled with its own floating-point contract
setting: the grid build, the plain FP64 kernel and the host ABI code must
round exactly as written (-ffp-contract=off); the FP32 wavefront kernel
fuses the multiply-adds within each expression (-ffp-contract=on, which
honours the source's contraction pragmas: its FP64 helpers round exactly
as written; =fast would fuse at code generation regardless).  Packed FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = {
    "grid_build.hip": ["-ffp-contract=off"],
    "render_plain.hip": ["-ffp-contract=off"],
    "render_wave.hip": ["-ffp-contract=on"],
    "frame_out.hip": ["-ffp-contract=off"],
    "measure.hip": ["-ffp-contract=off"],
    "tr_api.cpp": ["-ffp-contract=off", "-x", "hip"],
}

COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
          "-Wno-unused-result", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str, flags: list, out_dir: str) -> str:
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), msgs))
    if msgs.strip():
        sys.stderr.write(msgs + "\n")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link libtr.so in the package directory."""
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        futs = [ex.submit(_compile, s, f, out_dir) for s, f in SOURCES.items()]
        objs = [f.result() for f in futs]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), res.stdout + res.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
