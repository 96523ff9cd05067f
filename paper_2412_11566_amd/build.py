"""Compile the qtthom HIP library for gfx950 (in-tree, no JIT cache).

Usage: ``python -m paper_2412_11566_amd.build`` or ``build()`` from Python.
Produces ``paper_2412_11566_amd/libqtthom.so``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libqtthom.so")
HOSTLIB = os.path.join(HERE, "libqtthom_host.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["kernels.hip", "kernels_fact.hip", "kernels_qr_blk.hip", "kernels_qr_big.hip", "kernels_cholqr.hip", "kernels_mfma.hip", "engine.hip", "host_ops.cpp", "host_capi.cpp"]
ARCH = os.environ.get("QTTHOM_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}"]
# Packed FP32 instructions are disabled for all device code.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [_hipcc(), *COMMON, *DEVICE, "-x", "hip", "-c", path, "-o", obj]
    else:
        # host-only C++: plain g++, so the host library pulls in no HIP runtime
        cmd = ["g++", *COMMON, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    gpu_objs = [o for o in objs if not o.endswith("host_capi.o")]
    host_objs = [o for o in objs if o.endswith(("host_ops.o", "host_capi.o"))]
    for out, parts, linker in ((LIB, gpu_objs, [_hipcc(), f"--offload-arch={ARCH}"]),
                               (HOSTLIB, host_objs, ["g++"])):
        tmp = out + ".tmp"
        cmd = [*linker, "-shared", "-fPIC", *parts, "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, out)
        if verbose:
            print(f"built {out}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
