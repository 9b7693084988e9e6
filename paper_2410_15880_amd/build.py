"""Build the RFR shared library (librfr.so) for gfx950.

Device code (rfr_device.hip) is compiled by hipcc for --offload-arch=gfx950 with
packed-FP32 instruction selection disabled; the host core (rfr_host.cpp) by g++
without floating-point contraction (its double-double arithmetic relies on
exactly rounded adds and explicit fma); the ABI, batch and serving units are
host C++ compiled by hipcc against the HIP runtime.

Usage: python -m paper_2410_15880_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
OBJ = os.path.join(ROOT, "_build")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "librfr.so")

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + INC, "-I" + CSRC]
HOST_HIP_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-I" + INC, "-I" + CSRC]
GXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-I" + INC, "-I" + CSRC]

UNITS = [
    ("rfr_device.hip", "hip"),
    ("rfr_roots.hip", "hipexact"),
    ("rfr_host.cpp", "gxx"),
    ("rfr_abi.cpp", "hiphost"),
    ("rfr_batch.cpp", "hip"),
    ("rfr_serve.cpp", "hiphost"),
    ("rfr_tune.cpp", "hiphost"),
    ("rfr_sqf.cpp", "hiphost"),
]


def _cmd(src: str, kind: str, obj: str):
    path = os.path.join(CSRC, src)
    if kind == "hip":
        return [HIPCC] + HIP_FLAGS + ["-c", path, "-o", obj]
    if kind == "hipexact":  # double-double arithmetic: no contraction
        return [HIPCC] + HIP_FLAGS + ["-ffp-contract=off", "-c", path, "-o", obj]
    if kind == "hiphost":
        return [HIPCC] + HOST_HIP_FLAGS + ["-c", path, "-o", obj]
    return ["g++"] + GXX_FLAGS + ["-c", path, "-o", obj]


def build(verbose: bool = False) -> str:
    """Compile every unit and link librfr.so; returns the library path."""
    os.makedirs(OBJ, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    procs = []
    objs = []
    for src, kind in UNITS:
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = _cmd(src, kind, obj)
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((src, out.decode(errors="replace")))
        elif verbose and out:
            print(out.decode(errors="replace"))
    if failed:
        msg = "\n".join("--- %s ---\n%s" % f for f in failed)
        raise RuntimeError("librfr build failed:\n" + msg)
    tmp = LIB + ".tmp"
    link = [HIPCC, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread", "-ldl"]
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("librfr link failed:\n" + r.stdout.decode(errors="replace"))
    shutil.move(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
