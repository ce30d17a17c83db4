"""Build libwmi.so (HIP kernels + C-ABI runtime) for gfx950, in-tree.

    python -m paper_2204_09131_amd.build

Every HIP translation unit is compiled with packed FP32 instructions disabled
(-packed-fp32-ops); hipcc's host pass warns that it does not know the
feature, which is harmless.
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
LIB = os.path.join(HERE, "libwmi.so")
BUILD_DIR = os.path.join(ROOT, "_build")

SOURCES = ["wmi_kernels.hip", "wmi_runtime.cpp", "psi_table.cpp", "wmi_server.cpp", "wmi_search.cpp"]
ARCH = os.environ.get("WMI_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


# The main kernel is instantiated once per k (1..16) in a unit of its own:
# wmi_kernels.hip compiled again with WMI_MAIN_K = k.
MAIN_KS = range(1, 17)


def _units():
    units = [(src, ()) for src in SOURCES]
    units += [("wmi_kernels.hip", (f"-DWMI_MAIN_K={k}",)) for k in MAIN_KS]
    return units


def _compile(unit) -> str:
    src, defs = unit
    tag = "_".join(d.split("=")[-1] for d in defs)
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + (f".k{tag}" if tag else "") + ".o")
    cmd = [_hipcc(), *COMMON, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    workers = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, _units()))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libwmi.so failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
