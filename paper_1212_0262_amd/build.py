"""Build libmd.so (the HIP kernels and the C ABI of include/md.h) for gfx950.

Run ``python -m paper_1212_0262_amd.build`` (or call :func:`build`).  Objects go
to ``paper_1212_0262_amd/_build/``; the library lands next to this file, in-tree,
so that it travels with the source tree.  The compiler's resource-usage remarks
(registers, LDS, scratch, occupancy of every kernel) go to
``_build/kernel_resources.json``; a kernel with a private segment (scratch) fails
the build.  Measured on the HMF step, whose one-block reduction kernel once
spilled 28 bytes per lane: 34.1 -> 30.7 us per step at N = 1e5 (FP64) and 104 -> 99 us at
N = 1e7 (FP32 state) without the spill, about 1.2 us per dispatch.
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmd.so")
SOURCES = ["api.hip", "pair.hip", "hmf.hip", "energy.hip", "batch.hip", "adjoint.hip"]
ARCH = "gfx950"
RESOURCES = os.path.join(BUILD_DIR, "kernel_resources.json")

# Packed FP32 instructions are disabled for all device code.
FLAGS = [
    "-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-command-line-argument",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
    "-Rpass-analysis=kernel-resource-usage",
]

_REMARK = re.compile(r"remark:\s+(.*?) \[-Rpass-analysis=kernel-resource-usage\]")
_FIELDS = {"TotalSGPRs": "sgprs", "VGPRs": "vgprs", "AGPRs": "agprs", "ScratchSize [bytes/lane]": "scratch",
           "Dynamic Stack": "dynamic_stack", "Occupancy [waves/SIMD]": "occupancy", "SGPRs Spill": "sgpr_spill",
           "VGPRs Spill": "vgpr_spill", "LDS Size [bytes/block]": "lds"}


def _hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the ROCm toolchain is required to build libmd")
    return exe


def _resources(src: str, remarks: str) -> list:
    """Per-kernel figures from the compiler's resource-usage remarks of one source."""
    out, cur = [], None
    for m in _REMARK.finditer(remarks):
        text = m.group(1).strip()
        if text.startswith("Function Name:"):
            cur = {"source": src, "symbol": text.split(":", 1)[1].strip()}
            out.append(cur)
        elif cur is not None and ":" in text:
            key, val = (x.strip() for x in text.rsplit(":", 1))
            if key in _FIELDS:
                cur[_FIELDS[key]] = val == "True" if val in ("True", "False") else int(val)
    return out


def _demangle(names: list) -> list:
    exe = shutil.which("llvm-cxxfilt") or shutil.which("c++filt")
    if exe is None:
        return names
    r = subprocess.run([exe], input="\n".join(names), capture_output=True, text=True)
    out = r.stdout.splitlines()
    return out if r.returncode == 0 and len(out) == len(names) else names


def _compile(src: str):
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, _resources(src, r.stderr)


def build(verbose: bool = False) -> str:
    """Compile every source and link libmd.so; returns the library path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        done = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in done]
    kernels = [k for _, ks in done for k in ks]
    for k, name in zip(kernels, _demangle([k["symbol"] for k in kernels])):
        k["kernel"] = name
    with open(RESOURCES, "w") as fh:
        json.dump(kernels, fh, indent=1)
    bad = [k for k in kernels if k.get("scratch", 0) or k.get("dynamic_stack", False)]
    if bad:
        raise RuntimeError("kernels with a private segment (scratch): "
                           + "; ".join(f"{k['kernel']} ({k.get('scratch')} bytes/lane)" for k in bad))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
