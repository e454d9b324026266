"""Build libpt.so (the HIP kernels and the C-ABI runtime) for gfx950, in-tree.

    python -m paper_1107_3490_amd.build

Flags: -ffp-contract=off keeps every rounding written in the source (the FP64
path must reproduce a fixed operation order); packed FP32 instructions are
disabled for the device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpt.so")
SOURCES = [os.path.join(CSRC, f) for f in
           ("pt_k_run1m.hip", "pt_k_run2m.hip", "pt_k_run4m.hip", "pt_k_run1d.hip", "pt_k_run2d.hip",
            "pt_k_run4d.hip", "pt_k_pack.hip", "pt_k_flow.hip", "pt_k_sweep.hip", "pt_k_misc.hip", "pt_k_run.hip",
            "pt_runtime.cpp")]
ARCH = "gfx950"


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
            "-fno-fast-math", "-fvisibility=hidden", "-Wall",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC]


def _compile(src, extra, verbose):
    obj = os.path.join(CSRC, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [hipcc(), *flags(), *extra, *lang, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    if verbose and out.strip():
        print(out)
    return obj


def build(verbose: bool = False, extra=()) -> str:
    """Compiles the translation units in parallel (one hipcc each) and links
    them into libpt.so."""
    from concurrent.futures import ThreadPoolExecutor

    tmp = LIB + ".tmp"
    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, extra, verbose), SOURCES))
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
