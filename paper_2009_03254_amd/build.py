"""Build libbcmc.so in-tree with hipcc for gfx950.

    python -m paper_2009_03254_amd.build        # or build() from Python

Each source is compiled to an object under _build/ (in parallel), then linked
into paper_2009_03254_amd/libbcmc.so.  Always rebuilds.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libbcmc.so")
SOURCES = ["tables.cpp", "zfp.hip", "extract.hip", "batch.hip", "dense.hip", "capi.cpp",
           "batch_api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    "-fvisibility=hidden",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


GEN = os.path.join(BUILD, "gen")


def _generate():
    """Build and run gen_ntri (host only): writes _build/gen/mc_ntri.h, the
    bit-sliced triangle count of the marching-cubes table."""
    os.makedirs(GEN, exist_ok=True)
    exe = os.path.join(GEN, "gen_ntri")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-O2", "-std=c++17", "-x", "hip",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), os.path.join(CSRC, "gen_ntri.cpp"),
           os.path.join(CSRC, "tables.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building gen_ntri failed:\n{r.stdout}{r.stderr}")
    r = subprocess.run([exe, os.path.join(GEN, "mc_ntri.h")], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gen_ntri failed:\n{r.stdout}{r.stderr}")


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-I", os.path.join(ROOT, "include"), "-I", GEN, "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(line for line in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in line)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msgs}")
    if msgs.strip():
        print(msgs, file=sys.stderr)
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    _generate()
    with ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
