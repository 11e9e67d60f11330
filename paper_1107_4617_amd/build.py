"""Builds libbsk.so (HIP kernels for gfx950 + the C ABI) in place with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbsk.so")
# the largest sources first, so the parallel build finishes sooner
SOURCES = ["bsk_radius_1_8.hip", "bsk_radius_9_16.hip", "bsk_radius_17_24.hip", "bsk_radius_25_32.hip",
           "bsk_radius_33_40.hip", "bsk_radius_41_48.hip", "bsk_radius_49_56.hip", "bsk_radius_57_64.hip",
           "bsk_kernels.hip", "bsk_poly.hip", "bsk_patch_radius.hip", "bsk_radius.hip", "bsk_batched.hip", "bsk_noalloc.hip", "bsk_plan.cpp",
           "bsk_api.cpp", "bsk_batched.cpp"]

# Packed FP32 instructions are turned off in the device code; hipcc's host
# pass warns that it does not know this feature, which is harmless.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument"]


def _compile(src: str, verbose: bool) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(HERE, "_build", src + ".o")
    cmd = ["hipcc", *HIPFLAGS, "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compiles every source (in parallel, at most `jobs` at once; 0 = one per source
    up to the CPU count) and links libbsk.so."""
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    n = jobs or max(1, min(len(SOURCES), os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=n) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libbsk.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
