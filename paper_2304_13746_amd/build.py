"""Build libmhd.so (HIP for gfx950) in-tree with hipcc.

Every translation unit is compiled with -ffp-contract=off (no fused multiply-add,
so the FP64 arithmetic rounds exactly as written) and without packed FP32 ops.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmhd.so")
# a plain host program that drives the library through the C ABI only
EXAMPLE = os.path.join(HERE, "mhd_abi_example")
# the stage kernels in one unit per precision and Riemann solver, compiled in parallel
STAGE = [f"mhd_stage_{p}_{s}.hip" for p in ("f64", "f32") for s in ("hlld", "hll", "hllc")]
SOURCES = ["mhd_api.hip", *STAGE, "mhd_vpot.hip", "mhd_uct.hip"]
ARCH = os.environ.get("MHD_OFFLOAD_ARCH", "gfx950")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.environ.get("HIPCC", os.path.join(ROCM, "bin", "hipcc"))
# roctx markers (host side) around the library's calls, for rocprofv3 --marker-trace
LINK = ["-L" + os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx",
        "-Wl,-rpath," + os.path.join(ROCM, "lib")]
FLAGS = ["-O3", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
         "-Wno-unused-variable", "-Wno-unused-function"]
# FP64 (and the host-side API) round exactly as written, like the CPU reference;
# the FP32 kernels, checked against a tolerance, may fuse multiply-adds.
CONTRACT = {s: "-ffp-contract=fast" for s in STAGE if "_f32_" in s}


def _compile(src: str, defines=(), tag: str = "") -> str:
    obj = os.path.join(BUILD, src.replace(".hip", f"{tag}.o"))
    cmd = [HIPCC, "-c", *FLAGS, CONTRACT.get(src, "-ffp-contract=off"), *defines,
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile and link libmhd.so; ``defines`` (-D...) build a tuning variant
    into ``out``."""
    os.makedirs(BUILD, exist_ok=True)
    tag = "" if out == LIB else "_" + os.path.basename(out).replace(".so", "")
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, defines, tag), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs, *LINK]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    if out == LIB:
        cmd = [HIPCC, "-O2", "-std=c++17", os.path.join(CSRC, "mhd_abi_example.cpp"), "-o",
               EXAMPLE + ".tmp", "-L" + HERE, "-lmhd", "-Wl,-rpath,$ORIGIN"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"building the C ABI example failed:\n{r.stderr}")
        os.replace(EXAMPLE + ".tmp", EXAMPLE)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
