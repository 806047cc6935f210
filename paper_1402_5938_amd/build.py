"""Build libgllmg.so (HIP, gfx950) in-tree.

Usage: python -m paper_1402_5938_amd.build [-j JOBS]
Every .hip file under csrc/ is compiled by hipcc to an object under _build/, in parallel,
then linked into paper_1402_5938_amd/libgllmg.so.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgllmg.so")
ARCH = os.environ.get("GLLMG_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions are disabled for every HIP translation unit
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # fully unrolled element loops index their register arrays with constants only; the
         # default size limit for a requested full unroll is too small at p = 16
         "-mllvm", "-pragma-unroll-threshold=65536",
         "-Wall", "-Wno-unused-function", "-Wno-unused-result"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def compile_one(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int = 0, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


# The library with AddressSanitizer and UndefinedBehaviorSanitizer on its host side (device
# code unoptimized: the executable makes no GPU call), linked with a driver of host-side checks
# into an executable.
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def build_host_check(driver: str, out_dir: str, jobs: int = 0) -> str:
    """Compile the host side of every csrc/*.hip file and the driver source `driver` with the
    sanitizers into out_dir; returns the executable's path."""
    os.makedirs(out_dir, exist_ok=True)
    flags = ["-x", "hip", f"--offload-arch={ARCH}", "-O1", "-Xarch_device", "-O0", "-g",
             "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + SAN

    def one(src):
        obj = os.path.join(out_dir, os.path.basename(src).rsplit(".", 1)[0] + ".o")
        r = subprocess.run([HIPCC] + flags + ["-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        return obj

    srcs = sources() + [driver]
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(one, srcs))
    exe = os.path.join(out_dir, "host_check")
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}"] + SAN + ["-o", exe] + objs + ["-lpthread"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    return exe


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=0)
    a = ap.parse_args()
    try:
        build(a.j, verbose=True)
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
