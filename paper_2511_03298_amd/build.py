"""Compile the HIP library (gfx950) in-tree: paper_2511_03298_amd/libivfpq.so."""

from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "libivfpq.so")
BUILD_DIR = os.path.join(PKG, "_build")

SOURCES = ["abi.cpp", "tables.hip", "coarse.hip", "coarse_mfma.hip", "scan.hip", "rerank.hip",
           "batched.hip", "build_index.hip"]

# Canonical FP32 stages must not be contracted into FMAs; packed FP32 VALU
# instructions are disabled for the device code.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build (argument
# validation, layout and workspace planning run on the CPU): the sanitizers
# instrument host code only, the device code is compiled as usual. The
# shared sanitizer runtime has to be preloaded into the process that loads
# the library (see asan_runtime()).
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all",
                  "-shared-libsan"]
ASAN_OUT = os.path.join(BUILD_DIR, "asan", "libivfpq_asan.so")


def asan_runtime() -> str:
    """Path of the shared ASan runtime of hipcc's clang."""
    r = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("the clang ASan runtime was not found")
    return path


def build(verbose: bool = False, jobs: int = 8, sanitize: bool = False) -> str:
    bdir = os.path.join(BUILD_DIR, "asan") if sanitize else BUILD_DIR
    out = ASAN_OUT if sanitize else OUT
    extra = SANITIZE_FLAGS if sanitize else []
    # The sanitized library records where its runtime lives, so programs
    # linked against it find it.
    link_extra = [f"-Wl,-rpath,{os.path.dirname(asan_runtime())}"] if sanitize else []
    os.makedirs(bdir, exist_ok=True)
    cc = hipcc()

    def compile_one(src):
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        cmd = [cc, *FLAGS, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = out + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *extra, *link_extra, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
