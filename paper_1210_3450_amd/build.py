"""Builds libmdgpu.so (the HIP library behind include/md.h) for gfx950, in-tree.

Usage: python -m paper_1210_3450_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SOURCES = [os.path.join(PKG, "csrc", f) for f in ("md_api.hip", "md_kernels.hip", "md_bubbles.hip")]
HEADERS = [os.path.join(PKG, "csrc", "md_internal.h"), os.path.join(ROOT, "include", "md.h")]
LIB = os.path.join(PKG, "libmdgpu.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions (v_pk_*_f32) anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           "-o", LIB + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


SAN_DIR = os.path.join(PKG, "_san")


def build_host_check(out_dir: str = SAN_DIR, verbose: bool = False) -> str:
    """Builds the library with AddressSanitizer and UndefinedBehaviorSanitizer on its
    host code (device code as usual) and csrc/host_check.cpp against it; returns the
    path of the host_check executable.  Run it with ASAN_OPTIONS=detect_leaks=0 (the
    HIP runtime keeps allocations until exit)."""
    os.makedirs(out_dir, exist_ok=True)
    san = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    host_san = [x for f in san for x in ("-Xarch_host", f)]
    lib = os.path.join(out_dir, "libmdgpu_san.so")
    flags = [f for f in FLAGS if f != "-O3"]
    cmd = [HIPCC, *flags, "-O1", "-g", *host_san, "-I", os.path.join(ROOT, "include"), "-I",
           os.path.join(PKG, "csrc"), "-o", lib, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    # the driver has no device code: plain clang++ with the same sanitizer runtime
    exe = os.path.join(out_dir, "host_check")
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    cxx = os.path.join(rocm, "llvm", "bin", "clang++")
    cmd = [cxx, "-std=c++17", "-O1", "-g", *san, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
           "-I", os.path.join(ROOT, "include"), os.path.join(PKG, "csrc", "host_check.cpp"), "-o", exe,
           "-L", out_dir, "-lmdgpu_san", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(rocm, "lib")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return exe


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
