"""Build libgodunov.so for gfx950 with hipcc, in-tree.

Every HIP source is compiled with packed FP32 instructions disabled; the host
code needs only the HIP runtime.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgodunov.so")
SOURCES = ["godunov_kernels.hip", "godunov_adjoint.hip", "godunov_mhd.hip", "godunov_amr.hip",
           "godunov_ppm.hip", "godunov_noalloc.hip", "godunov_api.cpp"]
ARCH = os.environ.get("GODUNOV_ARCH", "gfx950")


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        "-Wall", "-Wno-unused-function",
    ]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer (each flag applies
# to the host compilation only; the device code is built as always). The
# runtime is clang's, loaded with LD_PRELOAD by the process that uses the
# library.
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer"]


def build(verbose: bool = False, jobs: int = 4, sanitize: bool = False, out: str = None) -> str:
    """Compile every source for gfx950 and link libgodunov.so (or `out`).
    sanitize=True instruments the host code (argument checks, tables,
    dispatch) with ASan and UBSan, in a build folder of its own."""
    build_dir = BUILD + ("_san" if sanitize else "")
    lib = out or LIB
    os.makedirs(build_dir, exist_ok=True)
    extra = SANITIZE_HOST if sanitize else []

    def compile_one(src):
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = [hipcc()] + lang + flags() + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = lib + ".tmp"
    link_extra = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-shared-libsan"] if sanitize else []
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + link_extra + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
