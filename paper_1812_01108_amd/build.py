"""Build the HIP library libangles2coords.so for gfx950 with hipcc (in-tree).

Each source compiles to its own object in parallel (there are no device
calls across files), then one hipcc line links the shared library."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libangles2coords.so")
# host code under AddressSanitizer + UndefinedBehaviorSanitizer (clang's
# runtimes; the process must preload libclang_rt.asan), for checking the
# host-side validation and plan building on a machine without a GPU; the
# device code is compiled as usual
LIB_SAN = os.path.join(HERE, "libangles2coords_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
INCLUDE = os.path.join(HERE, "..", "include")
SOURCES = ["api.hip", "backbone.hip", "fullatom.hip", "autotune.hip", "lrmsd.hip",
           "inverse.hip"]
ARCH = ["--offload-arch=gfx950"]
FLAGS = [
    *ARCH, "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _jobs() -> int:
    n = os.environ.get("MAX_JOBS")
    return max(1, min(len(SOURCES), int(n) if n and n.isdigit() else (os.cpu_count() or 1)))


def build(verbose: bool = False, extra=(), sanitize: bool = False) -> str:
    if sanitize:
        extra = (*extra, *SAN_FLAGS)
    out = LIB_SAN if sanitize else LIB
    tmpdir = tempfile.mkdtemp(prefix="a2c_build_")
    try:
        def compile_one(src):
            obj = os.path.join(tmpdir, os.path.splitext(src)[0] + ".o")
            cmd = ["hipcc", *FLAGS, *extra, "-I", INCLUDE, "-c", os.path.join(CSRC, src),
                   "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)
            return obj

        with ThreadPoolExecutor(_jobs()) as pool:
            objs = list(pool.map(compile_one, SOURCES))
        tmp = out + ".tmp"
        cmd = ["hipcc", *ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv)
