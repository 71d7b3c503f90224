"""Compile the FP64 oracle (plain C, gcc, OpenMP) into oracle/liba2c_oracle.so.

The oracle is test infrastructure; building it is not using it.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["a2c_oracle.c", "a2c_oracle_fullatom.c", "a2c_oracle_lrmsd.c"]
LIB = os.path.join(HERE, "liba2c_oracle.so")
# AddressSanitizer + UndefinedBehaviorSanitizer build (gcc's runtimes; the
# process must preload libasan), for checking the oracle itself
LIB_SAN = os.path.join(HERE, "liba2c_oracle_san.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    out = LIB_SAN if sanitize else LIB
    tmp = out + ".tmp"
    opt = SAN_FLAGS if sanitize else ["-O2"]
    cmd = ["gcc", "-std=c11", *opt, "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-Wno-unused-parameter", *srcs, "-lm", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv)
