"""The CPU test suite (-m "not gpu") under AddressSanitizer and
UndefinedBehaviorSanitizer, in two runs (the two builds use different
sanitizer runtimes, one per process):

1. the FP64 oracle built by gcc with -fsanitize=address,undefined
   (oracle/liba2c_oracle_san.so, selected by A2C_ORACLE_LIB), gcc's libasan
   preloaded;
2. the HIP library with its host code built by clang with the same
   sanitizers (libangles2coords_san.so, selected by A2C_LIB; the device code
   is compiled as usual and never runs here), clang's asan runtime preloaded.

Leak detection is off (the interpreter's own allocations would report);
any sanitizer report fails the run.  Not collected by pytest (no test_
prefix); run it with `python tests/sanitized_cpu_suite.py`.  Exit status:
that of the first failing run."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _runtime(cmd):
    return subprocess.run(cmd, check=True, capture_output=True, text=True).stdout.strip()


def _clang_asan():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise SystemExit("clang's asan runtime (libclang_rt.asan-x86_64.so) not found")
    return found[-1]


def _run(label, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    # --capture=sys: native sanitizer reports go to the real stderr
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-m", "not gpu", "-q",
           "-p", "no:cacheprovider", "--capture=sys"]
    print(f"[{label}] {' '.join(f'{k}={v}' for k, v in env_extra.items())} {' '.join(cmd)}",
          flush=True)
    rc = subprocess.run(cmd, env=env, cwd=ROOT).returncode
    print(f"[{label}] exit {rc}", flush=True)
    return rc


def main():
    from oracle.build import build as build_oracle
    from paper_1812_01108_amd.build import build as build_lib

    oracle_san = build_oracle(sanitize=True)
    lib_san = build_lib(sanitize=True)
    runs = [
        ("oracle asan+ubsan", {"A2C_ORACLE_LIB": oracle_san,
                               "LD_PRELOAD": _runtime(["gcc", "-print-file-name=libasan.so"])}),
        ("host library asan+ubsan", {"A2C_LIB": lib_san, "LD_PRELOAD": _clang_asan()}),
    ]
    for label, env in runs:
        rc = _run(label, env)
        if rc != 0:
            return rc
    return 0


if __name__ == "__main__":
    sys.exit(main())
