"""Build the FP64 oracle (oracle.c) into oracle/liboracle.so with gcc.

Test infrastructure: the library is loaded only by the tests, the smoke check
and the benchmark's CPU-baseline leg.

    python -m oracle.build               # oracle/liboracle.so
    python -m oracle.build --sanitize    # oracle/liboracle_san.so (ASan + UBSan)

The sanitised build is loaded through PSDF_ORACLE_LIB, with the ASan runtime
preloaded (sanitized_env() gives the environment)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SAN_LIB_PATH = os.path.join(HERE, "liboracle_san.so")

BASE = ["-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra"]
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=undefined"]


def build(verbose: bool = False, sanitize: bool = False, out: str | None = None) -> str:
    src = os.path.join(HERE, "oracle.c")
    dst = out or (SAN_LIB_PATH if sanitize else LIB_PATH)
    tmp = dst + ".tmp"
    flags = SANITIZE if sanitize else ["-O2"]
    cmd = ["gcc", *flags, *BASE, "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, dst)
    return dst


def sanitized_env(lib_path: str = SAN_LIB_PATH) -> dict:
    """Environment in which a Python process loads the sanitised oracle."""
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True, check=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True,
                           text=True, check=True).stdout.strip()
    env = dict(os.environ)
    env["LD_PRELOAD"] = " ".join(p for p in (asan, ubsan) if os.path.isabs(p))
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["PSDF_ORACLE_LIB"] = lib_path
    return env


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
