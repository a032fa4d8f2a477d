"""The oracle's pins, and a call of every oracle entry point on edge-case inputs
(oracle_san_calls.py), run once more against an AddressSanitizer +
UndefinedBehaviorSanitizer build of the oracle (gcc, CPU only): any out-of-bounds
access, use after free or undefined arithmetic in the oracle aborts the run.  One
OpenMP thread: the sanitisers make the oracle's parallel regions very slow."""
import glob
import os
import subprocess
import sys

import pytest

from oracle import build as ob

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = sorted(os.path.relpath(p, ROOT) for p in glob.glob(os.path.join(ROOT, "tests",
                                                                      "test_oracle_*pins*.py")))


def test_oracle_pins_clean_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    try:
        ob.build(sanitize=True, out=lib)
        env = ob.sanitized_env(lib)
    except (subprocess.CalledProcessError, FileNotFoundError) as e:
        pytest.skip(f"no sanitiser toolchain: {e}")
    if "libasan" not in env.get("LD_PRELOAD", ""):
        pytest.skip("libasan runtime not found")
    env["OMP_NUM_THREADS"] = "1"
    assert len(PINS) >= 6, PINS
    for cmd in ([sys.executable, os.path.join("tests", "oracle_san_calls.py")],
                [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *PINS]):
        r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
        tail = (r.stdout + r.stderr)[-4000:]
        assert r.returncode == 0, tail
        assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
