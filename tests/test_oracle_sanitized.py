"""The oracle's pins, run once more against an AddressSanitizer +
UndefinedBehaviorSanitizer build of the oracle (gcc, CPU only): any out-of-bounds
access, use after free or undefined arithmetic in the oracle aborts the run."""
import os
import subprocess
import sys

import pytest

from oracle import build as ob

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_pins_model.py",
        "tests/test_oracle_grad_pins.py"]


def test_oracle_pins_clean_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    try:
        ob.build(sanitize=True, out=lib)
        env = ob.sanitized_env(lib)
    except (subprocess.CalledProcessError, FileNotFoundError) as e:
        pytest.skip(f"no sanitiser toolchain: {e}")
    if "libasan" not in env.get("LD_PRELOAD", ""):
        pytest.skip("libasan runtime not found")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
