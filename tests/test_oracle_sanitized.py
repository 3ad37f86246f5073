"""The oracle's pins run again with the oracle built under AddressSanitizer
and UndefinedBehaviorSanitizer (host code only; any report fails the run)."""
import os
import subprocess
import sys

import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_check_pins.py", "tests/test_dubins_pins.py",
        "tests/test_halton_pins.py", "tests/test_inputs_and_di_oracle.py"]


@pytest.mark.slow
def test_pins_under_asan_and_ubsan(tmp_path):
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    ubsan = subprocess.check_output(["gcc", "-print-file-name=libubsan.so"], text=True).strip()
    if not (os.path.isabs(asan) and os.path.exists(asan) and os.path.isabs(ubsan) and os.path.exists(ubsan)):
        pytest.skip("no sanitizer runtime in this toolchain")
    lib = O.build_sanitized(str(tmp_path / "liborc_san.so"))
    env = dict(os.environ)
    env.update({"GMT_ORACLE_LIB": lib, "LD_PRELOAD": asan + " " + ubsan,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1", "OMP_NUM_THREADS": "4"})
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu and not slow", "-p",
                        "no:cacheprovider"] + PINS, cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=1200)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout, tail
