"""The oracle's pin suite under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only).

The oracle is rebuilt with gcc's -fsanitize=address,undefined (every finding
fatal) and the oracle's CPU pin files run against that build in a child
process that preloads gcc's ASan runtime. A first child checks that the
instrumentation is live: an oracle call handed a buffer shorter than the
filter it is told about must be stopped with a heap-buffer-overflow report.
"""

import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_pins.py", "tests/test_oracle_comparators.py", "tests/test_oracle_distinct.py",
             "tests/test_oracle_qgrams.py", "tests/test_oracle_subarrays.py", "tests/test_oracle_validation.py"]


@pytest.fixture(scope="module")
def san_env(tmp_path_factory):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.fail("gcc's libasan.so is missing")
    lib = oracle.build(sanitize=True, out=str(tmp_path_factory.mktemp("san") / "liboracle_san.so"))
    env = dict(os.environ)
    env.update({oracle.LIB_ENV: lib, "LD_PRELOAD": asan,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=86",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87",
                "PYTHONPATH": ROOT})
    return env


def test_sanitizer_is_live(san_env):
    """A 3-block filter read as 4 blocks overflows its heap buffer."""
    code = ("import numpy as np, oracle\n"
            "f = oracle.OracleFilter(4, 1, 3)\n"
            "w = np.zeros(8 * 3 + 1, dtype=np.uint64)[1:]\n"
            "f.block_loads(w)\n")
    r = subprocess.run([sys.executable, "-c", code], env=san_env, cwd=ROOT, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 86, (r.returncode, r.stderr[-2000:])
    assert "heap-buffer-overflow" in r.stderr


def test_oracle_pins_pass_under_asan_and_ubsan(san_env):
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:xdist", "-p", "no:cacheprovider",
                        "-m", "not gpu", *PIN_FILES], env=san_env, cwd=ROOT, capture_output=True, text=True,
                       timeout=900)
    tail = (r.stdout[-3000:] + r.stderr[-3000:])
    assert r.returncode == 0, tail
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, tail
    assert " passed" in r.stdout
