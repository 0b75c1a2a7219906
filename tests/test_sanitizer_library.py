"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only).

The C ABI's and the server's host code is rebuilt with sanitizers (every
finding fatal; device code untouched), linked with the regular objects, and
the library's CPU tests run against that build in a child process that
preloads the compiler's ASan runtime. A first child checks that the
instrumentation is live: the rank-table call handed an output array shorter
than the table it fills must be stopped with a heap-buffer-overflow report.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def san_env():
    from paper_2501_18977_amd import _build

    if any(not os.path.exists(os.path.join(_build.HERE, "_build", s + ".o")) for s in _build.SOURCES):
        _build.build()
    lib = _build.build_host_sanitized()
    clang = os.path.join(os.path.dirname(os.path.realpath(_build.hipcc())), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    rt = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.fail("the compiler's ASan runtime is missing")
    env = dict(os.environ)
    env.update({"BBFC_LIBRARY": lib, "LD_PRELOAD": rt,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=86",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=86",
                "PYTHONPATH": ROOT})
    return env


def test_sanitizer_is_live(san_env):
    """A rank table of k = 11 (12 * 513 entries) written into 100 entries."""
    code = ("import ctypes, numpy as np\n"
            "import paper_2501_18977_amd as bbfc\n"
            "out = np.zeros(100, dtype=np.uint16)\n"
            "bbfc.lib().bbfc_rank_table(bbfc._Cost(2, float('nan')), 11, out.ctypes.data)\n")
    r = subprocess.run([sys.executable, "-c", code], env=san_env, cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 86, (r.returncode, r.stderr[-2000:])
    assert "heap-buffer-overflow" in r.stderr


def test_library_cpu_tests_pass_under_asan_and_ubsan(san_env):
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:xdist", "-p", "no:cacheprovider",
                        "-s", "-m", "not gpu", "tests/test_abi_cpu.py"], env=san_env, cwd=ROOT,
                       capture_output=True, text=True, timeout=900)
    tail = (r.stdout[-3000:] + r.stderr[-3000:])
    assert r.returncode == 0, tail
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, tail
    assert " passed" in r.stdout
