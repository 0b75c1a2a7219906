"""The C ABI without Python (GPU only): tests/c_abi/bbfc_abi_check, a C
program built by the build step, creates filters, inserts and queries
through include/bbfc.h with hipMalloc'd buffers and compares with the
oracle (see its source for the checks)."""

import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "bbfc_abi_check")


def test_c_program_through_the_c_abi():
    assert os.path.exists(EXE), "tests/c_abi/bbfc_abi_check is missing: run the build step first"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "c abi check ok" in r.stdout
