"""The C ABI used from a C program, without Python (tests/c/ori_abi_smoke.c,
built next to the library by paper_1602_04691_amd/build.py): the
two-per-side closed form of eq. 2.19, the refusal of host pointers and
unsupported sizes, and a group of two problems solved in one launch per
kernel, bitwise each problem's own solve."""

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(__file__), "c", "ori_abi_smoke")


def test_c_program_solves_closed_form():
    assert os.path.exists(BIN), f"{BIN} is missing: build with python -m paper_1602_04691_amd.build"
    print("[c abi] running", BIN, file=sys.stderr, flush=True)
    p = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    print(p.stdout, p.stderr, file=sys.stderr, flush=True)
    assert p.returncode == 0, p.stderr
    assert p.stdout.startswith("OK ")
