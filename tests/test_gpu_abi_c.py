"""The C ABI used from a C program (no Python in the loop): tests/abi_c/solve_example."""
import os
import subprocess

import pytest

from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "abi_c", "solve_example")


def test_c_program_through_the_abi():
    need_gpu()
    assert os.path.exists(EXE), "tests/abi_c/solve_example is missing: run __graft_entry__.build()"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    say(r.stdout.strip())
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
