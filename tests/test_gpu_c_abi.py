"""The C ABI from plain C: tests/c_abi/bn_c_check (built by __graft_entry__.build())
creates a context, allocates with the HIP runtime's C API, runs batched add, subtract
and both multiplication forms on its own stream and checks closed forms."""
import os
import subprocess

import pytest

from conftest import announce

pytestmark = pytest.mark.gpu
BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "bn_c_check")


def test_c_program():
    announce("C ABI from plain C", BIN)
    assert os.path.exists(BIN), "bn_c_check not built (run __graft_entry__.build())"
    p = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    assert p.returncode == 0 and p.stdout.strip().endswith("ok"), p.stdout + p.stderr
