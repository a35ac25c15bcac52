"""The library driven from plain C: tests/c_abi_example (compiled by the
package build next to its source) runs a two-party Beaver matmul in the limb
and plain forms, an element-wise and a grouped product and the error codes
through include/mpc.h, and checks the revealed results exactly."""
import os
import subprocess

import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi_example")


def test_c_abi_example():
    say("c abi example")
    assert os.path.exists(EXE), "tests/c_abi_example is missing: run the package build first"
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "c_abi_example: all checks passed" in r.stdout
