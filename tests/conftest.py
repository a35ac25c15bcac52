import importlib.util
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def limb_gemm_asm(tmp_path_factory):
    """Device assembly of gemm_limb.hip for gfx950, built once per session
    with the library's own flags (skips where hipcc is absent)."""
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    spec = importlib.util.spec_from_file_location("mpc_build", os.path.join(ROOT, "paper_2109_00984_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    asm = tmp_path_factory.mktemp("isa") / "gemm_limb.s"
    cmd = ["hipcc", *[f for f in b.FLAGS if f != "-fPIC"], "-x", "hip", "--cuda-device-only", "-S",
           os.path.join(b.CSRC, "gemm_limb.hip"), "-o", str(asm)]
    subprocess.run(cmd, check=True, capture_output=True)
    return asm.read_text()
