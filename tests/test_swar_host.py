"""The byte-parallel (SWAR) helpers of the advance kernel, checked
exhaustively on the CPU: the header compiles for the host too."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_swar_helpers_exhaustive(tmp_path):
    from paper_1810_13132_amd.build import hipcc
    exe = str(tmp_path / "swar_check")
    src = os.path.join(ROOT, "tests", "swar_host_check.cpp")
    try:
        subprocess.check_call([hipcc(), "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1810_13132_amd", "csrc"),
                               "-I", os.path.join(ROOT, "include"), src, "-o", exe],
                              stderr=subprocess.DEVNULL)
    except (OSError, subprocess.CalledProcessError, RuntimeError):
        pytest.skip("hipcc host compile unavailable")
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "bad=0" in out.stdout
