"""The blend kernels' XCD-aware block -> tile mapping, checked on the host by
compiling the real header (tests/native/xcd_map_check.hip): a bijection for
random mixes of view sizes, smaller views first."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not on PATH")
def test_xcd_mapping_is_a_bijection(tmp_path):
    exe = tmp_path / "xcd_map_check"
    subprocess.run(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2503_18402_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "xcd_map_check.hip"), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
