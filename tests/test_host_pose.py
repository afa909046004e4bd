"""Host check of the bound with which lbm_set_pose places a moving solid
without waiting for the device: for random bodies and poses (many grazing a
face), an accepted pose never places a sample outside the domain under the
kernel's own placement arithmetic.  Compiles a small host program against the
kernel header with hipcc; CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_pose_bound_is_sound(tmp_path):
    exe = tmp_path / "host_pose_check"
    src = os.path.join(ROOT, "tests", "host_pose_check.cpp")
    cmd = ["hipcc", "-O2", "-std=c++17", "-x", "hip", "--cuda-host-only", f"-I{ROOT}/include",
           f"-I{ROOT}/paper_2101_11856_amd/csrc", src, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(out.stdout)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout[-3000:]
