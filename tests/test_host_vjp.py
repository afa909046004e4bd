"""Host check of the collision's hand-written reverse mode: collide_vjp
(the per-node transpose used by the adjoint kernels) against central
differences of the forward collision, both compiled for the CPU from the
kernel headers in FP64 (tests/host_vjp_check.cpp).  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_collision_vjp_matches_central_differences(tmp_path):
    exe = tmp_path / "host_vjp_check"
    src = os.path.join(ROOT, "tests", "host_vjp_check.cpp")
    cmd = ["hipcc", "-O2", "-std=c++17", "-x", "hip", "--cuda-host-only", f"-I{ROOT}/include",
           f"-I{ROOT}/paper_2101_11856_amd/csrc", src, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(out.stdout)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout[-3000:]
