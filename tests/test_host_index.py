"""Host checks of the kernels' index arithmetic: the invariant-divisor
division used to split a work item into (segment, y, z), the CSoA population
offsets (every (population, row, x) maps to a distinct element inside one
copy, also with a ragged last block), and the dense enumeration of the
face-layer nodes used by the adjoint's face kernel (every node on a
non-periodic face layer exactly once, nothing else).  Compiles a small host
program against the kernel header with hipcc; CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_divisor_and_layout_offsets(tmp_path):
    exe = tmp_path / "host_index_check"
    src = os.path.join(ROOT, "tests", "host_index_check.cpp")
    cmd = ["hipcc", "-O2", "-std=c++17", "-x", "hip", "--cuda-host-only", f"-I{ROOT}/include",
           f"-I{ROOT}/paper_2101_11856_amd/csrc", src, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout[-3000:]
