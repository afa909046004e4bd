"""The library used from plain C: the C client in tests/c_abi (built with the
library) runs on the GPU as a child process and checks uniform flow as a fixed
point with mass and momentum conserved, the force and torque of one sample in
a uniform stream against their closed forms, and the error codes of invalid
calls."""
import os
import subprocess

import pytest

from tests.gpu_cases import say

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "c_abi_check")


def test_plain_c_client():
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is not built (the repository's build step builds it)")
    say("plain C client of liblbm")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks hold" in r.stdout
