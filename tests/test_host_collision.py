"""The fused kernel's collision functions compiled for the CPU in FP64
(tests/host_collision_check.cpp, from the kernel header) against the oracle's
single-cell collisions, on random near-equilibrium states with forces: the
general central-moment form, its form specialised to unit rates of orders 3
to 6, BGK and raw-moment MRT (the paper's Sec. 5.1 comparison models).  The
kernel works on deviations d = f - w; both sides see the same f.  CPU only."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("hc") / "host_collision_check"
    cmd = ["hipcc", "-O2", "-std=c++17", "-x", "hip", "--cuda-host-only", f"-I{ROOT}/include",
           f"-I{ROOT}/paper_2101_11856_amd/csrc", os.path.join(ROOT, "tests", "host_collision_check.cpp"),
           "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return str(out)


def _cases(seed, n):
    c, w, _, _ = O.lattice()
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        drift = rng.uniform(-0.08, 0.08, 3)
        f = w * (1 + 0.05 * rng.standard_normal(27)) + 3 * w * (c @ drift)
        F = rng.normal(0, 2e-3, 3)
        rates = rng.uniform(0.3, 1.99, 6)
        out.append((f, F, rates))
    return out


def _run(exe, model, cases):
    _, w, _, _ = O.lattice()
    lines = []
    for f, F, r in cases:
        vals = [model, *r, *F, *(f - w)]
        lines.append(" ".join(repr(float(v)) if i else str(v) for i, v in enumerate(vals)))
    res = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    return np.array([[float(x) for x in ln.split()] for ln in res.stdout.strip().splitlines()]) + w


@pytest.mark.parametrize("model", ["cm", "cm_unit_high", "bgk", "rm"])
def test_kernel_collision_matches_oracle(exe, model):
    cases = _cases({"cm": 1, "cm_unit_high": 2, "bgk": 3, "rm": 4}[model], 64)
    if model == "cm_unit_high":
        cases = [(f, F, np.concatenate([r[:2], np.ones(4)])) for f, F, r in cases]
    code = {"cm": 0, "cm_unit_high": 1, "bgk": 2, "rm": 3}[model]
    got = _run(exe, code, cases)
    worst = 0.0
    for (f, F, r), g in zip(cases, got):
        if model in ("cm", "cm_unit_high"):
            ref = O.collide(f, F, r[0], r[1], r[2:])
        elif model == "bgk":
            ref = O.collide_bgk(f, F, r[0])
        else:
            ref = O.collide_rm(f, F, r[0], r[1], r[2:])
        worst = max(worst, float(np.abs(g - ref).max() / np.abs(ref - O.lattice()[1]).max()))
    print(f"{model}: worst |kernel - oracle| / max|oracle deviation| = {worst:.2e}")
    assert worst < 1e-12
