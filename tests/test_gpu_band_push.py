"""Band pieces: the fused kernel writes, for the next step's band nodes, the
sums of Eq. (2) split by source row (two values per row, nine rows), and the
band pre-pass reads them instead of pulling 27 scattered values.  The pull
form adds the same pieces in the same order, so the two give the same bits:
every run here is made twice, pieces forced on (LBM_BAND_PUSH=1) and off
(=0), and the states, scalar, macros and forces must be identical.

The scenes put band nodes at the first and last node of 64-node segments
(whose piece misses a value from the neighbouring segment), in the ragged
last segment, on and next to the faces (where the pre-pass pulls), and the
steps cross every point where the pieces go stale: a restore, a new set of
samples and a new pose before each step of a moving body.
"""
import numpy as np
import pytest
import torch

from paper_2101_11856_amd import synth
from tests.gpu_cases import FS, IN, NS, OUT, P, gpu_solver, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_11856_amd import lbm  # noqa: F401
    yield


SHAPE = (150, 18, 16)  # segments of 64, 64 and 22 nodes


def _scene(seed):
    nx, ny, nz = SHAPE
    rng = np.random.default_rng(seed)
    parts = [
        synth.fibonacci_sphere(500, 5.0, (64.0, ny / 2 + 0.3, nz / 2 - 0.2)),    # across x = 63 | 64
        synth.random_box(800, (125.0, 4.0, 5.0), (131.5, 11.0, 10.0), seed),     # across x = 127 | 128
        synth.fibonacci_sphere(200, 3.0, (144.0, ny / 2, nz / 2)),               # ragged segment, outflow face
        synth.random_box(300, (20.0, 0.2, 0.5), (30.0, 3.0, 4.0), seed + 1),     # y and z faces
        np.array([[0.5, 1.5], [8.0, 16.5], [7.0, 14.5]], np.float32),            # inlet face, high y and z
    ]
    xyz = np.concatenate(parts, axis=1).astype(np.float32)
    n = xyz.shape[1]
    ub = (0.01 * rng.standard_normal((3, n))).astype(np.float32)
    area = (0.3 + 0.4 * rng.random(n)).astype(np.float32)
    gain = (0.5 + rng.random(n)).astype(np.float32)
    return xyz, ub, area, gain


def _flow(seed):
    nx, ny, nz = SHAPE
    rng = np.random.default_rng(seed)
    rho = (1.0 + 1e-3 * rng.standard_normal((nz, ny, nx))).astype(np.float32)
    u = (0.03 + 0.005 * rng.standard_normal((3, nz, ny, nx))).astype(np.float32)
    return rho, u


def _static_run(storage, faces, push, monkeypatch):
    monkeypatch.setenv("LBM_BAND_PUSH", push)
    nx, ny, nz = SHAPE
    s = gpu_solver(nx, ny, nz, 0.03, storage=storage, faces=faces, u_in=(0.04, 0, 0), scalar=True,
                   scalar_inlet_height=6)
    rho, u = _flow(3)
    s.init_equilibrium(rho, u)
    s.set_scalar(np.random.default_rng(4).uniform(0.0, 1.0, (nz, ny, nx)).astype(np.float32))
    s.set_solids(*_scene(5))
    s.step(4)
    snap = s.checkpoint().clone()
    s.step(3)
    s.restore(snap)                       # pieces stale: the next pre-pass pulls
    s.step(2)
    F = np.asarray(s.ib_force())
    s.set_solids(*_scene(6))              # a new band
    s.step(3)
    r, v = s.macros()
    out = dict(f=s.get_populations().cpu(), sc=s.get_scalar().cpu(), rho=r.cpu(), u=v.cpu())
    torch.cuda.synchronize()
    return out, F, np.asarray(s.ib_force())


STATIC = [("periodic", (P, P, P, P, P, P)), ("inlet-outflow-walls", (IN, OUT, NS, FS, P, P)),
          ("channel", (IN, OUT, NS, NS, NS, FS))]


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16", "f64"])
@pytest.mark.parametrize("name,faces", STATIC, ids=[c[0] for c in STATIC])
def test_pieces_equal_pulls_bitwise(name, faces, storage, monkeypatch):
    say(f"band pieces on vs off, {SHAPE} {name} {storage}")
    (a, Fa1, Fa2), (b, Fb1, Fb2) = (_static_run(storage, faces, p, monkeypatch) for p in ("1", "0"))
    for k in a:
        assert torch.equal(a[k], b[k]), k
    assert np.array_equal(Fa1, Fb1) and np.array_equal(Fa2, Fb2)
    assert np.isfinite(a["f"].double().numpy()).all() and np.abs(Fa2).sum() > 0


def test_pieces_with_a_moving_body(monkeypatch):
    """A new pose before every step leaves no valid pieces (each pre-pass
    pulls), and steps between poses (two per pose here) use them."""
    nx, ny, nz = SHAPE
    X, area = synth.torus_body(5.0, 2.0, per_length=2.0)
    rng = np.random.default_rng(8)
    gain = rng.uniform(0.8, 1.2, X.shape[1]).astype(np.float32)
    ub = (0.002 * rng.standard_normal(X.shape)).astype(np.float32)
    say(f"band pieces on vs off, moving torus in {SHAPE}")
    runs = []
    for push in ("1", "0"):
        monkeypatch.setenv("LBM_BAND_PUSH", push)
        s = gpu_solver(nx, ny, nz, 0.03, storage="f32", faces=(IN, OUT, NS, FS, P, P), u_in=(0.04, 0, 0))
        s.init_equilibrium(*_flow(9))
        o = np.array([63.5, ny / 2, nz / 2])
        s.set_body(X, ub, area, gain, np.eye(3), o, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
        forces = []
        for t in range(5):
            R = synth.rotation(np.array([0.0, 0.0, 1.0]), 0.05 * t)
            s.set_pose(R, o + np.array([0.3 * t, 0.0, 0.0]), (0.3, 0.0, 0.0), (0.0, 0.0, 0.05))
            s.step(2)
            forces.append(np.asarray(s.ib_force()))
        runs.append((s.get_populations().cpu(), np.array(forces)))
    assert torch.equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
