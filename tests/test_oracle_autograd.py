"""Pins of the second FP64 model (plain PyTorch, differentiated by
torch.autograd) that the adjoint tests compare against.

Its objective equals the C oracle's on the same inputs (two independent
implementations of the step), and its autograd gradient equals central
differences of the C oracle.  CPU only."""
import numpy as np
import pytest
import torch

from oracle import autograd_model as AM
from oracle import oracle as O
from paper_2101_11856_amd import synth

TINY = dict(nx=16, ny=8, nz=8, nu=0.05, steps=10, probe_x=12, radius=1.5, center=(5.0, 4.0), n_around=8,
            mode_length=8.0)
CHANNEL = (O.INLET, O.OUTFLOW) + (O.NOSLIP,) * 4
# ground no-slip, free-slip top, periodic z: exercises the other face rules
OPEN = (O.INLET, O.OUTFLOW, O.NOSLIP, O.FREESLIP, O.PERIODIC, O.PERIODIC)


def _markers(c):
    xyz, ub, area, _ = synth.cylinder_markers(c["radius"], c["center"], c["nz"], c["n_around"])
    keep = xyz[2] < c["nz"] - 1
    return xyz[:, keep], ub[:, keep], area[keep]


def _gains(n):
    rng = np.random.default_rng(77)
    return (0.8 + 0.4 * rng.random(n)).astype(np.float32).astype(np.float64)


def oracle_J(c, faces, coeffs, gains):
    xyz, ub, area = _markers(c)
    S = O.OracleSim(c["nx"], c["ny"], c["nz"], c["nu"], faces=faces)
    S.set_inlet_profile(synth.inlet_profile(c["ny"], c["nz"], coeffs, length=c["mode_length"]))
    S.set_markers(xyz, ub.astype(np.float64), area.astype(np.float64), np.asarray(gains, np.float64))
    rho, u = synth.uniform(c["nx"], c["ny"], c["nz"], (0.04, 0, 0), dtype=np.float64)
    S.init_equilibrium(rho, u)
    S.step(c["steps"])
    F = S.ib_force()
    _, uu = S.macros()
    probe = uu[:, :, :, c["probe_x"]]
    return -F[0] + ((probe - np.array([0.04, 0, 0])[:, None, None]) ** 2).sum()


def autograd_J(c, faces, coeffs, gains):
    """Returns (J, dJ/dcoeffs, dJ/dgains) of the autograd model."""
    xyz, ub, area = _markers(c)
    M = AM.Channel(c["nx"], c["ny"], c["nz"], c["nu"], faces, xyz, ub, area)
    B = torch.as_tensor(synth.inlet_mode_basis(c["ny"], c["nz"], length=c["mode_length"]), dtype=torch.float64)
    a = torch.tensor(np.asarray(coeffs, np.float64), requires_grad=True)
    g = torch.tensor(np.asarray(gains, np.float64), requires_grad=True)
    ux = 0.04 + torch.tensordot(a, B, dims=1)
    u_in = torch.cat([ux.reshape(1, -1), torch.zeros((2, c["nz"] * c["ny"]), dtype=torch.float64)])
    rho, u = synth.uniform(c["nx"], c["ny"], c["nz"], (0.04, 0, 0), dtype=np.float64)
    J = M.run(u_in, g, c["steps"], rho, u, c["probe_x"])
    J.backward()
    return float(J.detach()), a.grad.numpy(), g.grad.numpy()


def test_lattice_tables_are_the_d3q27_moments():
    # closed forms of the weights: sum 1, zero mean, isotropic second moment
    assert abs(float(AM.W.sum()) - 1.0) < 1e-15
    assert torch.allclose(AM.W @ AM.CV, torch.zeros(3, dtype=torch.float64), atol=1e-16)
    second = (AM.W[:, None, None] * AM.CV[:, :, None] * AM.CV[:, None, :]).sum(0)
    assert torch.allclose(second, torch.eye(3, dtype=torch.float64) / 3, atol=1e-15)
    assert torch.equal(AM.CV.flip(0), -AM.CV)      # opposite of i is 26 - i


@pytest.mark.parametrize("faces", [CHANNEL, OPEN], ids=["channel", "open"])
def test_objective_equals_c_oracle(faces):
    c = TINY
    coeffs = 0.5 * synth.inlet_coefficients(seed=2105)
    gains = _gains(_markers(c)[0].shape[1])
    Jm, _, _ = autograd_J(c, faces, coeffs, gains)
    Jo = oracle_J(c, faces, coeffs, gains)
    assert abs(Jm - Jo) <= 1e-12 * abs(Jo), (Jm, Jo)


def test_autograd_gradient_equals_oracle_central_differences():
    c = TINY
    coeffs = 0.5 * synth.inlet_coefficients(seed=2105)
    gains = _gains(_markers(c)[0].shape[1])
    _, ga, gg = autograd_J(c, CHANNEL, coeffs, gains)
    h = 1e-6
    fd = np.zeros(16)
    for k in range(16):
        e = np.zeros(16)
        e[k] = h
        fd[k] = (oracle_J(c, CHANNEL, coeffs + e, gains) - oracle_J(c, CHANNEL, coeffs - e, gains)) / (2 * h)
    d = np.random.default_rng(5).standard_normal(gains.shape)
    fd_d = (oracle_J(c, CHANNEL, coeffs, gains + h * d) - oracle_J(c, CHANNEL, coeffs, gains - h * d)) / (2 * h)
    assert np.linalg.norm(ga - fd) <= 1e-7 * np.linalg.norm(fd)
    assert abs(gg @ d - fd_d) <= 1e-7 * abs(fd_d)
