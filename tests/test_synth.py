"""The seeded input generators produce what the input recipe states
(shapes, spectra, sample geometry).  CPU only."""
import math

import numpy as np

from paper_2101_11856_amd import synth


def test_turbulence_spectrum_rms_and_divergence():
    n = 48
    rho, u = synth.turbulence(n, kmax=12)
    assert u.shape == (3, n, n, n) and rho.shape == (n, n, n)
    rms = math.sqrt(float((u.astype(np.float64) ** 2).sum(0).mean()) / 3)
    assert abs(rms - 0.04) < 1e-6
    assert np.abs(rho - 1).max() <= 1e-3 + 1e-7
    # solenoidal: spectral divergence ~ 0
    k = np.fft.fftfreq(n, d=1.0 / n)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    U = [np.fft.fftn(u[a].astype(np.float64)) for a in range(3)]
    div = KX * U[0] + KY * U[1] + KZ * U[2]
    assert np.abs(div).max() < 1e-6 * max(np.abs(U[0]).max(), 1e-30) * n
    # shell energy slope ~ -5/3 over the forced shells
    kmag = np.rint(np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)).astype(int)
    E = np.bincount(kmag.ravel(), weights=sum(np.abs(Ua) ** 2 for Ua in U).ravel())
    shells = np.arange(2, 12)
    slope = np.polyfit(np.log(shells), np.log(E[shells]), 1)[0]
    assert abs(slope + 5.0 / 3.0) < 0.25
    assert E[13:].sum() < 1e-12 * E[1:13].sum()   # only float32 round-off outside the shells


def test_turbulence_box_periodic_solenoidal_and_cubic_consistent():
    nx, ny, nz = 64, 16, 8
    rho, u = synth.turbulence_box(nx, ny, nz, kmax=12)
    assert u.shape == (3, nz, ny, nx) and rho.shape == (nz, ny, nx)
    rms = math.sqrt(float((u.astype(np.float64) ** 2).sum(0).mean()) / 3)
    assert abs(rms - 0.04) < 1e-6
    # divergence-free in the box's own wave numbers (periodic on the box)
    L = max(nx, ny, nz)
    kx, ky, kz = (np.fft.fftfreq(n, d=1.0 / n) * (L / n) for n in (nx, ny, nz))
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    U = [np.fft.fftn(u[a].astype(np.float64)) for a in range(3)]
    div = KX * U[0] + KY * U[1] + KZ * U[2]
    assert np.abs(div).max() < 1e-6 * np.abs(U[0]).max() * L
    # only modes inside the shells carry energy
    shell = np.rint(np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)).astype(int)
    E = sum(np.abs(Ua) ** 2 for Ua in U)
    assert E[(shell > 12) | (shell < 1)].sum() < 1e-12 * E.sum()
    # on a cube it draws the same field as the cubic generator
    r1, u1 = synth.turbulence_box(24, 24, 24, kmax=8)
    r2, u2 = synth.turbulence(24, kmax=8)
    assert np.array_equal(r1, r2) and np.allclose(u1, u2, atol=1e-7)


def test_taylor_green_is_divergence_free_and_decays_in_closed_form():
    rho, u = synth.taylor_green(16, 0.05)
    assert np.allclose(rho, 1) and np.abs(u[2]).max() == 0
    # central-difference divergence vanishes for this field
    dudx = (np.roll(u[0], -1, 2) - np.roll(u[0], 1, 2)) / 2
    dvdy = (np.roll(u[1], -1, 1) - np.roll(u[1], 1, 1)) / 2
    assert np.abs(dudx + dvdy).max() < 1e-15


def test_sphere_scene_geometry():
    xyz, ub, area, gain = synth.sphere_scene()
    assert xyz.shape == (3, 213000) and ub.shape == (3, 213000)
    r = np.linalg.norm(xyz[:, :13000].astype(np.float64) - np.array([[128.0], [64.0], [64.0]]), axis=0)
    assert np.abs(r - 16).max() < 1e-4
    assert abs(area[:13000].sum() - 4 * math.pi * 256) < 1e-2
    box = xyz[:, 13000:]
    assert box[0].min() >= 284 and box[0].max() < 316 and box[1].min() >= 48 and box[2].max() < 80
    assert abs(area[13000:].sum() - 32 ** 3) < 1.0 and (gain == 1).all() and (ub == 0).all()


def test_city_scene():
    boxes = synth.city_boxes()
    assert boxes.shape == (400, 5)
    x0, z0, sx, sz, h = boxes.T
    assert (sx >= 10).all() and (sx <= 60).all() and (h >= 20).all() and (h <= 200).all()
    assert (x0 >= 150).all() and (x0 + sx <= 1000).all() and (z0 >= 2).all() and (z0 + sz <= 838).all()
    xyz, ub, area, gain = synth.city_markers(boxes)
    assert 3.5e6 < xyz.shape[1] < 4.2e6
    frac = xyz - np.floor(xyz)
    assert np.allclose(frac, 0.5)   # half-integer coordinates
    assert xyz[1].max() < 249 and xyz[1].min() > 0


def test_cylinder_and_inlet_modes():
    xyz, ub, area, gain = synth.cylinder_markers(8.0, (32.0, 32.0), 64, 50)
    assert xyz.shape == (3, 3200)
    r = np.hypot(xyz[0] - 32.0, xyz[1] - 32.0)
    assert np.abs(r - 8).max() < 1e-4 and abs(area[0] - 2 * math.pi * 8 / 50) < 1e-6
    B = synth.inlet_mode_basis(64, 64)
    assert B.shape == (16, 64, 64)
    G = B.reshape(16, -1) @ B.reshape(16, -1).T
    assert np.allclose(G, np.diag(np.diag(G)), atol=1e-9)    # orthogonal sin-sin modes
    a = synth.inlet_coefficients(2105)
    assert a.shape == (16,) and np.abs(a).max() <= 0.01
    prof = synth.inlet_profile(64, 64, a)
    assert prof.shape == (3, 64, 64) and np.allclose(prof[1:], 0)
    assert np.allclose(prof[0], 0.04 + np.tensordot(a, B, 1))


def test_torus_body_and_rotation():
    import math
    from scipy.spatial.transform import Rotation
    xyz, area = synth.torus_body(12.0, 4.0, per_length=2.0)
    p = xyz.astype(np.float64)
    tube = np.hypot(np.hypot(p[0], p[1]) - 12.0, p[2])     # distance to the tube's centre circle
    assert np.allclose(tube, 4.0, atol=1e-5)
    assert abs(area.astype(np.float64).sum() - 4 * math.pi ** 2 * 12.0 * 4.0) < 1e-4 * 4 * math.pi ** 2 * 48
    axis, ang = np.array([0.3, -0.5, 0.8]), 0.7
    R = synth.rotation(axis, ang)
    ref = Rotation.from_rotvec(axis / np.linalg.norm(axis) * ang).as_matrix()
    assert np.allclose(R, ref, atol=1e-14)
