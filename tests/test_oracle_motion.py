"""Pins of the oracle's moving-solid pieces: the rigid sample update and the
total torque of Alg. 2 (c).  Expected values are closed forms worked out by
hand, an independent rotation routine (scipy), or identities of rigid-body
mechanics, never a re-evaluation of the oracle's own formulas."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import oracle as orc

QUARTER_Z = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])   # +90 degrees about z


def test_identity_pose_returns_the_body_samples_exactly():
    rng = np.random.default_rng(7)
    X = rng.uniform(0.0, 30.0, (3, 50)).astype(np.float32)
    ub = rng.normal(0.0, 0.01, (3, 50)).astype(np.float32)
    xyz, u = orc.rigid_pose(X, ub, np.eye(3), (0, 0, 0), (0, 0, 0), (0, 0, 0))
    assert xyz.dtype == np.float32 and np.array_equal(xyz, X)
    assert np.array_equal(u, ub.astype(np.float64))


def test_quarter_turn_and_translation_closed_form():
    # body point (1, 2, 3) turned +90 degrees about z is (-2, 1, 3); placed at o
    xyz, u = orc.rigid_pose(np.array([[1.0], [2.0], [3.0]]), np.array([[1.0], [0.0], [0.0]]),
                            QUARTER_Z, (10.0, 20.0, 30.0), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    assert xyz[:, 0].tolist() == [8.0, 21.0, 33.0]
    assert u[:, 0].tolist() == [0.0, 1.0, 0.0]          # the body-frame velocity turns with the body


def test_rigid_velocity_closed_form():
    # spin about z at rate 0.5 through o, plus a drift v: a point 2 along +x
    # from o moves along +y at 1.0, a point 3 along +y moves along -x at 1.5
    X = np.array([[2.0, 0.0], [0.0, 3.0], [0.0, 0.0]])
    _, u = orc.rigid_pose(X, None, np.eye(3), (4.0, 5.0, 6.0), (0.01, 0.02, 0.03), (0.0, 0.0, 0.5))
    assert np.allclose(u[:, 0], [0.01, 1.02, 0.03], rtol=0, atol=1e-15)
    assert np.allclose(u[:, 1], [-1.49, 0.02, 0.03], rtol=0, atol=1e-15)


def test_rigid_velocity_is_the_time_derivative_of_the_motion():
    """u_b of a body turning at constant angular velocity w about a point moving
    at v equals the central difference of the placed positions."""
    rng = np.random.default_rng(11)
    X = rng.uniform(-1.0, 1.0, (3, 40))
    w = np.array([0.3, -0.2, 0.4])
    v = np.array([0.05, -0.03, 0.02])
    o0 = np.array([2.0, 3.0, 4.0])
    t, h = 0.7, 0.01

    def place(tt):
        R = Rotation.from_rotvec(w * tt).as_matrix()
        return orc.rigid_pose(X, None, R, o0 + v * tt, v, w)

    xp, _ = place(t + h)
    xm, _ = place(t - h)
    _, u = place(t)
    fd = (xp.astype(np.float64) - xm.astype(np.float64)) / (2 * h)
    assert np.max(np.abs(fd - u)) < 2e-4


def _uniform_sim(U, n=12):
    sim = orc.OracleSim(n, n, n, 0.05)
    rho = np.ones((n, n, n))
    u = np.zeros((3, n, n, n))
    for a in range(3):
        u[a] = U[a]
    sim.init_equilibrium(rho, u)
    return sim


def test_torque_of_uniform_flow_closed_form():
    """Samples at rest in a uniform stream U along x feel g_s = -gamma_s U (rho = 1,
    trilinear interpolation of a constant is the constant).  About o, a sample at
    o + 3 e_y gives torque 3 a gamma U e_z, one at o - 2 e_z gives 2 a gamma U e_y,
    and one at o + 1.5 e_x (lever parallel to the force) gives none."""
    U = 0.03
    sim = _uniform_sim((U, 0.0, 0.0))
    o = np.array([5.25, 6.5, 4.75])
    xyz = np.array([o + [0, 3, 0], o + [0, 0, -2], o + [1.5, 0, 0]]).T.astype(np.float32)
    area = np.array([0.5, 0.25, 0.7])
    gain = np.array([3.0, 2.0, 1.3])
    sim.set_markers(xyz, None, area, gain)
    F = sim.ib_force()
    T = sim.last_torque(o)
    assert np.allclose(F, [-U * (1.5 + 0.5 + 0.91), 0, 0], rtol=1e-12, atol=1e-15)
    assert np.allclose(T, [0.0, 2 * 0.5 * U, 3 * 1.5 * U], rtol=1e-12, atol=1e-15)


def test_torque_of_a_spinning_ring_in_fluid_at_rest():
    """A ring of radius r spinning at w e_z in fluid at rest drags the fluid with it:
    g_s = gamma w x (x_s - o), so the torque on the fluid is n a gamma r^2 w e_z and
    the net force vanishes."""
    n_s, r, w, a, gam = 64, 3.0, 0.01, 0.4, 2.5
    sim = _uniform_sim((0.0, 0.0, 0.0), n=16)
    th = 2 * np.pi * np.arange(n_s) / n_s
    X = np.array([r * np.cos(th), r * np.sin(th), np.zeros(n_s)])
    o = (8.0, 8.0, 8.0)
    xyz, ub = orc.rigid_pose(X, None, np.eye(3), o, (0, 0, 0), (0, 0, w))
    sim.set_markers(xyz, ub, np.full(n_s, a), np.full(n_s, gam))
    F = sim.ib_force()
    T = sim.last_torque(o)
    scale = n_s * a * gam * r * w                       # sum of the force magnitudes
    assert np.max(np.abs(F)) < 1e-7 * scale             # FP32 placement of the samples
    assert abs(T[2] - n_s * a * gam * r * r * w) < 1e-6 * n_s * a * gam * r * r * w
    assert np.max(np.abs(T[:2])) < 1e-7 * scale * r


def test_torque_moves_with_the_reference_point():
    """T(o') = T(o) + (o - o') x F for any two reference points."""
    rng = np.random.default_rng(5)
    n = 12
    sim = orc.OracleSim(n, n, n, 0.05)
    rho = 1.0 + 0.01 * rng.standard_normal((n, n, n))
    u = 0.03 * rng.standard_normal((3, n, n, n))
    sim.init_equilibrium(rho, u)
    xyz = rng.uniform(0.0, n, (3, 30)).astype(np.float32)
    sim.set_markers(xyz, 0.01 * rng.standard_normal((3, 30)), rng.uniform(0.5, 1.5, 30), rng.uniform(0.5, 2, 30))
    F = sim.ib_force()
    o, o2 = np.array([1.0, 2.0, 3.0]), np.array([7.5, -4.0, 0.25])
    d = o - o2
    shift = np.array([d[1] * F[2] - d[2] * F[1], d[2] * F[0] - d[0] * F[2], d[0] * F[1] - d[1] * F[0]])
    assert np.allclose(sim.last_torque(o2), sim.last_torque(o) + shift, rtol=1e-12, atol=1e-14)
