"""Pins of the oracle's lattice, moment basis and single-cell collision
against what the paper prints and what the mathematics fixes.

Paper: Sec. 3 Eqs. (2), (4), (5); Sec. 4.4.2 (expression for Omega_26);
Table 2.  The oracle is test infrastructure (oracle/), independent of the HIP
library.
"""
import itertools
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "inverse_moment_coefficients.txt")


def test_lattice_isotropy_and_weights():
    c, w, opp, e = O.lattice()
    cs2 = 1.0 / 3.0
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(w @ c).max() < 1e-15
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), cs2 * np.eye(3), atol=1e-15)
    # fourth-order isotropy: sum w c_a c_b c_c c_d = cs^4 (d_ab d_cd + d_ac d_bd + d_ad d_bc)
    d = np.eye(3)
    iso = cs2 * cs2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                       + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso, atol=1e-15)
    # classes by index: 0 rest, 1-6 faces, 7-18 edges, 19-26 corners
    nz = np.abs(c).sum(1)
    assert nz[0] == 0 and (nz[1:7] == 1).all() and (nz[7:19] == 2).all() and (nz[19:] == 3).all()
    assert np.allclose(w[[0, 1, 7, 19]], [8 / 27, 2 / 27, 1 / 54, 1 / 216], atol=1e-16)
    assert (c[opp] == -c).all()
    assert tuple(c[26]) == (-1, -1, -1)
    # the 27 velocities are all distinct; moments ordered by total order
    assert len({tuple(v) for v in c}) == 27
    order = e.sum(1)
    assert list(order) == sorted(order) and (np.bincount(order) == [1, 3, 6, 7, 6, 3, 1]).all()


@pytest.mark.parametrize("u", [(0.0, 0.0, 0.0), (0.03, -0.02, 0.05), (0.3, 0.7, -0.9)])
def test_central_transform_invertible(u):
    """T(u) is a Kronecker product of three 3x3 Vandermonde matrices of the
    points c - u_a, each of determinant 2, so |det T| = 2^27 for any u."""
    T = O.central_matrix(u)
    assert abs(abs(np.linalg.det(T)) / 2.0 ** 27 - 1.0) < 1e-12
    rng = np.random.default_rng(1)
    f = rng.random(27)
    M = O.basis_matrix(u)
    back = O.inverse(M) @ (M @ f)
    assert np.abs(back - f).max() / np.abs(f).max() < 1e-13


def _poly_coefficients():
    """M^{-1}(u) entries are polynomials of degree <= 2 in each u_a; recover
    all 27 coefficients per entry from a 3x3x3 grid of u (exact up to
    rounding)."""
    nodes = np.array([-0.5, 0.0, 0.5])
    V1 = np.stack([nodes ** 0, nodes, nodes ** 2], 1)
    V = np.kron(np.kron(V1, V1), V1)
    vals = np.array([O.inverse(O.basis_matrix(u)) for u in itertools.product(nodes, nodes, nodes)])
    return np.linalg.solve(V, vals.reshape(27, -1)).reshape(3, 3, 3, 27, 27)


def test_inverse_matches_printed_coefficients():
    """Every coefficient listed in the golden file (printed in the paper's
    Omega_26 expression, Sec. 4.4.2, and Table 2) is reproduced."""
    coef = _poly_coefficients()
    rows = 0
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        i, k, px, py, pz, num, den, _src = line.split()
        got = coef[int(px), int(py), int(pz), int(i), int(k)]
        assert abs(got - int(num) / int(den)) < 1e-10, line
        rows += 1
    assert rows >= 50


def test_equilibrium_is_maxwellian_in_central_moments():
    """The product-form equilibrium has exactly the Maxwellian central moments
    rho cs^(a+b+c) (all-even exponents), 0 otherwise; and is u-shifted
    consistently: sum f = rho, sum c f = rho u."""
    c, w, _, e = O.lattice()
    for rho, u in [(1.0, (0, 0, 0)), (1.03, (0.05, -0.02, 0.01)), (0.97, (0.2, 0.1, -0.3))]:
        feq = O.equilibrium(rho, u)
        kap = O.central_matrix(u) @ feq
        ref = np.array([0.0 if (ee == 1).any() else rho * (1 / 3) ** (ee.sum() // 2) for ee in e])
        assert np.abs(kap - ref).max() < 1e-14
        assert abs(feq.sum() - rho) < 1e-14
        assert np.abs(c.T @ feq - rho * np.asarray(u)).max() < 1e-14
    assert np.abs(O.equilibrium(1.0, (0, 0, 0)) - w).max() < 1e-16


def _rand_state(seed, rho=1.0, u=(0.04, -0.03, 0.02), amp=0.05):
    rng = np.random.default_rng(seed)
    feq = O.equilibrium(rho, u)
    return feq * (1.0 + amp * rng.standard_normal(27))


@pytest.mark.parametrize("seed", range(5))
def test_collision_conserves_mass_and_adds_force(seed):
    """Eq. (1) is conservative in rho and j (Sec. 3): post-collision mass
    equals pre-collision mass, and momentum rises by exactly F."""
    c, _, _, _ = O.lattice()
    rng = np.random.default_rng(100 + seed)
    f = _rand_state(seed)
    F = 1e-3 * rng.standard_normal(3)
    rates = dict(s_nu=1.0 + rng.random(), s_b=0.5 + rng.random(), s_high=tuple(0.5 + rng.random(4)))
    fp = O.collide(f, F, **rates)
    assert abs(fp.sum() - f.sum()) < 1e-14
    assert np.abs(c.T @ fp - (c.T @ f + F)).max() < 1e-14


def test_collision_fixed_points():
    """Rest state and uniform flow at equilibrium are fixed points of
    collision (m = m_eq exactly, Eq. 5)."""
    for u in [(0, 0, 0), (0.05, 0.0, 0.0), (0.03, -0.04, 0.02)]:
        feq = O.equilibrium(1.0, u)
        for s_nu in (1.0, 1.5, 1.9988):
            fp = O.collide(feq, (0, 0, 0), s_nu=s_nu, s_b=1.3, s_high=(0.7, 1.1, 1.2, 1.4))
            assert np.abs(fp - feq).max() < 1e-15


def test_unit_rates_give_equilibrium():
    """With every rate 1 and no force, collision returns f_eq(rho, u)
    (all non-conserved moments reset to their equilibrium values)."""
    c, _, _, _ = O.lattice()
    f = _rand_state(7)
    rho = f.sum()
    u = (c.T @ f) / rho
    fp = O.collide(f, (0, 0, 0), s_nu=1.0, s_b=1.0, s_high=(1, 1, 1, 1))
    assert np.abs(fp - O.equilibrium(rho, u)).max() < 1e-15


def test_zero_rates_keep_populations():
    """With every relaxation rate 0 and no force, collision is the identity."""
    f = _rand_state(8)
    fp = O.collide(f, (0, 0, 0), s_nu=0.0, s_b=0.0, s_high=(0, 0, 0, 0))
    assert np.abs(fp - f).max() < 1e-15


def _rotation_perm(R):
    c, _, _, _ = O.lattice()
    rc = c @ R.T
    return np.array([int(np.where((c == v).all(1))[0][0]) for v in rc])


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_collision_commutes_with_lattice_rotations(axis):
    """A 90-degree rotation of the lattice maps populations to populations;
    collision must commute with it (moment basis and rates are isotropic)."""
    R = np.zeros((3, 3))
    a, b = [(1, 2), (2, 0), (0, 1)][axis]
    R[axis, axis] = 1
    R[a, b] = -1
    R[b, a] = 1
    perm = _rotation_perm(R)
    f = _rand_state(11)
    F = np.array([2e-3, -1e-3, 5e-4])
    kw = dict(s_nu=1.7, s_b=1.2, s_high=(0.9, 1.1, 1.3, 0.8))
    fp = O.collide(f, F, **kw)
    fr = np.empty(27)
    fr[perm] = f        # population i moves to the rotated velocity
    fpr = O.collide(fr, R @ F, **kw)
    assert np.abs(fpr[perm] - fp).max() < 1e-14


def test_shear_rate_sets_viscous_stress_decay():
    """Order-2 deviatoric central moments relax with factor (1 - s_nu), the
    trace with (1 - s_b) toward rho (no force)."""
    c, _, _, e = O.lattice()
    f = _rand_state(13)
    rho = f.sum()
    u = (c.T @ f) / rho
    s_nu, s_b = 1.6, 0.7
    fp = O.collide(f, (0, 0, 0), s_nu=s_nu, s_b=s_b, s_high=(1, 1, 1, 1))
    T = O.central_matrix(u)
    k0, k1 = T @ f, T @ fp
    idx = {tuple(v): i for i, v in enumerate(e)}
    for ee in [(1, 1, 0), (1, 0, 1), (0, 1, 1)]:
        assert abs(k1[idx[ee]] - (1 - s_nu) * k0[idx[ee]]) < 1e-15
    xx, yy, zz = idx[(2, 0, 0)], idx[(0, 2, 0)], idx[(0, 0, 2)]
    assert abs((k1[xx] - k1[yy]) - (1 - s_nu) * (k0[xx] - k0[yy])) < 1e-15
    tr0, tr1 = k0[xx] + k0[yy] + k0[zz], k1[xx] + k1[yy] + k1[zz]
    assert abs(tr1 - (tr0 - s_b * (tr0 - rho))) < 1e-15


def test_high_order_rates_per_order():
    """Orders 3..6 relax by (1 - s_n) toward the Maxwellian value, one rate per
    order (no force)."""
    c, _, _, e = O.lattice()
    f = _rand_state(17)
    rho = f.sum()
    u = (c.T @ f) / rho
    sh = (0.6, 1.3, 0.8, 1.7)
    fp = O.collide(f, (0, 0, 0), s_nu=1.0, s_b=1.0, s_high=sh)
    T = O.central_matrix(u)
    k0, k1 = T @ f, T @ fp
    for k, ee in enumerate(e):
        n = ee.sum()
        if n < 3:
            continue
        keq = 0.0 if (ee == 1).any() else rho * (1 / 3) ** (n // 2)
        s = sh[n - 3]
        assert abs(k1[k] - ((1 - s) * k0[k] + s * keq)) < 1e-15, ee


def test_force_term_is_velocity_derivative_of_equilibrium():
    """With all rates 0 the step adds only the forcing term, which must equal
    the discrete form of F.(xi - u)/cs^2 f_M/rho = (F/rho) . d f_eq/du at the
    half-force velocity u = (j + F/2)/rho (closed form; derivative taken by a
    central difference of the product-form equilibrium)."""
    c, _, _, _ = O.lattice()
    f = _rand_state(19)
    F = np.array([3e-3, -2e-3, 1e-3])
    rho = f.sum()
    u = (c.T @ f + 0.5 * F) / rho
    fp = O.collide(f, F, s_nu=0.0, s_b=0.0, s_high=(0, 0, 0, 0))
    h = 1e-5
    dfeq = np.zeros(27)
    for a in range(3):
        du = np.zeros(3)
        du[a] = h
        dfeq += F[a] / rho * (O.equilibrium(rho, u + du) - O.equilibrium(rho, u - du)) / (2 * h)
    assert np.abs((fp - f) - dfeq).max() < 1e-12
