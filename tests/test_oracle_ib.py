"""Pins of the oracle's immersed boundary (Sec. 3.1 Eqs. 6-8; Sec. 4.3.2
scattering vs gathering; Table 1) and solid-sample maps (Sec. 4.2.2)."""
import numpy as np
import pytest

from oracle import oracle as O

P, NS = O.PERIODIC, O.NOSLIP


def _markers(n, shape, seed, margin=0.0):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    hi = np.array([nx, ny, nz], dtype=np.float64)[:, None] - margin
    return (margin + (hi - margin) * rng.random((3, n))).astype(np.float32)


def test_interpolation_reproduces_linear_fields():
    """Trilinear 2x2x2 kernel: weights sum to 1 (rho_s = 1 for rho = 1) and a
    linear velocity field is interpolated exactly (Eq. 6).  With u_b = 0 and
    gain 1 the penalty force is -u(x_s) (Eq. 7)."""
    nx, ny, nz = 9, 8, 7
    S = O.OracleSim(nx, ny, nz, 0.1)
    xyz = _markers(40, (nz, ny, nx), 5, margin=0.0)
    xyz = np.minimum(xyz, np.array([nx - 1.01, ny - 1.01, nz - 1.01], np.float32)[:, None])
    S.set_markers(xyz)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    A = np.array([[0.01, -0.02, 0.005], [0.003, 0.01, -0.007], [-0.004, 0.002, 0.008]])
    b = np.array([0.02, -0.01, 0.03])
    u = np.stack([A[a, 0] * x + A[a, 1] * y + A[a, 2] * z + b[a] for a in range(3)])
    G = S.ib_interp(np.ones((nz, ny, nx)), u)
    p = xyz.astype(np.float64)
    ref = A @ p + b[:, None]
    assert np.abs(-G - ref).max() < 1e-15


def test_spreading_conserves_total_force_and_is_interp_transpose():
    """sum_f g(x_f) = sum_s a_s g_s (weights sum to 1), and with a_s = 1
    <Spread G, v> = <G, Interp v> (Eq. 8 uses the same kernel as Eq. 6)."""
    nx, ny, nz = 7, 6, 5
    S = O.OracleSim(nx, ny, nz, 0.1)
    xyz = _markers(60, (nz, ny, nx), 6)
    S.set_markers(xyz)                   # periodic: stencils wrap
    rng = np.random.default_rng(7)
    G = rng.standard_normal((3, 60))
    g = S.ib_spread(G)
    assert np.abs(g.reshape(3, -1).sum(1) - G.sum(1)).max() < 1e-13
    v = rng.standard_normal((3, nz, ny, nx))
    Iv = S.ib_interp(np.ones((nz, ny, nx)), -v)   # u_b = 0, gain 1: G = Interp(v)
    assert abs((g * v).sum() - (G * Iv).sum()) < 1e-12


def test_gathering_equals_scattering_brute_force():
    """The oracle spreads in 'gathering' form (per fluid node, Eq. 8 as
    written); per-sample 'scattering' (Sec. 4.3.2) computed here by brute
    force in numpy must give the same field."""
    nx, ny, nz = 6, 5, 7
    S = O.OracleSim(nx, ny, nz, 0.1)
    n = 35
    xyz = _markers(n, (nz, ny, nx), 8)
    rng = np.random.default_rng(9)
    area = rng.random(n) + 0.5
    S.set_markers(xyz, area=area)
    G = rng.standard_normal((3, n))
    g = S.ib_spread(G)
    ref = np.zeros((3, nz, ny, nx))
    for s in range(n):
        p = xyz[:, s].astype(np.float64)
        b = np.floor(xyz[:, s]).astype(int)
        t = p - b
        for d in np.ndindex(2, 2, 2):
            K = np.prod([t[a] if d[a] else 1 - t[a] for a in range(3)])
            q = [(b[a] + d[a]) % [nx, ny, nz][a] for a in range(3)]
            ref[:, q[2], q[1], q[0]] += area[s] * K * G[:, s]
    assert np.abs(g - ref).max() < 1e-14


def test_hand_computed_spread():
    """4x4x4, marker at (1.25, 2.5, 0.0), area 2, g_s = (1, 0, 0):
    weights 0.75/0.25 in x, 0.5/0.5 in y, 1/0 in z."""
    S = O.OracleSim(4, 4, 4, 0.1)
    S.set_markers(np.array([[1.25], [2.5], [0.0]], np.float32), area=np.array([2.0]))
    g = S.ib_spread(np.array([[1.0], [0.0], [0.0]]))
    exp = {(1, 2, 0): 0.75, (2, 2, 0): 0.25, (1, 3, 0): 0.75, (2, 3, 0): 0.25}
    for (x, y, z), v in exp.items():
        assert g[0, z, y, x] == v
    assert abs(g[0].sum() - 2.0) < 1e-15 and np.count_nonzero(g[0]) == 4


def test_step_force_and_momentum_budget():
    """One step on a periodic domain with samples: the spread field sums to
    the recorded total force, and the domain momentum rises by exactly that
    total (conservative LBE + forcing)."""
    nx, ny, nz = 8, 7, 6
    rng = np.random.default_rng(10)
    S = O.OracleSim(nx, ny, nz, 0.05)
    rho = 1.0 + 0.01 * rng.standard_normal((nz, ny, nx))
    u = 0.02 * rng.standard_normal((3, nz, ny, nx))
    S.init_equilibrium(rho, u)
    xyz = _markers(25, (nz, ny, nx), 11)
    ub = 0.01 * rng.standard_normal((3, 25))
    S.set_markers(xyz, ub=ub, area=rng.random(25), gain=0.5 + rng.random(25))
    c0 = S.conserved()
    S.step(1)
    F = S.last_force()
    assert np.abs(S.force_field().reshape(3, -1).sum(1) - F).max() < 1e-14
    c1 = S.conserved()
    assert np.abs(c1[1:] - c0[1:] - F).max() < 1e-14
    assert abs(c1[0] - c0[0]) < 1e-12


def test_markers_outside_domain_rejected():
    S = O.OracleSim(4, 4, 4, 0.1, faces=(P, P, NS, NS, P, P))
    with pytest.raises(ValueError):
        S.set_markers(np.array([[1.0], [3.2], [1.0]], np.float32))   # stencil crosses a wall
    with pytest.raises(ValueError):
        S.set_markers(np.array([[4.0], [1.0], [1.0]], np.float32))   # outside periodic extent
    S.set_markers(np.array([[3.9], [2.9], [3.99]], np.float32))


def _brute_maps(shape, xyz, ell=4):
    """Independent recomputation of the sample maps: base cell by floor,
    band flags over each 2x2x2 stencil, and the order (l^3 block in x-y-z
    order, then Z-order of the position quantised to 1024 steps per axis
    inside the block, then the original index)."""
    nz, ny, nx = shape
    n = xyz.shape[1]
    nb = [(nx + ell - 1) // ell, (ny + ell - 1) // ell, (nz + ell - 1) // ell]
    flags = np.zeros(shape, np.uint8)
    cell = np.zeros(n, np.int32)
    keys = []
    for s in range(n):
        p = xyz[:, s]
        b = [int(np.floor(p[a])) for a in range(3)]
        cell[s] = b[0] + nx * (b[1] + ny * b[2])
        for d in np.ndindex(2, 2, 2):
            q = [(b[a] + d[a]) % [nx, ny, nz][a] for a in range(3)]
            flags[q[2], q[1], q[0]] |= 1
        flags[b[2], b[1], b[0]] |= 2
        B = [b[a] // ell for a in range(3)]
        q = [int(np.floor((np.float32(p[a]) - np.float32(ell * B[a])) * np.float32(1024 // ell)))
             for a in range(3)]
        m = 0
        for bit in range(10):
            for a in range(3):
                m |= ((q[a] >> bit) & 1) << (3 * bit + a)
        block = B[0] + nb[0] * (B[1] + nb[1] * B[2])
        keys.append((block, m, s))
    perm = np.array([k[2] for k in sorted(keys)], np.int32)
    return flags, cell, perm


def test_maps_match_brute_force():
    shape = (9, 10, 13)   # ragged against the 4^3 blocks
    rng = np.random.default_rng(12)
    xyz = _markers(300, shape, 13)
    # many samples in one cell and exact node positions
    xyz[:, :40] = (np.array([[5.5], [3.25], [2.0]]) + 0.4 * rng.random((3, 40))).astype(np.float32)
    xyz[:, 40:45] = np.array([[4.0, 8.0, 0.0, 12.0, 3.0], [0.0, 4.0, 9.0, 1.0, 7.0],
                              [8.0, 0.0, 4.0, 3.0, 6.0]], np.float32)
    S = O.OracleSim(13, 10, 9, 0.1)
    S.set_markers(xyz)
    f, c, p = S.maps()
    bf, bc, bp = _brute_maps(shape, xyz)
    assert np.array_equal(f, bf) and np.array_equal(c, bc) and np.array_equal(p, bp)
    # samples of one cell are contiguous in the sorted order
    cells = c[p]
    seen = set()
    prev = None
    for v in cells:
        if v != prev:
            assert v not in seen
            seen.add(v)
            prev = v


def test_penalty_force_uses_gain_and_area():
    """Eq. (7) with the sample's gain and Eq. (8)'s area weight, by hand: in a
    uniform state (rho, U) the interpolation of constants is exact, so
    G_s = gamma_s rho (u_b,s - U) and the total force is sum_s a_s G_s."""
    nx, ny, nz = 8, 8, 8
    rho0, U = 1.02, np.array([0.03, -0.01, 0.02])
    S = O.OracleSim(nx, ny, nz, 0.05)
    S.init_equilibrium(np.full((nz, ny, nx), rho0), np.broadcast_to(U[:, None, None, None], (3, nz, ny, nx)).copy())
    xyz = np.array([[2.25, 5.5, 3.75], [3.5, 2.0, 6.25], [4.75, 4.5, 1.5]], np.float32)
    ub = np.array([[0.01, 0.0, -0.02], [0.0, 0.03, 0.01], [0.02, 0.0, 0.0]])
    gain = np.array([0.5, 2.0, 1.5])
    area = np.array([0.3, 1.7, 0.9])
    S.set_markers(xyz, ub=ub, area=area, gain=gain)
    F, G = S.ib_force(per_marker=True)
    G_hand = gain * rho0 * (ub - U[:, None])
    assert np.abs(G - G_hand).max() < 1e-15
    assert np.abs(F - G_hand @ area).max() < 1e-15


def test_sample_order_hand_computed():
    """Sec. 4.2.2 order worked out by hand on a 12x8x8 periodic grid (l = 4,
    so 3 x 2 x 2 blocks, block index Bx + 3 (By + 2 Bz)); positions inside a
    block are quantised to 256 steps per cell (1024 per block edge).
      sample 0 (9.5, 1, 1)      block 2
      sample 1 (1.25, 1, 1)     block 0, q = (320, 256, 256)
      sample 2 (1, 1.25, 1)     block 0, q = (256, 320, 256)
      sample 3 (5, 0.5, 0.5)    block 1
      sample 4 (0.5, 4.5, 0.5)  block 3
      sample 5 = sample 1       same key: the lower index first
      sample 6 (0.5, 0.5, 4.5)  block 6
      sample 7 (3.9, 3.9, 3.9)  block 0, q = (998, 998, 998): bit 9 set, last
    Inside block 0, samples 1 and 2 first differ at bit 6 of q (320 = 256 +
    64): x's bit lands at Morton position 18, y's at 19, so 1 < 2.  Sorted:
    blocks 0 (1, 5, 2, 7), 1 (3), 2 (0), 3 (4), 6 (6)."""
    xyz = np.array([[9.5, 1.25, 1.0, 5.0, 0.5, 1.25, 0.5, 3.9],
                    [1.0, 1.0, 1.25, 0.5, 4.5, 1.0, 0.5, 3.9],
                    [1.0, 1.0, 1.0, 0.5, 0.5, 1.0, 4.5, 3.9]], np.float32)
    S = O.OracleSim(12, 8, 8, 0.1)
    S.set_markers(xyz)
    _, cell, perm = S.maps()
    assert list(perm) == [1, 5, 2, 7, 3, 0, 4, 6]
    # base cells x + 12 (y + 8 z) by hand
    assert list(cell) == [9 + 12 * 9, 1 + 12 * 9, 1 + 12 * 9, 5, 48, 1 + 12 * 9, 384, 3 + 12 * (3 + 8 * 3)]
