"""Seeded synthetic inputs shaped like the paper's scenes.

Flow fields and solid samples only: nothing in this module computes any step
of the lattice Boltzmann method.  Both the GPU library and the CPU oracle are
fed from here, so each side then applies its own equilibrium, streaming,
collision and immersed-boundary arithmetic.

Arrays use the library's layout: scalar fields [nz, ny, nx] (x fastest),
vector fields [3, nz, ny, nx], marker arrays [3, n] (float32 positions in
lattice units, a node sits at integer coordinates).

The paper's scenes (Sec. 5, Table 3) use meshes and smoke that are not
available; these generators stand in for them:
  * Taylor-Green vortex (32^3 parity case),
  * decaying turbulence with an E(k) ~ k^-5/3 spectrum (256^3 throughput case,
    and the same spectrum on a periodic box),
  * a sphere sampled on a Fibonacci lattice plus a box of random samples
    (flow past an immersed sphere, 512x128x128),
  * a field of axis-aligned boxes sampled on walls and roofs (city blocks,
    1200x250x840),
  * a cylinder along z with a modal inlet profile (adjoint channel),
  * a torus in prescribed rigid rotation (the rotating torus of Sec. 5).
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# flow fields
# ---------------------------------------------------------------------------


def taylor_green(n: int, u0: float = 0.05, kind: str = "2d", dtype=np.float64):
    """Taylor-Green vortex on an n^3 periodic grid, nodes at integer x.

    kind="2d": u = u0 (sin kx cos ky, -cos kx sin ky, 0), k = 2 pi / n, an
    exact z-invariant Navier-Stokes solution whose kinetic energy decays as
    exp(-4 nu k^2 t).  kind="3d": u = u0 (sin kx cos ky cos kz,
    -cos kx sin ky cos kz, 0).  Density is 1.
    """
    k = 2.0 * math.pi / n
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    if kind == "2d":
        u = np.stack([u0 * np.sin(k * x) * np.cos(k * y), -u0 * np.cos(k * x) * np.sin(k * y), 0.0 * x])
    else:
        u = np.stack([u0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z),
                      -u0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z), 0.0 * x])
    rho = np.ones((n, n, n))
    return rho.astype(dtype), u.astype(dtype)


def turbulence(n: int, kmin: int = 1, kmax: int = 16, rms: float = 0.04, seed: int = 2101,
               rho_noise: float = 1e-3, rho_seed: int = 2102, dtype=np.float32):
    """Random solenoidal velocity on an n^3 periodic grid with shell energy
    E(k) ~ k^(-5/3) for integer shells round(|k|) in [kmin, kmax].

    Complex Gaussian coefficients are projected perpendicular to k, scaled per
    shell, transformed back (real part), and the field is scaled so that the
    per-component rms sqrt(<|u|^2>/3) equals ``rms``.  Density is
    1 + U(-rho_noise, rho_noise) from its own seed.
    """
    rng = np.random.default_rng(seed)
    kk = np.fft.fftfreq(n, d=1.0 / n)
    KZ, KY, KX = np.meshgrid(kk, kk, kk, indexing="ij")
    kmag = np.sqrt(KX * KX + KY * KY + KZ * KZ)
    shell = np.rint(kmag).astype(np.int64)
    active = (shell >= kmin) & (shell <= kmax)
    counts = np.bincount(shell[active], minlength=kmax + 1).astype(np.float64)
    amp = np.zeros_like(kmag)
    s_act = shell[active]
    amp[active] = np.sqrt(s_act.astype(np.float64) ** (-5.0 / 3.0) / counts[s_act])
    kn = np.where(kmag > 0, kmag, 1.0)
    khat = (KX / kn, KY / kn, KZ / kn)
    c = [(rng.standard_normal(kmag.shape) + 1j * rng.standard_normal(kmag.shape)) for _ in range(3)]
    kdotc = khat[0] * c[0] + khat[1] * c[1] + khat[2] * c[2]
    u = np.empty((3, n, n, n), dtype=np.float64)
    for a in range(3):
        ca = (c[a] - khat[a] * kdotc) * amp
        u[a] = np.real(np.fft.ifftn(ca))
    del c, kdotc
    u -= u.mean(axis=(1, 2, 3), keepdims=True)
    cur = math.sqrt(float(np.mean(np.sum(u * u, axis=0))) / 3.0)
    u *= rms / cur
    rng_r = np.random.default_rng(rho_seed)
    rho = 1.0 + rng_r.uniform(-rho_noise, rho_noise, size=(n, n, n))
    return rho.astype(dtype), u.astype(dtype)


def turbulence_box(nx: int, ny: int, nz: int, kmin: int = 1, kmax: int = 16, rms: float = 0.04,
                   seed: int = 2101, rho_noise: float = 1e-3, rho_seed: int = 2102, dtype=np.float32):
    """The spectrum of ``turbulence`` on a periodic nx x ny x nz box.

    Wave numbers are counted in units of 2 pi / L with L the longest edge, so
    mode m along an axis of n_a nodes has k = m L / n_a; shells round(|k|) in
    [kmin, kmax] get E(k) ~ k^(-5/3) as in the cubic generator, and the field
    stays periodic on the box.  Same projection, scaling and density noise.
    """
    L = max(nx, ny, nz)
    rng = np.random.default_rng(seed)
    kx = np.fft.fftfreq(nx, d=1.0 / nx) * (L / nx)
    ky = np.fft.fftfreq(ny, d=1.0 / ny) * (L / ny)
    kz = np.fft.fftfreq(nz, d=1.0 / nz) * (L / nz)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    kmag = np.sqrt(KX * KX + KY * KY + KZ * KZ)
    shell = np.rint(kmag).astype(np.int64)
    active = (shell >= kmin) & (shell <= kmax)
    counts = np.bincount(shell[active], minlength=kmax + 1).astype(np.float64)
    amp = np.zeros_like(kmag)
    s_act = shell[active]
    amp[active] = np.sqrt(s_act.astype(np.float64) ** (-5.0 / 3.0) / counts[s_act])
    kn = np.where(kmag > 0, kmag, 1.0)
    khat = (KX / kn, KY / kn, KZ / kn)
    c = [(rng.standard_normal(kmag.shape) + 1j * rng.standard_normal(kmag.shape)) for _ in range(3)]
    kdotc = khat[0] * c[0] + khat[1] * c[1] + khat[2] * c[2]
    u = np.empty((3, nz, ny, nx), dtype=np.float64)
    for a in range(3):
        u[a] = np.real(np.fft.ifftn((c[a] - khat[a] * kdotc) * amp))
    u -= u.mean(axis=(1, 2, 3), keepdims=True)
    u *= rms / math.sqrt(float(np.mean(np.sum(u * u, axis=0))) / 3.0)
    rho = 1.0 + np.random.default_rng(rho_seed).uniform(-rho_noise, rho_noise, size=(nz, ny, nx))
    return rho.astype(dtype), u.astype(dtype)


def uniform(nx, ny, nz, u=(0.0, 0.0, 0.0), rho=1.0, dtype=np.float32):
    r = np.full((nz, ny, nx), rho, dtype=dtype)
    v = np.empty((3, nz, ny, nx), dtype=dtype)
    for a in range(3):
        v[a] = u[a]
    return r, v


# ---------------------------------------------------------------------------
# solid samples
# ---------------------------------------------------------------------------


def fibonacci_sphere(n: int, radius: float, center) -> np.ndarray:
    """n samples on a sphere: z_i = 1 - (2i+1)/n, phi_i = i pi (3 - sqrt 5)."""
    i = np.arange(n, dtype=np.float64)
    zc = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - zc * zc))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    p = np.stack([r * np.cos(phi), r * np.sin(phi), zc]) * radius
    p += np.asarray(center, dtype=np.float64)[:, None]
    return p.astype(np.float32)


def torus_body(major: float, minor: float, per_length: float = 3.0):
    """Body-frame samples of a torus about the z axis, centred on the origin:
    rings of the tube at n_t = round(2 pi major k) angles theta, each with
    n_p = round(2 pi minor k) samples (k = per_length), every other ring
    turned by half a step.  Area weight of a sample: the surface element
    minor (major + minor cos phi) dtheta dphi, so the weights sum to the
    torus area 4 pi^2 major minor.  Returns (xyz float32 [3, n], area float32 [n])."""
    nt = max(3, int(round(2.0 * math.pi * major * per_length)))
    nph = max(3, int(round(2.0 * math.pi * minor * per_length)))
    dt, dp = 2.0 * math.pi / nt, 2.0 * math.pi / nph
    th = np.repeat(np.arange(nt) * dt, nph)
    ph = (np.tile(np.arange(nph), nt) + 0.5 * (np.repeat(np.arange(nt), nph) % 2)) * dp
    ring = major + minor * np.cos(ph)
    xyz = np.stack([ring * np.cos(th), ring * np.sin(th), minor * np.sin(ph)])
    area = minor * ring * dt * dp
    return xyz.astype(np.float32), area.astype(np.float32)


def rotation(axis, angle: float) -> np.ndarray:
    """Rotation matrix by `angle` (radians, right-handed) about `axis`."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)


def random_box(n: int, lo, hi, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    p = lo[:, None] + (hi - lo)[:, None] * rng.random((3, n))
    return p.astype(np.float32)


def sphere_scene(nx=512, ny=128, nz=128, radius=16.0, center=(128.0, 64.0, 64.0), n_sphere=13000,
                 n_random=200000, box_lo=(284.0, 48.0, 48.0), box_hi=(316.0, 80.0, 80.0), seed=2103):
    """Sphere (Fibonacci lattice, area 4 pi R^2 / n each) plus a box of
    uniform random samples (area = box volume / n each), all at rest."""
    ps = fibonacci_sphere(n_sphere, radius, center)
    pr = random_box(n_random, box_lo, box_hi, seed) if n_random > 0 else np.zeros((3, 0), np.float32)
    xyz = np.concatenate([ps, pr], axis=1)
    vol = float(np.prod(np.asarray(box_hi) - np.asarray(box_lo)))
    area = np.concatenate([
        np.full(n_sphere, 4.0 * math.pi * radius * radius / n_sphere),
        np.full(pr.shape[1], vol / max(n_random, 1)),
    ]).astype(np.float32)
    ub = np.zeros((3, xyz.shape[1]), np.float32)
    gain = np.ones(xyz.shape[1], np.float32)
    return xyz, ub, area, gain


def city_boxes(nx=1200, ny=250, nz=840, n_boxes=400, seed=2104, side=(10.0, 60.0), height=(20.0, 200.0),
               x_range=(150.0, 1000.0)):
    """Axis-aligned boxes standing on the ground y = 0 (y is vertical).

    Footprint sides and heights are log-uniform; boxes lie inside x_range
    and inside z with a 2-cell margin.  Returns an int array [n_boxes, 5] of
    (x0, z0, sx, sz, h).
    """
    rng = np.random.default_rng(seed)
    out = np.zeros((n_boxes, 5), np.int64)
    for b in range(n_boxes):
        sx = int(round(math.exp(rng.uniform(math.log(side[0]), math.log(side[1])))))
        sz = int(round(math.exp(rng.uniform(math.log(side[0]), math.log(side[1])))))
        h = int(round(math.exp(rng.uniform(math.log(height[0]), math.log(height[1])))))
        h = min(h, ny - 10)
        x0 = int(rng.integers(int(x_range[0]), int(x_range[1]) - sx))
        z0 = int(rng.integers(2, nz - sz - 2))
        out[b] = (x0, z0, sx, sz, h)
    return out


def city_markers(boxes: np.ndarray, spacing: float = 1.0):
    """Samples on the four walls and the roof of each box at ``spacing``,
    at half-integer coordinates (cell centres of the surface grid)."""
    pts = []
    for (x0, z0, sx, sz, h) in boxes:
        xs = x0 + 0.5 + np.arange(0, sx, spacing)
        zs = z0 + 0.5 + np.arange(0, sz, spacing)
        ys = 0.5 + np.arange(0, h, spacing)
        # walls at x = x0 and x = x0 + sx
        Y, Z = np.meshgrid(ys, zs, indexing="ij")
        for xw in (x0 + 0.5, x0 + sx - 0.5):
            pts.append(np.stack([np.full(Y.size, xw), Y.ravel(), Z.ravel()]))
        # walls at z = z0 and z = z0 + sz
        X, Y = np.meshgrid(xs, ys, indexing="ij")
        for zw in (z0 + 0.5, z0 + sz - 0.5):
            pts.append(np.stack([X.ravel(), Y.ravel(), np.full(X.size, zw)]))
        # roof
        X, Z = np.meshgrid(xs, zs, indexing="ij")
        pts.append(np.stack([X.ravel(), np.full(X.size, h - 0.5), Z.ravel()]))
    xyz = np.concatenate(pts, axis=1).astype(np.float32)
    n = xyz.shape[1]
    return xyz, np.zeros((3, n), np.float32), np.ones(n, np.float32), np.ones(n, np.float32)


def cylinder_markers(radius=8.0, center=(32.0, 32.0), nz=64, n_around=50):
    """Cylinder along z: n_around samples per z-layer at z = 0.5 .. nz-0.5,
    area = 2 pi R / n_around each."""
    th = 2.0 * math.pi * (np.arange(n_around) + 0.5) / n_around
    zs = 0.5 + np.arange(nz)
    TH, Z = np.meshgrid(th, zs, indexing="ij")
    xyz = np.stack([center[0] + radius * np.cos(TH.ravel()), center[1] + radius * np.sin(TH.ravel()),
                    Z.ravel()]).astype(np.float32)
    n = xyz.shape[1]
    area = np.full(n, 2.0 * math.pi * radius / n_around, np.float32)
    return xyz, np.zeros((3, n), np.float32), area, np.ones(n, np.float32)


def inlet_mode_basis(ny: int, nz: int, pmax: int = 4, qmax: int = 4, length: float = 64.0) -> np.ndarray:
    """Modes phi_pq(y, z) = sin(p pi (y+1/2)/L) sin(q pi (z+1/2)/L),
    p, q = 1..4; returned as [pmax*qmax, nz, ny]."""
    y = np.arange(ny) + 0.5
    z = np.arange(nz) + 0.5
    out = np.zeros((pmax * qmax, nz, ny))
    for p in range(1, pmax + 1):
        for q in range(1, qmax + 1):
            out[(p - 1) * qmax + (q - 1)] = np.outer(np.sin(q * math.pi * z / length),
                                                    np.sin(p * math.pi * y / length))
    return out


def inlet_coefficients(seed: int = 2105, n: int = 16, amp: float = 0.01) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-amp, amp, n)


def inlet_profile(ny: int, nz: int, coeffs, base: float = 0.04, length: float = 64.0) -> np.ndarray:
    """u_x(y, z) = base + sum_pq a_pq phi_pq(y, z); u_y = u_z = 0; [3, nz, ny]."""
    B = inlet_mode_basis(ny, nz, length=length)
    prof = np.zeros((3, nz, ny))
    prof[0] = base + np.tensordot(np.asarray(coeffs, dtype=np.float64), B, axes=1)
    return prof
