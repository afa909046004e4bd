"""Shared helpers of the GPU parity tests: run the same seeded case through the
HIP library (C-ABI via the binding) and through the FP64 oracle."""
from __future__ import annotations

import sys

import numpy as np

from oracle import oracle as O

P, NS, FS, IN, OUT = 0, 1, 2, 3, 4


def say(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def rel_l2_dev(a, b, ref=1.0) -> float:
    """Stricter density diagnostic: ||a - b|| / ||b - ref||."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm((b - ref).ravel()), 1e-300))


def random_populations(shape, seed, amp=0.05, drift=(0.02, -0.01, 0.015)):
    """Populations w_i (1 + amp xi) plus a small drift along c_i: an arbitrary
    near-rest state (input data only)."""
    c, w, _, _ = O.lattice()
    rng = np.random.default_rng(seed)
    f = w[:, None, None, None] * (1.0 + amp * rng.standard_normal((27,) + tuple(shape)))
    f += 3.0 * w[:, None, None, None] * (c @ np.asarray(drift))[:, None, None, None]
    return f


def gpu_solver(nx, ny, nz, nu, storage="f32", **kw):
    from paper_2101_11856_amd import lbm
    return lbm.Solver(nx, ny, nz, nu, storage=storage, **kw)


def to_np(t):
    return t.detach().to("cpu").double().numpy()


def smooth_fields(nx, ny, nz):
    """Non-trivial smooth initial fields (float32, separable products), so that
    the first step changes every node: rho = 1 + 1e-3 a, u = (0.05 + 0.01 b,
    0.005 c, 0.005 d), scalar in [0, 1]."""
    X = np.arange(nx, dtype=np.float32)
    Y = np.arange(ny, dtype=np.float32)
    Z = np.arange(nz, dtype=np.float32)
    two_pi = np.float32(2 * np.pi)

    def sep(fx, fy, fz):
        return (fz[:, None, None] * fy[None, :, None]) * fx[None, None, :]

    sx, cy, sz = np.sin(two_pi * 3 * X / nx), np.cos(two_pi * 2 * Y / ny), np.sin(two_pi * 5 * Z / nz)
    cx, sy, cz = np.cos(two_pi * 4 * X / nx), np.sin(two_pi * 3 * Y / ny), np.cos(two_pi * 2 * Z / nz)
    rho = np.float32(1) + np.float32(1e-3) * sep(sx, sy, cz)
    u = np.empty((3, nz, ny, nx), np.float32)
    u[0] = np.float32(0.05) + np.float32(0.01) * sep(cx, cy, sz)
    u[1] = np.float32(0.005) * sep(sx, cy, cz)
    u[2] = np.float32(0.005) * sep(cx, sy, sz)
    sc = np.float32(0.5) + np.float32(0.5) * sep(sx, cy, cz)
    return rho, u, sc
