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
