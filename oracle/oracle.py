"""ctypes wrapper of the FP64 CPU oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product package never imports it.

The oracle follows the paper's Sec. 3 (Eqs. 1-5, collision and streaming),
Sec. 3.1 (Eqs. 6-8, immersed boundary), Alg. 1 (bounce-back) and Alg. 2 (step
order); see the header of ``lbm_oracle.c`` for the readings it takes where the
paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")

PERIODIC, NOSLIP, FREESLIP, INLET, OUTFLOW = 0, 1, 2, 3, 4


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP, IEEE FP64, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # LBM_ORACLE_LIBRARY: a deliberately broken copy, for the mutation test
        # of the pins (tests/test_oracle_mutants.py); never set otherwise
        alt = os.environ.get("LBM_ORACLE_LIBRARY")
        if alt:
            L = C.CDLL(alt)
        else:
            build()
            L = C.CDLL(LIB)
        dp, ip, fp = C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_float)
        vp = C.c_void_p
        L.orc_lattice.argtypes = [ip, dp, ip, ip]
        L.orc_central_matrix.argtypes = [dp, dp]
        L.orc_combination_matrix.argtypes = [dp]
        L.orc_basis_matrix.argtypes = [dp, dp]
        L.orc_inverse.argtypes = [dp, dp, C.c_int]
        L.orc_inverse.restype = C.c_int
        L.orc_equilibrium.argtypes = [C.c_double, dp, dp]
        L.orc_collide.argtypes = [dp, dp, C.c_double, C.c_double, dp, dp]
        L.orc_collide.restype = C.c_int
        L.orc_collide_bgk.argtypes = [dp, dp, C.c_double, dp]
        L.orc_collide_bgk.restype = C.c_int
        L.orc_collide_rm.argtypes = [dp, dp, C.c_double, C.c_double, dp, dp]
        L.orc_collide_rm.restype = C.c_int
        L.orc_forcing_shape.argtypes = [dp, dp, dp]
        L.orc_set_model.argtypes = [vp, C.c_int]
        L.orc_set_model.restype = C.c_int
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, ip, dp, C.c_double, dp, dp, C.c_int]
        L.orc_create.restype = vp
        L.orc_destroy.argtypes = [vp]
        L.orc_num_cells.argtypes = [vp]
        L.orc_num_cells.restype = C.c_int64
        L.orc_set_state.argtypes = [vp, dp]
        L.orc_get_state.argtypes = [vp, dp]
        L.orc_set_inlet_profile.argtypes = [vp, dp]
        L.orc_init_equilibrium.argtypes = [vp, dp, dp]
        L.orc_check_markers.argtypes = [vp, C.c_int64, fp]
        L.orc_check_markers.restype = C.c_int64
        L.orc_set_markers.argtypes = [vp, C.c_int64, fp, dp, dp, dp]
        L.orc_set_markers.restype = C.c_int
        L.orc_step.argtypes = [vp, C.c_int]
        L.orc_step.restype = C.c_int
        L.orc_macros.argtypes = [vp, dp, dp]
        L.orc_last_force.argtypes = [vp, dp]
        L.orc_ib_force.argtypes = [vp, dp, dp]
        L.orc_last_torque.argtypes = [vp, dp, dp]
        L.orc_get_force_field.argtypes = [vp, dp]
        L.orc_conserved.argtypes = [vp, dp]
        L.orc_marker_key.argtypes = [vp, fp]
        L.orc_marker_key.restype = C.c_uint64
        L.orc_maps.argtypes = [vp, C.POINTER(C.c_uint8), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.orc_set_scalar.argtypes = [vp, dp, C.c_int]
        L.orc_get_scalar.argtypes = [vp, dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_stream.argtypes = [vp, dp]
        L.orc_ib_interp.argtypes = [vp, dp, dp, dp]
        L.orc_ib_spread.argtypes = [vp, dp, dp]
        _lib = L
    return _lib


def _p(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# --------------------------------------------------------------------------
# single-cell and matrix helpers
# --------------------------------------------------------------------------

def lattice():
    """(c[27,3], w[27], opp[27], moment exponents[27,3])."""
    c = np.zeros((27, 3), np.int32)
    w = np.zeros(27)
    opp = np.zeros(27, np.int32)
    e = np.zeros((27, 3), np.int32)
    lib().orc_lattice(_p(c, C.c_int), _p(w, C.c_double), _p(opp, C.c_int), _p(e, C.c_int))
    return c, w, opp, e


def central_matrix(u) -> np.ndarray:
    T = np.zeros((27, 27))
    lib().orc_central_matrix(_p(_d(u), C.c_double), _p(T, C.c_double))
    return T


def combination_matrix() -> np.ndarray:
    Cm = np.zeros((27, 27))
    lib().orc_combination_matrix(_p(Cm, C.c_double))
    return Cm


def basis_matrix(u) -> np.ndarray:
    M = np.zeros((27, 27))
    lib().orc_basis_matrix(_p(_d(u), C.c_double), _p(M, C.c_double))
    return M


def inverse(A) -> np.ndarray:
    A = _d(A)
    n = A.shape[0]
    R = np.zeros_like(A)
    rc = lib().orc_inverse(_p(A, C.c_double), _p(R, C.c_double), n)
    if rc != 0:
        raise np.linalg.LinAlgError("singular")
    return R


def equilibrium(rho, u) -> np.ndarray:
    out = np.zeros(27)
    lib().orc_equilibrium(float(rho), _p(_d(u), C.c_double), _p(out, C.c_double))
    return out


def collide(fs, F=(0.0, 0.0, 0.0), s_nu=1.0, s_b=1.0, s_high=(1.0, 1.0, 1.0, 1.0)) -> np.ndarray:
    out = np.zeros(27)
    rc = lib().orc_collide(
        _p(_d(fs), C.c_double), _p(_d(F), C.c_double), float(s_nu), float(s_b),
        _p(_d(s_high), C.c_double), _p(out, C.c_double)
    )
    if rc != 0:
        raise np.linalg.LinAlgError("singular moment matrix")
    return out


def collide_bgk(fs, F=(0.0, 0.0, 0.0), omega=1.0) -> np.ndarray:
    """Lattice BGK with the product-form equilibrium and Guo forcing (the
    paper's Sec. 5.1 comparison model; reading: same equilibrium and forcing as
    the central-moment model)."""
    out = np.zeros(27)
    lib().orc_collide_bgk(_p(_d(fs), C.c_double), _p(_d(F), C.c_double), float(omega), _p(out, C.c_double))
    return out


def collide_rm(fs, F=(0.0, 0.0, 0.0), s_nu=1.0, s_b=1.0, s_high=(1.0, 1.0, 1.0, 1.0)) -> np.ndarray:
    """Raw-moment MRT: the same combination basis and rates, moments taken
    about zero velocity (the paper's Sec. 5.1 comparison model)."""
    out = np.zeros(27)
    rc = lib().orc_collide_rm(_p(_d(fs), C.c_double), _p(_d(F), C.c_double), float(s_nu), float(s_b),
                              _p(_d(s_high), C.c_double), _p(out, C.c_double))
    if rc != 0:
        raise np.linalg.LinAlgError("singular moment matrix")
    return out


def forcing_shape(u, F) -> np.ndarray:
    """G_i = sum_a F_a d Phi_i / d u_a of the product-form equilibrium Phi."""
    out = np.zeros(27)
    lib().orc_forcing_shape(_p(_d(u), C.c_double), _p(_d(F), C.c_double), _p(out, C.c_double))
    return out


MODELS = {"cm": 0, "bgk": 1, "rm": 2}


def rigid_pose(X, ub, R, o, v, w):
    """Sample update of Alg. 2 (c) for a rigid body in prescribed motion.

    The paper moves its solids (rotating torus, moving airplane) without giving
    a kinematics rule; the reading taken here is rigid motion.  Body samples
    X_s [3, n] with body-frame boundary velocity ub_s [3, n] are placed at
    x_s = o + R X_s and move with u_b = R ub_s + v + w x (x_s - o).

    x_s is formed in FP64 as o_a + ((R_a0 X + R_a1 Y) + R_a2 Z), one rounding
    per operation, then rounded to FP32 (the precision in which the base cell
    floor(x_s) is taken); the lever arm x_s - o uses that FP32 position, and
    (R ub)_a is summed in the same order.
    Returns (xyz float32 [3, n], ub float64 [3, n]).
    """
    X = np.asarray(X, dtype=np.float64).reshape(3, -1)
    ub = np.zeros_like(X) if ub is None else np.asarray(ub, dtype=np.float64).reshape(3, -1)
    R = np.asarray(R, dtype=np.float64).reshape(3, 3)
    o, v, w = (np.asarray(a, dtype=np.float64).reshape(3) for a in (o, v, w))
    xyz = np.empty(X.shape, dtype=np.float32)
    for a in range(3):
        xyz[a] = (o[a] + ((R[a, 0] * X[0] + R[a, 1] * X[1]) + R[a, 2] * X[2])).astype(np.float32)
    r = xyz.astype(np.float64) - o[:, None]
    rot_ub = np.array([(R[a, 0] * ub[0] + R[a, 1] * ub[1]) + R[a, 2] * ub[2] for a in range(3)])
    ub_w = np.empty_like(X)
    ub_w[0] = rot_ub[0] + v[0] + (w[1] * r[2] - w[2] * r[1])
    ub_w[1] = rot_ub[1] + v[1] + (w[2] * r[0] - w[0] * r[2])
    ub_w[2] = rot_ub[2] + v[2] + (w[0] * r[1] - w[1] * r[0])
    return xyz, ub_w


def num_threads() -> int:
    return int(lib().orc_num_threads())


# --------------------------------------------------------------------------
# whole-domain simulation
# --------------------------------------------------------------------------

class OracleSim:
    """FP64 reference simulation on an nx x ny x nz grid.

    Arrays follow the library's conventions: a scalar field is [nz, ny, nx]
    (x fastest), a vector field [3, nz, ny, nx], populations [27, nz, ny, nx].
    ``faces`` is (-x, +x, -y, +y, -z, +z) with PERIODIC/NOSLIP/FREESLIP/INLET/
    OUTFLOW codes.
    """

    def __init__(self, nx, ny, nz, nu, faces=(0,) * 6, u_in=(0.0, 0.0, 0.0), s_bulk=1.0,
                 s_high=(1.0, 1.0, 1.0, 1.0), body=(0.0, 0.0, 0.0), scalar=False, model="cm"):
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        fc = np.ascontiguousarray(np.asarray(faces, dtype=np.int32))
        self._h = lib().orc_create(nx, ny, nz, float(nu), _p(fc, C.c_int), _p(_d(u_in), C.c_double),
                                   float(s_bulk), _p(_d(s_high), C.c_double), _p(_d(body), C.c_double),
                                   1 if scalar else 0)
        if not self._h:
            raise ValueError("invalid oracle parameters")
        if lib().orc_set_model(self._h, MODELS[model] if isinstance(model, str) else int(model)) != 0:
            raise ValueError(f"unknown collision model {model!r}")
        self.n_markers = 0

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # state ------------------------------------------------------------
    def init_equilibrium(self, rho, u):
        lib().orc_init_equilibrium(self._h, _p(_d(rho).ravel(), C.c_double), _p(_d(u).ravel(), C.c_double))

    def set_state(self, f):
        f = _d(f).reshape(27, self.N)
        lib().orc_set_state(self._h, _p(f, C.c_double))

    def get_state(self) -> np.ndarray:
        f = np.zeros((27,) + self.shape)
        lib().orc_get_state(self._h, _p(f, C.c_double))
        return f

    def set_inlet_profile(self, prof):
        if prof is None:
            lib().orc_set_inlet_profile(self._h, None)
        else:
            lib().orc_set_inlet_profile(self._h, _p(_d(prof).ravel(), C.c_double))

    def set_markers(self, xyz, ub=None, area=None, gain=None):
        xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32))
        n = xyz.shape[1]
        ub = None if ub is None else _d(ub)
        area = None if area is None else _d(area)
        gain = None if gain is None else _d(gain)
        rc = lib().orc_set_markers(
            self._h, n, _p(xyz, C.c_float),
            None if ub is None else _p(ub, C.c_double),
            None if area is None else _p(area, C.c_double),
            None if gain is None else _p(gain, C.c_double))
        if rc != 0:
            raise ValueError("marker outside the domain")
        self.n_markers = n
        self._xyz = xyz

    def step(self, n=1):
        if lib().orc_step(self._h, int(n)) != 0:
            raise FloatingPointError("singular moment matrix (non-finite state)")

    def macros(self):
        rho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        lib().orc_macros(self._h, _p(rho, C.c_double), _p(u, C.c_double))
        return rho, u

    def last_force(self):
        out = np.zeros(3)
        lib().orc_last_force(self._h, _p(out, C.c_double))
        return out

    def ib_force(self, per_marker=False):
        out = np.zeros(3)
        gs = np.zeros((3, max(self.n_markers, 1)))
        lib().orc_ib_force(self._h, _p(out, C.c_double), _p(gs, C.c_double) if per_marker else None)
        return (out, gs[:, : self.n_markers]) if per_marker else out

    def last_torque(self, origin=(0.0, 0.0, 0.0)):
        """Torque sum_s (x_s - o) x (a_s g_s) of the penalty forces last computed (Alg. 2 (c))."""
        out = np.zeros(3)
        lib().orc_last_torque(self._h, _p(_d(origin), C.c_double), _p(out, C.c_double))
        return out

    def force_field(self):
        g = np.zeros((3,) + self.shape)
        lib().orc_get_force_field(self._h, _p(g, C.c_double))
        return g

    def conserved(self):
        out = np.zeros(4)
        lib().orc_conserved(self._h, _p(out, C.c_double))
        return out

    def maps(self):
        n = self.n_markers
        flags = np.zeros(self.shape, np.uint8)
        cell = np.zeros(max(n, 1), np.int32)
        perm = np.zeros(max(n, 1), np.int32)
        lib().orc_maps(self._h, _p(flags, C.c_uint8), _p(cell, C.c_int32), _p(perm, C.c_int32))
        return flags, cell[:n], perm[:n]

    def marker_key(self, p) -> int:
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        return int(lib().orc_marker_key(self._h, _p(p, C.c_float)))

    def stream(self) -> np.ndarray:
        out = np.zeros((27,) + self.shape)
        lib().orc_stream(self._h, _p(out, C.c_double))
        return out

    def ib_interp(self, rho, u) -> np.ndarray:
        G = np.zeros((3, max(self.n_markers, 1)))
        lib().orc_ib_interp(self._h, _p(_d(rho).ravel(), C.c_double), _p(_d(u).ravel(), C.c_double),
                            _p(G, C.c_double))
        return G[:, : self.n_markers]

    def ib_spread(self, G) -> np.ndarray:
        g = np.zeros((3,) + self.shape)
        Gd = _d(G).reshape(3, -1) if self.n_markers else np.zeros((3, 1))
        lib().orc_ib_spread(self._h, _p(np.ascontiguousarray(Gd), C.c_double), _p(g, C.c_double))
        return g

    def set_scalar(self, s, inlet_height):
        lib().orc_set_scalar(self._h, _p(_d(s).ravel(), C.c_double), int(inlet_height))

    def get_scalar(self):
        s = np.zeros(self.shape)
        lib().orc_get_scalar(self._h, _p(s, C.c_double))
        return s
