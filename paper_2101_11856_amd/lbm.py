"""ctypes binding of liblbm (include/lbm.h).

Argument marshalling only: PyTorch provides device memory and the stream,
every step of the method runs in the library's HIP kernels.  If liblbm.so is
missing this module raises at import time; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(HERE, "liblbm.so")

PERIODIC, NOSLIP, FREESLIP, INLET, OUTFLOW = 0, 1, 2, 3, 4
F32, F16DEV, BF16DEV, F64 = 0, 1, 2, 3
STORAGE = {"f32": F32, "f16": F16DEV, "bf16": BF16DEV, "f64": F64}
CM, BGK, RMMRT = 0, 1, 2
COLLISION = {"cm": CM, "bgk": BGK, "rm": RMMRT}
STATUS = {0: "LBM_OK", 1: "LBM_E_INVAL", 2: "LBM_E_NOMEM", 3: "LBM_E_HIP", 4: "LBM_E_NONFINITE",
          5: "LBM_E_STATE", 6: "LBM_E_UNSUPPORTED"}


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("nu", C.c_double),
        ("face", C.c_int32 * 6),
        ("u_in", C.c_double * 3),
        ("inlet_profile", C.c_void_p),
        ("body_force", C.c_double * 3),
        ("s_bulk", C.c_double),
        ("s_high", C.c_double * 4),
        ("storage", C.c_int32),
        ("passive_scalar", C.c_int32),
        ("scalar_inlet_height", C.c_int32),
        ("collision", C.c_int32),
    ]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2101_11856_amd.build (hipcc, gfx950) first")

_L = C.CDLL(LIB_PATH)
_vp, _i32, _i64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
_pp = C.POINTER(Params)
_SIG = {
    "lbm_default_params": [_pp, _i32, _i32, _i32, C.c_double],
    "lbm_workspace_size": [_pp, C.POINTER(_sz)],
    "lbm_create": [_pp, _vp, _sz, _vp, C.POINTER(_vp)],
    "lbm_set_stream": [_vp, _vp],
    "lbm_init_equilibrium": [_vp, _vp, _vp],
    "lbm_set_populations": [_vp, _vp],
    "lbm_get_populations": [_vp, _vp],
    "lbm_set_scalar": [_vp, _vp],
    "lbm_get_scalar": [_vp, _vp],
    "lbm_solids_ws_size": [_vp, _i64, C.POINTER(_sz)],
    "lbm_set_solids": [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _sz],
    "lbm_step": [_vp, _i32],
    "lbm_macros": [_vp, _vp, _vp],
    "lbm_conserved": [_vp, C.POINTER(C.c_double)],
    "lbm_conserved_static": [_vp, C.POINTER(C.c_double)],
    "lbm_ib_force": [_vp, C.POINTER(C.c_double)],
    "lbm_ib_force_eval": [_vp, C.POINTER(C.c_double)],
    "lbm_ib_torque": [_vp, C.POINTER(C.c_double)],
    "lbm_set_pose": [_vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                     C.POINTER(C.c_double)],
    "lbm_set_body": [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _sz, C.POINTER(C.c_double), C.POINTER(C.c_double),
                     C.POINTER(C.c_double), C.POINTER(C.c_double)],
    "lbm_solid_maps": [_vp, _vp, _vp, _vp],
    "lbm_state_bytes": [_vp, C.POINTER(_sz)],
    "lbm_checkpoint": [_vp, _vp],
    "lbm_restore": [_vp, _vp],
    "lbm_set_gains": [_vp, _vp],
    "lbm_record_tape": [_vp, _i32, _vp],
    "lbm_adjoint_ws_size": [_vp, C.POINTER(_sz)],
    "lbm_adjoint_init": [_vp, _vp, _sz],
    "lbm_adjoint_seed_macros": [_vp, _vp, _vp, _vp],
    "lbm_adjoint_seed_force": [_vp, C.POINTER(C.c_double), _vp, _vp],
    "lbm_adjoint_step": [_vp, _i32, _vp, _vp, _vp],
    "lbm_adjoint_get": [_vp, _vp],
    "lbm_adjoint_set": [_vp, _vp],
}
for _name, _args in _SIG.items():
    _fn = getattr(_L, _name)
    _fn.argtypes = _args
    _fn.restype = C.c_int
_L.lbm_destroy.argtypes = [_vp]
_L.lbm_destroy.restype = None
_L.lbm_last_error.argtypes = [_vp]
_L.lbm_last_error.restype = C.c_char_p
_L.lbm_version.restype = C.c_char_p

lib = _L


def _check(status: int, ctx=None):
    if status != 0:
        raise LbmError(status, _L.lbm_last_error(ctx).decode())


def _pose_args(R, o, v, w):
    def dbl(a, k, what):
        a = np.asarray(a, dtype=np.float64).reshape(-1)
        if a.size != k:
            raise ValueError(f"{what} needs {k} values, got {a.size}")
        return (C.c_double * k)(*a.tolist())
    return dbl(R, 9, "R"), dbl(o, 3, "o"), dbl(v, 3, "v"), dbl(w, 3, "w")


def _ptr(t: torch.Tensor | None):
    """Device pointer of a contiguous GPU tensor (the library dereferences it
    in kernels: a host tensor here would be a GPU memory fault, so it is
    refused)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _need(t: torch.Tensor | None, nbytes: int, what: str, dtype=None):
    """Refuse a caller buffer that is too small (or of the wrong dtype) before
    the library writes or reads past its end."""
    if t is None:
        return
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    if t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{what} too small: {t.numel() * t.element_size()} bytes, need {nbytes}")


def make_params(nx, ny, nz, nu, faces=(PERIODIC,) * 6, u_in=(0.0, 0.0, 0.0), body=(0.0, 0.0, 0.0),
                s_bulk=1.0, s_high=(1.0, 1.0, 1.0, 1.0), storage="f32", scalar=False,
                scalar_inlet_height=0, collision="cm") -> Params:
    p = Params()
    _check(_L.lbm_default_params(C.byref(p), nx, ny, nz, float(nu)))
    for k in range(6):
        p.face[k] = int(faces[k])
    for a in range(3):
        p.u_in[a] = float(u_in[a])
        p.body_force[a] = float(body[a])
    p.s_bulk = float(s_bulk)
    for k in range(4):
        p.s_high[k] = float(s_high[k])
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.passive_scalar = 1 if scalar else 0
    p.scalar_inlet_height = int(scalar_inlet_height)
    p.collision = COLLISION[collision] if isinstance(collision, str) else int(collision)
    return p


def workspace_size(p: Params) -> int:
    n = C.c_size_t()
    _check(_L.lbm_workspace_size(C.byref(p), C.byref(n)))
    return n.value


class Solver:
    """One lattice Boltzmann domain on the current CUDA/HIP device.

    Arrays follow the library layout: scalar fields [nz, ny, nx], vector fields
    [3, nz, ny, nx], populations [27, nz, ny, nx], samples [3, n].  The real
    dtype is float32, or float64 for storage "f64".
    """

    def __init__(self, nx, ny, nz, nu, faces=(PERIODIC,) * 6, u_in=(0.0, 0.0, 0.0), inlet_profile=None,
                 body=(0.0, 0.0, 0.0), s_bulk=1.0, s_high=(1.0, 1.0, 1.0, 1.0), storage="f32", scalar=False,
                 scalar_inlet_height=0, collision="cm", device="cuda", stream=None):
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.device = torch.device(device)
        self.storage = storage
        self.real = torch.float64 if storage == "f64" else torch.float32
        self._p = make_params(nx, ny, nz, nu, faces, u_in, body, s_bulk, s_high, storage, scalar, scalar_inlet_height,
                              collision)
        self._inlet = None
        if inlet_profile is not None:
            self._inlet = self._real(inlet_profile, (3, nz, ny))
            self._p.inlet_profile = self._inlet.data_ptr()
        self.ws = torch.empty(workspace_size(self._p), dtype=torch.uint8, device=self.device)
        if self.ws.data_ptr() % 256:
            raise RuntimeError("workspace allocation is not 256-byte aligned")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(_L.lbm_create(C.byref(self._p), _ptr(self.ws), self.ws.numel(), C.c_void_p(self.stream.cuda_stream),
                             C.byref(h)))
        self._h = h
        self._mws = None
        self.n_markers = 0

    # ------------------------------------------------------------------
    def _real(self, t, shape=None) -> torch.Tensor:
        t = torch.as_tensor(t, device=self.device).to(self.real).contiguous()
        if shape is not None and tuple(t.shape) != tuple(shape):
            t = t.reshape(shape)
        return t

    def close(self):
        if getattr(self, "_h", None):
            _L.lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        """Issue this solver's further work on `stream` (a torch.cuda.Stream).
        Tensors the binding creates or reads are produced on torch's current
        stream: use the solver inside `torch.cuda.stream(stream)`."""
        self.stream = stream
        _check(_L.lbm_set_stream(self._h, C.c_void_p(stream.cuda_stream)), self._h)

    def set_inlet_profile(self, prof):
        """Replace the contents of the inlet profile given at construction."""
        if self._inlet is None:
            raise LbmError(5, "solver was created without an inlet profile")
        self._inlet.copy_(self._real(prof, self._inlet.shape))

    # ------------------------------------------------------------------
    def init_equilibrium(self, rho, u):
        self._rho0 = self._real(rho, self.shape)
        self._u0 = self._real(u, (3,) + self.shape)
        _check(_L.lbm_init_equilibrium(self._h, _ptr(self._rho0), _ptr(self._u0)), self._h)

    def set_populations(self, f):
        self._f0 = self._real(f, (27,) + self.shape)
        _check(_L.lbm_set_populations(self._h, _ptr(self._f0)), self._h)

    def get_populations(self) -> torch.Tensor:
        f = torch.empty((27,) + self.shape, dtype=self.real, device=self.device)
        _check(_L.lbm_get_populations(self._h, _ptr(f)), self._h)
        return f

    def set_scalar(self, s):
        self._s0 = torch.as_tensor(s, device=self.device).to(torch.float32).contiguous().reshape(self.shape)
        _check(_L.lbm_set_scalar(self._h, _ptr(self._s0)), self._h)

    def get_scalar(self) -> torch.Tensor:
        s = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        _check(_L.lbm_get_scalar(self._h, _ptr(s)), self._h)
        return s

    def _samples(self, xyz, ub, area, gain):
        f32 = lambda t: None if t is None else torch.as_tensor(t, device=self.device).to(torch.float32).contiguous()
        xyz, ub, area, gain = f32(xyz), f32(ub), f32(area), f32(gain)
        if xyz is not None and (xyz.dim() != 2 or xyz.shape[0] != 3):
            raise ValueError(f"sample positions must be [3, n], got {tuple(xyz.shape)}")
        n = 0 if xyz is None else int(xyz.shape[1])
        if n == 0:
            return 0, None
        if xyz.shape != (3, n):
            raise ValueError(f"sample positions must be [3, n], got {tuple(xyz.shape)}")
        if ub is None:
            ub = torch.zeros((3, n), dtype=torch.float32, device=self.device)
        _need(ub, 3 * n * 4, "ub ([3, n])")
        _need(area, n * 4, "area ([n])")
        _need(gain, n * 4, "gain ([n])")
        nb = C.c_size_t()
        _check(_L.lbm_solids_ws_size(self._h, n, C.byref(nb)), self._h)
        self._mws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        return n, (_ptr(xyz), _ptr(ub), _ptr(area), _ptr(gain), _ptr(self._mws), self._mws.numel())

    def set_solids(self, xyz, ub=None, area=None, gain=None):
        n, args = self._samples(xyz, ub, area, gain)
        self.n_markers = 0
        if n == 0:
            _check(_L.lbm_set_solids(self._h, 0, None, None, None, None, None, 0), self._h)
            return
        _check(_L.lbm_set_solids(self._h, n, *args), self._h)
        self.n_markers = n

    def set_body(self, X, ub, area, gain, R, o, v=(0.0, 0.0, 0.0), w=(0.0, 0.0, 0.0)):
        """Samples in body coordinates, placed at the pose (R, o, v, w) (see lbm_set_body)."""
        n, args = self._samples(X, ub, area, gain)
        if n == 0:
            raise ValueError("set_body needs at least one sample")
        self.n_markers = 0
        _check(_L.lbm_set_body(self._h, n, *args, *_pose_args(R, o, v, w)), self._h)
        self.n_markers = n

    def set_pose(self, R, o, v=(0.0, 0.0, 0.0), w=(0.0, 0.0, 0.0)):
        """Place the body samples at o + R X (rigid motion, see lbm_set_pose)."""
        _check(_L.lbm_set_pose(self._h, *_pose_args(R, o, v, w)), self._h)

    def ib_torque(self) -> np.ndarray:
        out = (C.c_double * 3)()
        _check(_L.lbm_ib_torque(self._h, out), self._h)
        return np.array(out[:])

    def step(self, n: int = 1):
        _check(_L.lbm_step(self._h, int(n)), self._h)

    def macros(self):
        rho = torch.empty(self.shape, dtype=self.real, device=self.device)
        u = torch.empty((3,) + self.shape, dtype=self.real, device=self.device)
        _check(_L.lbm_macros(self._h, _ptr(rho), _ptr(u)), self._h)
        return rho, u

    def conserved(self) -> np.ndarray:
        out = (C.c_double * 4)()
        _check(_L.lbm_conserved(self._h, out), self._h)
        return np.array(out[:])

    def conserved_static(self) -> np.ndarray:
        """conserved() through lbm_conserved_static (scratch in the library's
        static device array; nothing allocated, calls on one GPU must not overlap)."""
        out = (C.c_double * 4)()
        _check(_L.lbm_conserved_static(self._h, out), self._h)
        return np.array(out[:])

    def ib_force(self) -> np.ndarray:
        out = (C.c_double * 3)()
        _check(_L.lbm_ib_force(self._h, out), self._h)
        return np.array(out[:])

    def ib_force_eval(self) -> np.ndarray:
        out = (C.c_double * 3)()
        _check(_L.lbm_ib_force_eval(self._h, out), self._h)
        return np.array(out[:])

    def solid_maps(self):
        flags = torch.empty(self.shape, dtype=torch.uint8, device=self.device)
        n = max(self.n_markers, 1)
        cell = torch.empty(n, dtype=torch.int32, device=self.device)
        perm = torch.empty(n, dtype=torch.int32, device=self.device)
        _check(_L.lbm_solid_maps(self._h, _ptr(flags), _ptr(cell), _ptr(perm)), self._h)
        return flags, cell[: self.n_markers], perm[: self.n_markers]

    def state_bytes(self) -> int:
        n = C.c_size_t()
        _check(_L.lbm_state_bytes(self._h, C.byref(n)), self._h)
        return n.value

    def checkpoint(self, dst: torch.Tensor | None = None) -> torch.Tensor:
        if dst is None:
            dst = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        _need(dst, self.state_bytes(), "snapshot buffer")
        _check(_L.lbm_checkpoint(self._h, _ptr(dst)), self._h)
        return dst

    def restore(self, src: torch.Tensor):
        _need(src, self.state_bytes(), "snapshot")
        _check(_L.lbm_restore(self._h, _ptr(src)), self._h)

    def _grads(self, g_inlet, g_gain):
        nz, ny, _ = self.shape
        _need(g_inlet, 3 * nz * ny * 8, "g_inlet ([3, nz, ny])", torch.float64)
        _need(g_gain, self.n_markers * 8, "g_gain ([n samples])", torch.float64)


    # ------------------------------------------------------------------
    # adjoint
    def set_gains(self, gain):
        self._gain = torch.as_tensor(gain, device=self.device).to(torch.float32).contiguous()
        _need(self._gain, self.n_markers * 4, "gain ([n])", torch.float32)
        _check(_L.lbm_set_gains(self._h, _ptr(self._gain)), self._h)

    def record_tape(self, n: int, tape: torch.Tensor | None = None) -> torch.Tensor:
        """Advance n steps, storing the state before each one (n x state_bytes)."""
        sb = self.state_bytes()
        if tape is None:
            tape = torch.empty((max(n, 1), sb), dtype=torch.uint8, device=self.device)
        _need(tape, n * sb, "tape")
        _check(_L.lbm_record_tape(self._h, int(n), _ptr(tape)), self._h)
        return tape

    def adjoint_init(self):
        n = C.c_size_t()
        _check(_L.lbm_adjoint_ws_size(self._h, C.byref(n)), self._h)
        self._aws = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        _check(_L.lbm_adjoint_init(self._h, _ptr(self._aws), self._aws.numel()), self._h)

    def new_grad_inlet(self) -> torch.Tensor:
        nz, ny, _ = self.shape
        return torch.zeros((3, nz, ny), dtype=torch.float64, device=self.device)

    def new_grad_gain(self) -> torch.Tensor:
        return torch.zeros(max(self.n_markers, 1), dtype=torch.float64, device=self.device)

    def adjoint_seed_macros(self, g_rho=None, g_u=None, g_inlet=None):
        gr = None if g_rho is None else self._real(g_rho, self.shape)
        gu = None if g_u is None else self._real(g_u, (3,) + self.shape)
        self._grads(g_inlet, None)
        _check(_L.lbm_adjoint_seed_macros(self._h, _ptr(gr), _ptr(gu), _ptr(g_inlet)), self._h)

    def adjoint_seed_force(self, g_force, g_inlet=None, g_gain=None):
        gf = (C.c_double * 3)(*[float(v) for v in g_force])
        self._grads(g_inlet, g_gain)
        _check(_L.lbm_adjoint_seed_force(self._h, gf, _ptr(g_inlet), _ptr(g_gain)), self._h)

    def adjoint_step(self, n: int, tape: torch.Tensor, g_inlet=None, g_gain=None):
        _need(tape, int(n) * self.state_bytes(), "tape")
        self._grads(g_inlet, g_gain)
        _check(_L.lbm_adjoint_step(self._h, int(n), _ptr(tape), _ptr(g_inlet), _ptr(g_gain)), self._h)

    def adjoint_get(self) -> torch.Tensor:
        lam = torch.empty((27,) + self.shape, dtype=self.real, device=self.device)
        _check(_L.lbm_adjoint_get(self._h, _ptr(lam)), self._h)
        return lam

    def adjoint_set(self, lam):
        self._lam = self._real(lam, (27,) + self.shape)
        _check(_L.lbm_adjoint_set(self._h, _ptr(self._lam)), self._h)


def version() -> str:
    return _L.lbm_version().decode()
