"""GPU parity of the fused step's collision models against the FP64 oracle
(through the C-ABI): the comparison models of the paper's Sec. 5.1, BGK and
raw-moment MRT, and the central-moment form specialised to unit rates of
orders 3 to 6 (the default, which every other parity test with default
rates also runs) beside the general form.  FP64 storage: one step from an
arbitrary state, every population, every face rule, body force, to
round-off.  FP32 storage: 50 steps, rel-L2 of rho and u <= 1e-5.  Immersed
samples: 20 steps with each model."""
import zlib

import numpy as np
import pytest
import torch

from oracle import oracle as O
from tests.gpu_cases import gpu_solver, random_populations, rel_l2, say, to_np
from tests.test_gpu_parity import FACE_CASES, IB_CASES, _ib_scene, _inlet

pytestmark = pytest.mark.gpu

# model name of the library and of the oracle, and the high-order rates used
MODELS = [("bgk", "bgk", (0.9, 1.1, 1.3, 0.8)), ("rm", "rm", (0.9, 1.1, 1.3, 0.8)),
          ("cm", "cm", (1.0, 1.0, 1.0, 1.0))]   # the last: unit high-order rates (specialised form)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_11856_amd import lbm  # noqa: F401
    yield


@pytest.mark.parametrize("name,shape,faces,profile", FACE_CASES, ids=[c[0] for c in FACE_CASES])
@pytest.mark.parametrize("model,omodel,s_high", MODELS, ids=[m[0] + ("1" if m[2][0] == 1.0 else "") for m in MODELS])
def test_one_step_all_populations_fp64(model, omodel, s_high, name, shape, faces, profile):
    nx, ny, nz = shape
    say(f"one step fp64 {model} s_high={s_high} {name} {shape}")
    f0 = random_populations((nz, ny, nx), seed=zlib.crc32((name + model).encode()) % 1000)
    body = (1e-5, -2e-5, 5e-6)
    prof = _inlet(ny, nz) if profile else None
    S = O.OracleSim(nx, ny, nz, 0.02, faces=faces, u_in=(0.05, 0, 0), body=body, s_bulk=1.2, s_high=s_high,
                    model=omodel)
    if prof is not None:
        S.set_inlet_profile(prof)
    S.set_state(f0)
    S.step(1)
    ref = S.get_state()
    s = gpu_solver(nx, ny, nz, 0.02, storage="f64", faces=faces, u_in=(0.05, 0, 0), inlet_profile=prof, body=body,
                   s_bulk=1.2, s_high=s_high, collision=model)
    s.set_populations(f0)
    s.step(1)
    err = np.abs(to_np(s.get_populations()) - ref).max()
    say(f"  max |diff| = {err:.3e}")
    assert err < 1e-14


@pytest.mark.parametrize("name,shape,faces,profile", FACE_CASES[:5], ids=[c[0] for c in FACE_CASES[:5]])
@pytest.mark.parametrize("model,omodel,s_high", MODELS, ids=[m[0] + ("1" if m[2][0] == 1.0 else "") for m in MODELS])
def test_fifty_steps_fp32(model, omodel, s_high, name, shape, faces, profile):
    nx, ny, nz = shape
    say(f"fifty steps fp32 {model} {name} {shape}")
    f0 = random_populations((nz, ny, nx), seed=zlib.crc32((name + model).encode()) % 1000, amp=0.01)
    f0 = f0.astype(np.float32).astype(np.float64)
    prof = _inlet(ny, nz) if profile else None
    S = O.OracleSim(nx, ny, nz, 0.02, faces=faces, u_in=(0.05, 0, 0), s_high=s_high, model=omodel)
    if prof is not None:
        S.set_inlet_profile(prof)
    S.set_state(f0)
    S.step(50)
    r_ref, u_ref = S.macros()
    s = gpu_solver(nx, ny, nz, 0.02, storage="f32", faces=faces, u_in=(0.05, 0, 0), inlet_profile=prof,
                   s_high=s_high, collision=model)
    s.set_populations(f0)
    s.step(50)
    r, u = (to_np(t) for t in s.macros())
    e_u, e_r = rel_l2(u, u_ref), rel_l2(r, r_ref)
    say(f"  rel-L2 u={e_u:.3e} rho={e_r:.3e}")
    assert e_u <= 1e-5 and e_r <= 1e-5


@pytest.mark.parametrize("model", ["bgk", "rm"])
@pytest.mark.parametrize("storage,gate", [("f64", 1e-12), ("f32", 1e-5)])
def test_ib_steps_with_model(model, storage, gate):
    name, (nx, ny, nz), faces = IB_CASES[1]
    say(f"ib steps {name} {model} {storage}")
    xyz, ub, area, gain = _ib_scene(nx, ny, nz, 7)
    rng = np.random.default_rng(3)
    rho = (1.0 + 1e-3 * rng.standard_normal((nz, ny, nx))).astype(np.float32)
    u = np.zeros((3, nz, ny, nx), np.float32)
    u[0] = 0.03
    u += (0.005 * rng.standard_normal(u.shape)).astype(np.float32)
    S = O.OracleSim(nx, ny, nz, 0.05, faces=faces, u_in=(0.03, 0, 0), model=model)
    S.set_markers(xyz, ub.astype(np.float64), area.astype(np.float64), gain.astype(np.float64))
    S.init_equilibrium(rho.astype(np.float64), u.astype(np.float64))
    S.step(20)
    r_ref, u_ref = S.macros()
    F_ref = S.last_force()
    s = gpu_solver(nx, ny, nz, 0.05, storage=storage, faces=faces, u_in=(0.03, 0, 0), collision=model)
    s.set_solids(xyz, ub, area, gain)
    real = np.float64 if storage == "f64" else np.float32
    s.init_equilibrium(rho.astype(real), u.astype(real))
    s.step(20)
    r, uu = (to_np(t) for t in s.macros())
    F = s.ib_force()
    e_u, e_r, e_F = rel_l2(uu, u_ref), rel_l2(r, r_ref), rel_l2(F, F_ref)
    say(f"  rel-L2 u={e_u:.3e} rho={e_r:.3e} force={e_F:.3e}")
    assert e_u <= gate and e_r <= gate and e_F <= (1e-11 if storage == "f64" else 1e-4)


def test_adjoint_refuses_other_models():
    from paper_2101_11856_amd import lbm
    s = gpu_solver(8, 6, 5, 0.05, collision="bgk")
    with pytest.raises(lbm.LbmError) as e:
        s.adjoint_init()
    assert e.value.status == 6
