"""The population layout (rows per block, or the plain plane-major form) is a
storage choice only: within one compiled kernel every layout runs the same
arithmetic in the same order, so all results must be bit-identical across
layouts.  The fused kernel's two addressing forms (32-bit buffer offsets or
64-bit pointers) are separately compiled kernels: the compiler may contract
the band-force arithmetic into FMAs differently in each, so between the two
forms results agree to FP32 round-off (measured: 1 ulp at a few band nodes
after one step), not bit for bit.  Exercised on a channel
with every face rule, immersed samples, an inlet profile and the passive
scalar, in FP32 and FP16 storage, on a grid whose row count is not a multiple
of the block height (ragged last block)."""
import numpy as np
import pytest
import torch

from paper_2101_11856_amd import synth
from tests.gpu_cases import FS, IN, NS, OUT, P, say
from tests.test_gpu_parity import _ib_scene, _inlet

pytestmark = pytest.mark.gpu

SHAPE = (70, 18, 15)          # nx, ny, nz: 270 rows, nx padded to 96
FACES = (IN, OUT, NS, FS, P, P)
# rows per block: plane-major, 1/2/8 rows per block, default
LAYOUTS = ["0", "1", "2", "8", None]


def _run(storage, rows, pointers, monkeypatch):
    from paper_2101_11856_amd import lbm
    if rows is None:
        monkeypatch.delenv("LBM_BLOCK_ROWS", raising=False)
    else:
        monkeypatch.setenv("LBM_BLOCK_ROWS", rows)
    monkeypatch.setenv("LBM_POINTER_PATH", "1" if pointers else "0")
    nx, ny, nz = SHAPE
    s = lbm.Solver(nx, ny, nz, 0.02, faces=FACES, inlet_profile=_inlet(ny, nz), storage=storage, scalar=True,
                   scalar_inlet_height=6)
    xyz, ub, area, gain = _ib_scene(nx, ny, nz, 11)
    s.set_solids(xyz, ub, area, gain)
    rho, u = synth.uniform(nx, ny, nz, (0.04, 0.0, 0.0))
    s.init_equilibrium(rho, u)
    s.step(25)
    out = dict(f=s.get_populations().cpu(), scalar=s.get_scalar().cpu())
    r, v = s.macros()
    out["rho"], out["u"] = r.cpu(), v.cpu()
    out["force"] = np.asarray(s.ib_force())
    out["mass"] = np.asarray(s.conserved())
    snap = s.checkpoint()
    s.step(3)
    after = s.get_populations().cpu()
    s.restore(snap)
    s.step(3)
    out["replay_equal"] = bool(torch.equal(after, s.get_populations().cpu()))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_layouts_are_bit_identical(storage, monkeypatch):
    say(f"layout invariance, {SHAPE}, storage={storage}")
    refs = {}
    for pointers in (False, True):
        ref = _run(storage, LAYOUTS[0], pointers, monkeypatch)
        assert ref["replay_equal"]
        refs[pointers] = ref
        for rows in LAYOUTS[1:]:
            say(f"  rows per block={rows or 'default'}, pointer path={pointers}")
            o = _run(storage, rows, pointers, monkeypatch)
            for k in ("f", "scalar", "rho", "u"):
                assert torch.equal(o[k], ref[k]), (rows, pointers, k)
            assert np.array_equal(o["force"], ref["force"]) and np.array_equal(o["mass"], ref["mass"]), rows
            assert o["replay_equal"], rows
    # buffer form vs pointer form: FP32 round-off only (25 steps)
    a, b = refs[False], refs[True]
    for k in ("f", "u", "scalar"):
        e = float((a[k].double() - b[k].double()).norm() / b[k].double().norm())
        say(f"  buffer vs pointer form, {k}: rel-L2 {e:.2e}")
        assert e <= 1e-6, (k, e)


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("shape,faces", [((200, 6, 5), (P, P, NS, FS, P, P)), ((256, 5, 4), (P, P, P, P, P, P))],
                         ids=["ragged-row-with-walls", "full-row-periodic"])
def test_row_staging_matches_direct_pull(shape, faces, storage, monkeypatch):
    """Rows of 193-256 nodes with periodic x take the LDS row-staged pull in
    the fused kernel (one workgroup per row).  It must give the direct pull's
    result (separately compiled kernels: to round-off), and match the FP64
    oracle after 10 steps."""
    from paper_2101_11856_amd import lbm
    from tests.gpu_cases import random_populations, rel_l2
    from oracle import oracle as O
    nx, ny, nz = shape
    say(f"row staging {shape} {storage}")
    f0 = random_populations((nz, ny, nx), seed=7)
    out = {}
    for stage in ("1", "0"):
        monkeypatch.setenv("LBM_ROW_STAGE", stage)
        s = lbm.Solver(nx, ny, nz, 0.02, faces=faces, storage=storage)
        s.set_populations(f0)
        s.step(10)
        out[stage] = s.get_populations().double().cpu().numpy()
        torch.cuda.synchronize()
    e_ab = float(np.abs(out["1"] - out["0"]).max())
    S = O.OracleSim(nx, ny, nz, 0.02, faces=faces)
    S.set_state(f0)
    S.step(10)
    ref = S.get_state()
    e_ref = rel_l2(out["1"], ref)
    say(f"  staged vs direct max |diff| {e_ab:.2e}, staged vs oracle rel-L2 {e_ref:.2e}")
    assert e_ab <= (1e-6 if storage == "f32" else 1e-5)
    assert e_ref <= (1e-6 if storage == "f32" else 1e-4)
