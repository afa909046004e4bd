"""lbm_conserved_static, the entry point that allocates nothing (its partial
sums, counter and totals sit in the library's static device array), against
lbm_conserved (the same reduction in the context's workspace), both called
through the C-ABI.  The two share their kernels and summation order, so the
FP64 totals must agree bit for bit.  Two calls in a row, the second on a
smaller grid (fewer partial sums than the array still holds from the first),
then a state with a NaN and a clean state after it (the counter the array
keeps must be cleared at every call)."""
import numpy as np
import pytest
import torch

from tests.gpu_cases import gpu_solver, random_populations, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_11856_amd import lbm  # noqa: F401  (fails loudly if liblbm.so is missing)
    yield


def _solver(shape, seed, storage="f32", nan_at=None):
    nz, ny, nx = shape
    f = random_populations(shape, seed=seed)
    if nan_at is not None:
        f[nan_at] = np.nan
    s = gpu_solver(nx, ny, nz, 0.05, storage=storage)
    s.set_populations(f.astype(np.float64 if storage == "f64" else np.float32))
    return s


@pytest.mark.parametrize("storage", ["f32", "f16", "f64"])
def test_static_scratch_totals_equal_workspace_totals(storage):
    # call 1: 80x64x64 = 327,680 nodes -> 1024 per-block partials (the cap);
    # call 2: 9x5x6 = 270 nodes -> 2 partials, the rest of the array still
    # holding call 1's partials
    for shape, seed in (((64, 64, 80), 11), ((6, 5, 9), 12)):
        say(f"lbm_conserved_static vs lbm_conserved, {storage}, grid {shape[::-1]}")
        s = _solver(shape, seed, storage)
        ref = s.conserved()
        got = s.conserved_static()
        assert np.array_equal(got, ref), (got, ref)
        if storage == "f64":
            # and against a plain host sum of the FP64 state (the 32- and
            # 16-bit forms read back as rounded f = w + d, which moves the
            # host sum by the rounding of w itself)
            f = s.get_populations().double().cpu().numpy()
            host = [f.sum()] + [0.0] * 3
            from oracle import oracle as O
            c = O.lattice()[0]
            for a in range(3):
                host[a + 1] = float((c[:, a][:, None, None, None] * f).sum())
            assert abs(got[0] - host[0]) <= 1e-12 * abs(host[0])
            assert np.allclose(got[1:], host[1:], rtol=0, atol=1e-12 * abs(host[0]))
        del s
        torch.cuda.synchronize()


def test_static_scratch_counter_cleared_between_calls():
    from paper_2101_11856_amd import lbm
    say("lbm_conserved_static: NaN state, then a clean smaller state")
    bad = _solver((10, 7, 70), 21, nan_at=(5, 3, 2, 33))
    for call in (bad.conserved, bad.conserved_static):
        with pytest.raises(lbm.LbmError) as e:
            call()
        assert e.value.status == 4
    good = _solver((3, 4, 5), 22)
    assert np.array_equal(good.conserved_static(), good.conserved())
