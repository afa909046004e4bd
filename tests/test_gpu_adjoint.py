"""Adjoint of the collide-stream-IB step.

1. Dot-product tests of one step and of the two seeds in FP64 storage:
   <lambda, J v> by central differences of the forward step equals
   <J^T lambda, v> from the hand-written adjoint; likewise for the inlet
   profile and the sample gains.
2. Independent FP64 reference: central finite differences of the CPU oracle
   on a small channel; the GPU adjoint (FP64 and FP32) must match.
3. Full channel configuration (128x64x64, 2000 steps, checkpoint every 100):
   FP32 adjoint through torch.autograd against FP64 central differences of
   the GPU forward, within 1e-3 relative.
4. Bookkeeping: interleaved forward runs keep their own gradients; a reverse
   sweep split over several calls equals the single call.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2101_11856_amd import synth
from tests.gpu_cases import FS, IN, NS, OUT, P, gpu_solver, random_populations, rel_l2, say, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2101_11856_amd import lbm  # noqa: F401
    yield


def _dot(a, b):
    return float((to_np(a) * to_np(b)).sum())


def _scene(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    xyz = synth.fibonacci_sphere(120, 2.5, (nx / 3, ny / 2 - 0.3, nz / 2 + 0.2))
    box = synth.random_box(60, (nx / 2, 2.0, 2.0), (nx / 2 + 3, 5.0, 5.0), seed)
    xyz = np.concatenate([xyz, box], axis=1)
    n = xyz.shape[1]
    ub = (0.01 * rng.standard_normal((3, n))).astype(np.float32)
    area = np.concatenate([np.full(120, 4 * np.pi * 2.5 ** 2 / 120), np.full(60, 27 / 60)]).astype(np.float32)
    gain = (0.7 + 0.6 * rng.random(n)).astype(np.float32)
    return xyz, ub, area, gain


STEP_CASES = [
    ("periodic", (P, P, P, P, P, P)),
    ("inlet-outflow-walls", (IN, OUT, NS, FS, P, P)),
    ("channel", (IN, OUT, NS, NS, NS, NS)),
]


@pytest.mark.parametrize("name,faces", STEP_CASES, ids=[c[0] for c in STEP_CASES])
def test_one_step_dot_product_fp64(name, faces):
    nx, ny, nz = 70, 10, 9
    say(f"adjoint dot-product one step {name}")
    rng = np.random.default_rng(31)
    xyz, ub, area, gain = _scene(nx, ny, nz, 5)
    prof = np.zeros((3, nz, ny))
    prof[0] = 0.04 + 0.005 * rng.standard_normal((nz, ny))
    prof[1] = 0.002 * rng.standard_normal((nz, ny))
    kw = dict(faces=faces, inlet_profile=prof, body=(1e-5, 0, -1e-5), s_bulk=1.1, s_high=(0.9, 1.2, 1.1, 0.8))
    s = gpu_solver(nx, ny, nz, 0.02, storage="f64", **kw)
    s.set_solids(xyz, ub, area, gain)
    s.adjoint_init()
    f0 = random_populations((nz, ny, nx), seed=32, amp=0.02)
    v = rng.standard_normal((27, nz, ny, nx)) * 1e-3
    lam = rng.standard_normal((27, nz, ny, nx))
    pin = np.zeros((3, nz, ny))
    pin[0] = rng.standard_normal((nz, ny))
    pin[2] = rng.standard_normal((nz, ny))
    qg = rng.standard_normal(xyz.shape[1])

    def step_from(f, profile=prof, g=gain):
        s.set_inlet_profile(profile)
        s.set_gains(g)
        s.set_populations(f)
        s.step(1)
        return s.get_populations()

    eps = 1e-6
    lam_t = torch.as_tensor(lam, device="cuda")
    fd_f = _dot(lam_t, step_from(f0 + eps * v) - step_from(f0 - eps * v)) / (2 * eps)
    fd_in = _dot(lam_t, step_from(f0, prof + eps * pin) - step_from(f0, prof - eps * pin)) / (2 * eps)
    fd_g = _dot(lam_t, step_from(f0, prof, (gain + eps * qg).astype(np.float32))
                - step_from(f0, prof, (gain - eps * qg).astype(np.float32))) / (2 * eps)
    # gains are stored as float: use the float perturbation actually applied
    dq = ((gain + eps * qg).astype(np.float32).astype(np.float64) - (gain - eps * qg).astype(np.float32)) / (2 * eps)

    s.set_inlet_profile(prof)
    s.set_gains(gain)
    s.set_populations(f0)
    tape = s.record_tape(1)
    s.adjoint_set(lam)
    g_in, g_g = s.new_grad_inlet(), s.new_grad_gain()
    s.adjoint_step(1, tape, g_in, g_g)
    ad_f = _dot(s.adjoint_get(), torch.as_tensor(v, device="cuda"))
    ad_in = float((g_in.cpu().numpy() * pin).sum())
    ad_g = float((g_g.cpu().numpy()[: len(qg)] * dq).sum())
    say(f"  f: {ad_f:.10e} vs {fd_f:.10e}; inlet: {ad_in:.8e} vs {fd_in:.8e}; gain: {ad_g:.8e} vs {fd_g:.8e}")
    assert abs(ad_f - fd_f) <= 1e-7 * abs(fd_f)
    if faces[0] == IN:
        assert abs(ad_in - fd_in) <= 1e-6 * abs(fd_in)
    assert abs(ad_g - fd_g) <= 1e-6 * abs(fd_g)


def test_seeds_dot_product_fp64():
    nx, ny, nz = 70, 10, 9
    say("adjoint seeds")
    rng = np.random.default_rng(41)
    xyz, ub, area, gain = _scene(nx, ny, nz, 6)
    prof = np.zeros((3, nz, ny))
    prof[0] = 0.04
    s = gpu_solver(nx, ny, nz, 0.02, storage="f64", faces=(IN, OUT, NS, FS, P, P), inlet_profile=prof)
    s.set_solids(xyz, ub, area, gain)
    f0 = random_populations((nz, ny, nx), seed=42, amp=0.02)
    v = rng.standard_normal((27, nz, ny, nx)) * 1e-3
    g_rho = rng.standard_normal((nz, ny, nx))
    g_u = rng.standard_normal((3, nz, ny, nx))
    gf = np.array([0.7, -0.2, 0.4])
    eps = 1e-5   # rho ~ 1: a larger step keeps the FP64 round-off of the differences small

    def macros_force(f):
        s.set_populations(f)
        r, u = s.macros()
        return to_np(r), to_np(u), s.ib_force_eval()

    rp, up, Fp = macros_force(f0 + eps * v)
    rm, um, Fm = macros_force(f0 - eps * v)
    fd_m = ((rp - rm) * g_rho).sum() / (2 * eps) + ((up - um) * g_u).sum() / (2 * eps)
    fd_F = float(((Fp - Fm) * gf).sum() / (2 * eps))
    s.set_populations(f0)
    s.adjoint_init()
    s.adjoint_seed_macros(g_rho, g_u)
    ad_m = _dot(s.adjoint_get(), torch.as_tensor(v, device="cuda"))
    s.adjoint_init()
    g_g = s.new_grad_gain()
    s.adjoint_seed_force(gf, None, g_g)
    ad_F = _dot(s.adjoint_get(), torch.as_tensor(v, device="cuda"))
    # gain part of the force seed: dF/dgamma . gf = sum_s a_s rho_s (u_b - u_s) . gf
    _, gs = _oracle_penalty(f0, nx, ny, nz, xyz, ub, area, np.ones_like(gain))
    ref_gain = (area.astype(np.float64)[None, :] * gs * gf[:, None]).sum(0)
    say(f"  macros: {ad_m:.10e} vs {fd_m:.10e}; force: {ad_F:.10e} vs {fd_F:.10e}")
    assert abs(ad_m - fd_m) <= 1e-6 * abs(fd_m)
    assert abs(ad_F - fd_F) <= 1e-6 * abs(fd_F)
    assert np.abs(g_g.cpu().numpy()[: len(gain)] - ref_gain).max() <= 1e-10 * np.abs(ref_gain).max()


def _oracle_penalty(f0, nx, ny, nz, xyz, ub, area, gain):
    S = O.OracleSim(nx, ny, nz, 0.02, faces=(IN, OUT, NS, FS, P, P), u_in=(0.04, 0, 0))
    S.set_markers(xyz, ub.astype(np.float64), area.astype(np.float64), gain.astype(np.float64))
    S.set_state(f0)
    return S.ib_force(per_marker=True)


# ---------------------------------------------------------------------------
# independent FP64 reference: oracle finite differences on a small channel
# ---------------------------------------------------------------------------
SMALL = dict(nx=24, ny=12, nz=12, nu=0.02, steps=30, probe_x=18, radius=2.5, center=(8.0, 6.0), n_around=12,
             mode_length=12.0)


def _small_markers():
    xyz, ub, area, _ = synth.cylinder_markers(SMALL["radius"], SMALL["center"], SMALL["nz"], SMALL["n_around"])
    keep = xyz[2] < SMALL["nz"] - 1
    return xyz[:, keep], ub[:, keep], area[keep]


def _oracle_J(coeffs, gains):
    c = SMALL
    xyz, ub, area = _small_markers()
    prof = synth.inlet_profile(c["ny"], c["nz"], coeffs, length=c["mode_length"])
    S = O.OracleSim(c["nx"], c["ny"], c["nz"], c["nu"], faces=(IN, OUT, NS, NS, NS, NS))
    S.set_inlet_profile(prof)
    S.set_markers(xyz, ub.astype(np.float64), area.astype(np.float64), np.asarray(gains, np.float64))
    rho, u = synth.uniform(c["nx"], c["ny"], c["nz"], (0.04, 0, 0), dtype=np.float64)
    S.init_equilibrium(rho, u)
    S.step(c["steps"])
    F = S.ib_force()
    _, uu = S.macros()
    probe = uu[:, :, :, c["probe_x"]]
    return -F[0] + ((probe - np.array([0.04, 0, 0])[:, None, None]) ** 2).sum()


@pytest.fixture(scope="module")
def small_fd():
    """Central differences of the oracle objective in the 16 inflow
    coefficients and in 2 random gain directions (FP64)."""
    rng = np.random.default_rng(51)
    coeffs = np.asarray(synth.inlet_coefficients(seed=2105)) * 0.5
    xyz, _, _ = _small_markers()
    gains = (0.8 + 0.4 * rng.random(xyz.shape[1])).astype(np.float32).astype(np.float64)
    dirs = rng.standard_normal((2, xyz.shape[1]))
    h = 1e-6
    g_c = np.zeros(16)
    for k in range(16):
        e = np.zeros(16)
        e[k] = h
        g_c[k] = (_oracle_J(coeffs + e, gains) - _oracle_J(coeffs - e, gains)) / (2 * h)
    g_d = np.array([(_oracle_J(coeffs, gains + h * d) - _oracle_J(coeffs, gains - h * d)) / (2 * h) for d in dirs])
    return coeffs, gains, dirs, g_c, g_d


@pytest.mark.parametrize("storage,gate", [("f64", 1e-6), ("f32", 1e-3)])
def test_adjoint_matches_oracle_finite_differences(small_fd, storage, gate):
    from paper_2101_11856_amd.adjoint import AdjointRun, ChannelProblem
    coeffs, gains, dirs, g_c_ref, g_d_ref = small_fd
    say(f"adjoint vs oracle FD, small channel, storage={storage}")
    c = SMALL
    prob = ChannelProblem(nx=c["nx"], ny=c["ny"], nz=c["nz"], nu=c["nu"], steps=c["steps"], checkpoint_every=7,
                          storage=storage, probe_x=c["probe_x"], radius=c["radius"], center=c["center"],
                          n_around=c["n_around"], mode_length=c["mode_length"])
    a = torch.tensor(coeffs, dtype=torch.float64, device="cuda", requires_grad=True)
    g = torch.tensor(gains, dtype=torch.float64, device="cuda", requires_grad=True)
    drag, probe = AdjointRun.apply(prob, a, g)
    J = prob.objective(drag, probe)
    J.backward()
    g_c = a.grad.cpu().numpy()
    g_d = dirs @ g.grad.cpu().numpy()
    e_c, e_d = rel_l2(g_c, g_c_ref), rel_l2(g_d, g_d_ref)
    say(f"  J={float(J.detach()):.10e} rel err coeffs={e_c:.3e} gain dirs={e_d:.3e}")
    assert e_c <= gate and e_d <= gate


# ---------------------------------------------------------------------------
# exact reference: torch.autograd through the independent FP64 model
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("storage,gate", [("f64", 1e-9), ("f32", 1e-3)])
def test_adjoint_matches_fp64_autograd_model(storage, gate):
    """Every component of both gradients (16 inflow coefficients, one gain
    per sample) against the exact gradient of the plain-PyTorch FP64 model,
    whose objective equals the C oracle's."""
    from paper_2101_11856_amd.adjoint import AdjointRun, ChannelProblem
    from tests.test_oracle_autograd import CHANNEL, TINY, _gains, _markers, autograd_J
    c = dict(TINY, steps=20)
    coeffs = 0.5 * synth.inlet_coefficients(seed=2105)
    gains = _gains(_markers(c)[0].shape[1])
    J_ref, ga_ref, gg_ref = autograd_J(c, CHANNEL, coeffs, gains)
    say(f"adjoint vs FP64 autograd model, tiny channel, storage={storage}")
    prob = ChannelProblem(nx=c["nx"], ny=c["ny"], nz=c["nz"], nu=c["nu"], steps=c["steps"], checkpoint_every=6,
                          storage=storage, probe_x=c["probe_x"], radius=c["radius"], center=c["center"],
                          n_around=c["n_around"], mode_length=c["mode_length"])
    a = torch.tensor(coeffs, dtype=torch.float64, device="cuda", requires_grad=True)
    g = torch.tensor(gains, dtype=torch.float64, device="cuda", requires_grad=True)
    drag, probe = AdjointRun.apply(prob, a, g)
    J = prob.objective(drag, probe)
    J.backward()
    e_J = abs(float(J) - J_ref) / abs(J_ref)
    e_a = rel_l2(a.grad.cpu().numpy(), ga_ref)
    e_g = rel_l2(g.grad.cpu().numpy(), gg_ref)
    say(f"  J rel err {e_J:.3e}, coeff gradient {e_a:.3e}, gain gradient {e_g:.3e}")
    assert e_J <= gate and e_a <= gate and e_g <= gate


# ---------------------------------------------------------------------------
# full channel configuration
# ---------------------------------------------------------------------------
def test_adjoint_full_channel_vs_gpu_finite_differences():
    from paper_2101_11856_amd.adjoint import AdjointRun, ChannelProblem
    say("adjoint full channel 128x64x64, 2000 steps: fp32 adjoint vs fp64 central differences")
    coeffs = synth.inlet_coefficients(seed=2105)
    p64 = ChannelProblem(storage="f64")
    gains = np.ones(p64.n)
    rng = np.random.default_rng(61)
    gdirs = rng.standard_normal((2, p64.n))

    def J64(cf, gn):
        d, pr, _ = p64.run_forward(torch.as_tensor(cf, device="cuda"), torch.as_tensor(gn, device="cuda"),
                                   keep_checkpoints=False)
        return float(p64.objective(d, pr))

    h = 1e-4 * 0.01
    fd_c = np.zeros(16)
    for k in range(16):
        e = np.zeros(16)
        e[k] = h
        fd_c[k] = (J64(coeffs + e, gains) - J64(coeffs - e, gains)) / (2 * h)
    hg = 1e-4
    fd_g, dq = [], []
    for d in gdirs:   # gains are stored as float: use the perturbation actually applied
        gp, gm = (gains + hg * d).astype(np.float32), (gains - hg * d).astype(np.float32)
        fd_g.append((J64(coeffs, gp) - J64(coeffs, gm)) / (2 * hg))
        dq.append((gp.astype(np.float64) - gm.astype(np.float64)) / (2 * hg))
    fd_g, dq = np.array(fd_g), np.array(dq)
    del p64
    torch.cuda.empty_cache()

    p32 = ChannelProblem(storage="f32")
    a = torch.tensor(coeffs, dtype=torch.float64, device="cuda", requires_grad=True)
    g = torch.tensor(gains, dtype=torch.float64, device="cuda", requires_grad=True)
    drag, probe = AdjointRun.apply(p32, a, g)
    J = p32.objective(drag, probe)
    J.backward()
    e_c = rel_l2(a.grad.cpu().numpy(), fd_c)
    e_g = rel_l2(dq @ g.grad.cpu().numpy(), fd_g)
    say(f"  J={float(J):.8e} drag={float(drag):.6e} rel err coeffs={e_c:.3e} gain dirs={e_g:.3e}")
    assert e_c <= 1e-3 and e_g <= 1e-3


# ---------------------------------------------------------------------------
# several forward runs on one problem before their backward passes
# ---------------------------------------------------------------------------
def test_interleaved_forwards_keep_their_own_gradients():
    """Two forward runs with different inflow coefficients and gains on one
    problem, then their backward passes in reverse order: each gradient equals
    the one its run gives alone, because each autograd context holds its own
    parameters, checkpoints and final state.  The adjoint's face and
    interpolation transposes add with atomics, so the comparison allows FP32
    round-off (1e-5).  The two runs' coefficient gradients differ by about
    7e-3 (relative), so a backward pass that used the other run's
    checkpoints would miss the gate by orders of magnitude."""
    from paper_2101_11856_amd.adjoint import AdjointRun, ChannelProblem
    c = SMALL
    prob = ChannelProblem(nx=c["nx"], ny=c["ny"], nz=c["nz"], nu=c["nu"], steps=c["steps"], checkpoint_every=7,
                          storage="f32", probe_x=c["probe_x"], radius=c["radius"], center=c["center"],
                          n_around=c["n_around"], mode_length=c["mode_length"])
    rng = np.random.default_rng(71)
    runs = [(0.5 * synth.inlet_coefficients(seed=2105), np.ones(prob.n)),
            (-0.7 * synth.inlet_coefficients(seed=2106), 0.8 + 0.4 * rng.random(prob.n))]

    def leaves(cf, gn):
        return (torch.tensor(cf, dtype=torch.float64, device="cuda", requires_grad=True),
                torch.tensor(gn, dtype=torch.float64, device="cuda", requires_grad=True))

    alone = []
    for cf, gn in runs:
        a, g = leaves(cf, gn)
        prob.objective(*AdjointRun.apply(prob, a, g)).backward()
        alone.append((a.grad.cpu().numpy(), g.grad.cpu().numpy()))
    say("adjoint: two forward runs, then their backward passes in reverse order")
    lv = [leaves(cf, gn) for cf, gn in runs]
    Js = [prob.objective(*AdjointRun.apply(prob, a, g)) for a, g in lv]
    Js[1].backward()
    Js[0].backward()
    errs = []
    for (a, g), (ga, gg) in zip(lv, alone):
        errs += [rel_l2(a.grad.cpu().numpy(), ga), rel_l2(g.grad.cpu().numpy(), gg)]
    apart = rel_l2(alone[0][0], alone[1][0])
    say(f"  interleaved vs alone: max rel err {max(errs):.2e}; the two runs' coefficient gradients differ by {apart:.2e}")
    assert max(errs) <= 1e-5 and apart > 1e-3
    # a run without checkpoints has no reverse sweep and says so
    _, _, rec = prob.run_forward(torch.as_tensor(runs[0][0], device="cuda"), torch.as_tensor(runs[0][1], device="cuda"),
                                 keep_checkpoints=False)
    with pytest.raises(RuntimeError):
        prob.run_backward(rec, 1.0, torch.zeros((3, prob.nz, prob.ny), dtype=torch.float64, device="cuda"))


# ---------------------------------------------------------------------------
# one reverse sweep split over several calls
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("storage,gate", [("f64", 1e-12), ("f32", 1e-5)])
def test_split_reverse_sweep_equals_one_call(storage, gate):
    """K adjoint steps in one call against the same K steps in two calls of
    K/2 (the later half of the tape first), with nothing, an adjoint_get, or
    an adjoint_get + adjoint_set of what it returned between the calls.  The
    reverse streaming is folded into the next step's collision, so a call
    can end with the adjoint state not yet formed; adjoint_get must form it
    without disturbing the sweep, and adjoint_set must hand it back exactly.
    The adjoint state and both gradient accumulators (inlet profile, sample
    gains) must agree with the single call; they differ only by the order of
    the atomic additions in the face and interpolation transposes."""
    nx, ny, nz, K = 70, 10, 9, 6
    say(f"adjoint: {K} steps in one call vs two calls ({storage})")
    rng = np.random.default_rng(91)
    xyz, ub, area, gain = _scene(nx, ny, nz, 8)
    prof = np.zeros((3, nz, ny))
    prof[0] = 0.04 + 0.005 * rng.standard_normal((nz, ny))
    s = gpu_solver(nx, ny, nz, 0.02, storage=storage, faces=(IN, OUT, NS, FS, P, P), inlet_profile=prof,
                   body=(1e-5, 0, -1e-5))
    s.set_solids(xyz, ub, area, gain)
    s.adjoint_init()
    s.set_populations(random_populations((nz, ny, nx), seed=92, amp=0.02))
    tape = s.record_tape(K)
    lam0 = torch.as_tensor(rng.standard_normal((27, nz, ny, nx)), device="cuda").to(s.real)

    def sweep(between):
        gi, gg = s.new_grad_inlet(), s.new_grad_gain()
        s.adjoint_set(lam0)
        if between is None:
            s.adjoint_step(K, tape, gi, gg)
        else:
            s.adjoint_step(K // 2, tape[K // 2:], gi, gg)
            if between != "nothing":
                mid = s.adjoint_get()
                if between == "get+set":
                    s.adjoint_set(mid.clone())
            s.adjoint_step(K // 2, tape[:K // 2], gi, gg)
        return to_np(s.adjoint_get()), to_np(gi), to_np(gg)

    one = sweep(None)
    assert np.isfinite(one[0]).all() and np.abs(one[1]).sum() > 0 and np.abs(one[2]).sum() > 0
    for between in ("nothing", "get", "get+set"):
        got = sweep(between)
        errs = [rel_l2(g, r) for g, r in zip(got, one)]
        say(f"  two calls, {between} between: rel err lambda {errs[0]:.1e}, inlet {errs[1]:.1e}, gains {errs[2]:.1e}")
        assert max(errs) <= gate, (between, errs)
