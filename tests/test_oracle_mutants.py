"""Mutation test of the oracle's pins: each entry plants one plausible mistake
in a temporary copy of the oracle source (the C file, or the Python rigid
placement) (a dropped term, a wrong sign, index
or operand, a misplaced face rule), builds it, and runs the pin suite against
it; every mutant must make some pin fail.  An unmutated copy built the same
way must pass, so a broken harness cannot pass for a caught mutant.  The
committed oracle is never modified.  CPU only (gcc)."""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_oracle.c")
PINS = ["tests/test_oracle_moments.py", "tests/test_oracle_flows.py", "tests/test_oracle_ib.py",
        "tests/test_oracle_motion.py", "tests/test_oracle_models.py"]
SKIP_SLOW = "not taylor_green_decay_rate and not magic_odd_rates"   # 15 s of the suite; never the only catcher

# name: (text in lbm_oracle.c, replacement)
MUTANTS = {
    # collision (Eqs. 4-5) and the readings R2-R8
    "force_sign": ("return F[axis] * ipow(CS2, twos);", "return -F[axis] * ipow(CS2, twos);"),
    "force_high_orders_dropped": ("if (ones != 1) return 0.0;", "if (ones != 1 || twos > 0) return 0.0;"),
    "no_half_force_shift": ("u[a] = (j[a] + 0.5 * F[a]) / rho;", "u[a] = j[a] / rho;"),
    "trace_at_shear_rate": ("return (k == 9) ? s_b : s_nu;", "return s_nu;"),
    "high_rates_reversed": ("return s_high[order - 3];", "return s_high[6 - order];"),
    "equilibrium_moment_power": ("if (e[a] == 2) v *= CS2;", "if (e[a] == 2) v = rho * CS2;"),
    "central_matrix_transposed": ("T[k * Q + i] = v;", "T[i * Q + k] = v;"),
    "trace_row_sign": ("C[9 * Q + k002] = 1.0;", "C[9 * Q + k002] = -1.0;"),
    "weights_swapped": ("(CV[i][a] == 0) ? 2.0 / 3.0 : 1.0 / 6.0", "(CV[i][a] == 0) ? 1.0 / 6.0 : 2.0 / 3.0"),
    "equilibrium_velocity_sign": ("else v *= (1.0 / 3.0 + CV[i][a] * ua + ua * ua) * 0.5;",
                                  "else v *= (1.0 / 3.0 - CV[i][a] * ua + ua * ua) * 0.5;"),
    # streaming and faces (Eq. 3, Alg. 1, reading R16)
    "pull_wrong_direction": ("src[a] = p[a] - CV[i][a];", "src[a] = p[a] + CV[i][a];"),
    "bounce_back_same_direction": ("    case F_NOSLIP:\n        return f[opposite(i) * N + lin(S, px, py, pz)];",
                                   "    case F_NOSLIP:\n        return f[i * N + lin(S, px, py, pz)];"),
    "inlet_missing_factor_2": ("+ 2.0 * weight(i) * cu / CS2;", "+ weight(i) * cu / CS2;"),
    "inlet_sign": ("+ 2.0 * weight(i) * cu / CS2;", "- 2.0 * weight(i) * cu / CS2;"),
    "inlet_profile_yz_swapped": ("if (S->inlet) return S->inlet[((int64_t)a * S->n[2] + z) * S->n[1] + y];",
                                 "if (S->inlet) return S->inlet[((int64_t)a * S->n[2] + y) * S->n[1] + z];"),
    "outflow_two_inward": ("q[bestaxis] += bestside ? -1 : 1;", "q[bestaxis] += bestside ? -2 : 2;"),
    "free_slip_reflects_all": ("            if (crossed[a]) {\n                cr[a] = -cr[a];",
                               "            if (1) {\n                cr[a] = -cr[a];"),
    # macros and immersed boundary (Eqs. 2, 6-8; readings R10-R15)
    "macros_no_rho_division": ("for (int a = 0; a < 3; ++a) S->u0[a * N + k] = j[a] / rho;",
                               "for (int a = 0; a < 3; ++a) S->u0[a * N + k] = j[a];"),
    "penalty_sign": ("S->gain[s] * rs * (S->ub[a * n + s] - us[a]);", "S->gain[s] * rs * (us[a] - S->ub[a * n + s]);"),
    "penalty_without_gain": ("S->gain[s] * rs * (S->ub[a * n + s] - us[a]);", "rs * (S->ub[a * n + s] - us[a]);"),
    "trilinear_weights_swapped": ("K *= d[a] ? t : 1.0 - t;", "K *= d[a] ? 1.0 - t : t;"),
    "spreading_without_area": ("acc[a] += S->area[s] * K * S->Gs[a * n + s];", "acc[a] += K * S->Gs[a * n + s];"),
    "gather_offset_bits_swapped": ("const int d[3] = {code & 1, (code >> 1) & 1, (code >> 2) & 1};",
                                   "const int d[3] = {(code >> 2) & 1, (code >> 1) & 1, code & 1};"),
    "morton_axis_order": ("<< (3 * bit + a);", "<< (3 * bit + (2 - a));"),
    "block_order_yx": ("const uint64_t block = (uint64_t)B[0] + (uint64_t)nb[0] * ((uint64_t)B[1] + (uint64_t)nb[1] * B[2]);",
                       "const uint64_t block = (uint64_t)B[1] + (uint64_t)nb[1] * ((uint64_t)B[0] + (uint64_t)nb[0] * B[2]);"),
    # total torque of the samples (Alg. 2 (c))
    "torque_z_sign": ("t[2] += r[0] * F[1] - r[1] * F[0];", "t[2] += r[1] * F[0] - r[0] * F[1];"),
    "torque_x_sign": ("t[0] += r[1] * F[2] - r[2] * F[1];", "t[0] += r[2] * F[1] - r[1] * F[2];"),
    "torque_without_area": ("const double F[3] = {S->area[s] * S->Gs[s], S->area[s] * S->Gs[n + s], S->area[s] * S->Gs[2 * n + s]};",
                            "const double F[3] = {S->Gs[s], S->Gs[n + s], S->Gs[2 * n + s]};"),
    "torque_lever_reversed": ("const double r[3] = {(double)S->mx[s] - o[0], (double)S->mx[n + s] - o[1], (double)S->mx[2 * n + s] - o[2]};",
                              "const double r[3] = {o[0] - (double)S->mx[s], o[1] - (double)S->mx[n + s], o[2] - (double)S->mx[2 * n + s]};"),
    # comparison collision models (Sec. 5.1): BGK and raw-moment MRT
    "bgk_force_factor": ("+ (1.0 - 0.5 * omega) * G[i];", "+ (1.0 - omega) * G[i];"),
    "bgk_equilibrium_without_half_force": ("    orc_equilibrium(rho, u, feq);\n    orc_forcing_shape(u, F, G);\n    for (int i = 0; i < Q; ++i) fpost[i]",
                                           "    const double u0[3] = {u[0] - 0.5 * F[0] / rho, u[1] - 0.5 * F[1] / rho, u[2] - 0.5 * F[2] / rho};\n    orc_equilibrium(rho, u0, feq);\n    orc_forcing_shape(u, F, G);\n    for (int i = 0; i < Q; ++i) fpost[i]"),
    "models_no_half_force_shift": ("u[a] = (j[a] + F[a] / 2.0) / rho;", "u[a] = j[a] / rho;"),
    "forcing_shape_derivative_sign": ("dphi[a] = (CV[i][a] + 2.0 * ua) * 0.5;", "dphi[a] = (CV[i][a] - 2.0 * ua) * 0.5;"),
    "rm_moments_about_u": ("orc_basis_matrix(zero, M0);", "orc_basis_matrix(u, M0);"),
    "rm_force_moments_dropped": ("mp[k] = m - s * (m - me) + (1.0 - 0.5 * s) * mf;", "mp[k] = m - s * (m - me);"),
    "rm_trace_rate": ("        const double s = rate_of(k, s_nu, s_b, s_high);\n        mp[k] = m - s",
                      "        const double s = rate_of(k == 9 ? 7 : k, s_nu, s_b, s_high);\n        mp[k] = m - s"),
    "model_switch_swapped": ("if (S->model == 1) rc = orc_collide_bgk", "if (S->model == 2) rc = orc_collide_bgk"),
    # passive scalar (reading R21)
    "scalar_downwind": ("if (u[a] > 0.0) v -= u[a]", "if (u[a] < 0.0) v -= u[a]"),
    "scalar_inlet_height_off_by_one": ("y < S->scalar_inlet_height) v = 1.0;", "y <= S->scalar_inlet_height) v = 1.0;"),
}


# mistakes planted in the oracle's Python part (the rigid placement of Alg. 2 (c))
PY_SRC = os.path.join(ROOT, "oracle", "oracle.py")
PY_PINS = ["tests/test_oracle_motion.py"]
PY_MUTANTS = {
    "pose_rotation_transposed": ("(o[a] + ((R[a, 0] * X[0] + R[a, 1] * X[1]) + R[a, 2] * X[2]))",
                                 "(o[a] + ((R[0, a] * X[0] + R[1, a] * X[1]) + R[2, a] * X[2]))"),
    "pose_origin_dropped": ("(o[a] + ((R[a, 0] * X[0] + R[a, 1] * X[1]) + R[a, 2] * X[2]))",
                            "(((R[a, 0] * X[0] + R[a, 1] * X[1]) + R[a, 2] * X[2]))"),
    "pose_spin_sign_x": ("ub_w[0] = rot_ub[0] + v[0] + (w[1] * r[2] - w[2] * r[1])",
                         "ub_w[0] = rot_ub[0] + v[0] - (w[1] * r[2] - w[2] * r[1])"),
    "pose_body_velocity_not_rotated": ("rot_ub = np.array([(R[a, 0] * ub[0] + R[a, 1] * ub[1]) + R[a, 2] * ub[2] for a in range(3)])",
                                       "rot_ub = ub"),
    "pose_lever_from_coordinate_origin": ("r = xyz.astype(np.float64) - o[:, None]", "r = xyz.astype(np.float64)"),
    "pose_drift_dropped": ("ub_w[1] = rot_ub[1] + v[1] + (w[2] * r[0] - w[0] * r[2])",
                           "ub_w[1] = rot_ub[1] + (w[2] * r[0] - w[0] * r[2])"),
}


def _run_py_pins(source: str, workdir: str, name: str, library: str) -> subprocess.CompletedProcess:
    """Pins of the Python part against a copy of the oracle package whose
    oracle.py is `source`, in a tree of its own (the committed files stay)."""
    root = os.path.join(workdir, name)
    os.makedirs(os.path.join(root, "oracle"))
    os.makedirs(os.path.join(root, "tests"))
    shutil.copy(os.path.join(ROOT, "oracle", "__init__.py"), os.path.join(root, "oracle", "__init__.py"))
    with open(os.path.join(root, "oracle", "oracle.py"), "w") as fh:
        fh.write(source)
    for f in ["conftest.py", *[os.path.basename(p) for p in PY_PINS]]:
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(root, "tests", f))
    env = dict(os.environ, LBM_ORACLE_LIBRARY=library, OMP_NUM_THREADS="2")
    return subprocess.run([sys.executable, "-m", "pytest", *PY_PINS, "-q", "-x", "-p", "no:cacheprovider"],
                          cwd=root, env=env, capture_output=True, text=True, timeout=600)


def _run_pins(source: str, workdir: str, name: str) -> subprocess.CompletedProcess:
    c = os.path.join(workdir, f"{name}.c")
    so = os.path.join(workdir, f"{name}.so")
    with open(c, "w") as fh:
        fh.write(source)
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", c, "-o", so, "-lm"], check=True,
                   capture_output=True)
    env = dict(os.environ, LBM_ORACLE_LIBRARY=so, OMP_NUM_THREADS="2")
    return subprocess.run([sys.executable, "-m", "pytest", *PINS, "-q", "-x", "-k", SKIP_SLOW, "-p", "no:cacheprovider"],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_every_planted_mistake_fails_a_pin():
    src = open(SRC).read()
    for name, (old, _) in MUTANTS.items():
        assert src.count(old) == 1, f"mutant {name}: its source text is not found exactly once"
    with tempfile.TemporaryDirectory() as td:
        control = _run_pins(src, td, "control")
        assert control.returncode == 0, "unmutated copy fails the pins:\n" + control.stdout[-2000:]
        with cf.ThreadPoolExecutor(4) as ex:
            futs = {name: ex.submit(_run_pins, src.replace(old, new), td, name)
                    for name, (old, new) in MUTANTS.items()}
            survivors = [name for name, fut in futs.items()
                         if fut.result().returncode == 0 or fut.result().returncode == 5]
    assert not survivors, f"mutants no pin catches: {survivors}"


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_every_planted_mistake_in_the_placement_fails_a_pin():
    from oracle import oracle as O
    library = O.build()
    src = open(PY_SRC).read()
    for name, (old, _) in PY_MUTANTS.items():
        assert src.count(old) == 1, f"mutant {name}: its source text is not found exactly once"
    with tempfile.TemporaryDirectory() as td:
        control = _run_py_pins(src, td, "control", library)
        assert control.returncode == 0, "unmutated copy fails the pins:\n" + control.stdout[-2000:]
        with cf.ThreadPoolExecutor(4) as ex:
            futs = {name: ex.submit(_run_py_pins, src.replace(old, new), td, name, library)
                    for name, (old, new) in PY_MUTANTS.items()}
            survivors = [name for name, fut in futs.items()
                         if fut.result().returncode == 0 or fut.result().returncode == 5]
    assert not survivors, f"mutants no pin catches: {survivors}"
