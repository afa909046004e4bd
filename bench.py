#!/usr/bin/env python3
"""Throughput of the D3Q27 central-moment MRT step on one MI355X.

Workload (the headline configuration): decaying turbulence on a 256^3 periodic
grid, no solids, FP32 populations, nu = 1e-4, equilibrium initialisation from
a seeded E(k) ~ k^-5/3 solenoidal field (rms u = 0.04, rho = 1 +- 1e-3).  A
"step" is one full time step of the method (pull streaming, macroscopic
values, central-moment collision, store) over all cells.

Prints one JSON line: MLUPS, the roofline of the fused kernel (algorithmic
bytes per launch / measured launch time, against 8 TB/s), the FP64 CPU oracle
timed on a bounded slab of the same field, and extra objects for the 16-bit
storage forms, the immersed-sphere, city, rotating-torus and adjoint workloads.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS (D3Q27 ACM-MRT+IBM), % HBM roofline; FP16-store vs FP32 at stated error"
HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "k_fused_turbulence256_f32_counters.txt")
# sources that decide the fused kernel's code and memory layout, the calibration copy, and the build flags
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2101_11856_amd", "csrc", f)
                  for f in ("lbm_step.hip", "lbm_step.hpp", "lbm_step_inst.hip", "lbm_internal.hpp", "lbm_api.hip",
                            "lbm_ctx.hpp", "lbm_aux.hip")]
KERNEL_SOURCES.append(os.path.join(ROOT, "paper_2101_11856_amd", "build.py"))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    if not os.path.exists(COUNTERS):
        return None
    text = open(COUNTERS).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != kernel_hash():
        return None
    return float(t.group(1))


def timed_steps(solver, steps, warmup):
    import torch
    solver.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(solver.stream)
    solver.step(steps)
    e1.record(solver.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def measured_copy(solver, reps=5):
    """Device copy bandwidth on this GPU: the library's plain 16-byte-per-lane
    copy (lbm_checkpoint) of the whole population state, read + write bytes
    over HIP-event time on the solver's stream."""
    import torch
    dst = solver.checkpoint()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(solver.stream)
    for _ in range(reps):
        solver.checkpoint(dst)
    e1.record(solver.stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3
    return 2 * solver.state_bytes() * reps / t / 1e9


def turbulence_solver(n, storage, rho, u, collision="cm"):
    from paper_2101_11856_amd import lbm
    s = lbm.Solver(n, n, n, 1e-4, storage=storage, collision=collision)
    s.init_equilibrium(rho, u)
    return s


def collision_models(n, rho, u, steps, warmup):
    """Cost of the collision models in the fused step (the paper's Sec. 5.1
    compares its central-moment model with BGK and raw-moment MRT): the
    headline workload per model and storage form.  "cm" is the default form
    (unit rates of orders 3-6, specialised), "cm_general" the general
    central-moment form at the same rates."""
    import torch
    out = {}
    for storage in ("f32", "f16"):
        for name, coll, env in (("cm", "cm", None), ("cm_general", "cm", "1"), ("bgk", "bgk", None),
                                ("rm", "rm", None)):
            old = os.environ.pop("LBM_CM_GENERAL", None)
            if env:
                os.environ["LBM_CM_GENERAL"] = env
            try:
                s = turbulence_solver(n, storage, rho, u, collision=coll)
            finally:
                os.environ.pop("LBM_CM_GENERAL", None)
                if old is not None:
                    os.environ["LBM_CM_GENERAL"] = old
            t = timed_steps(s, steps, warmup) / steps
            out[f"{name}_{storage}"] = {"ms_per_step": round(1e3 * t, 4), "MLUPS": round(n ** 3 / t / 1e6, 1)}
            del s
            torch.cuda.empty_cache()
    for storage in ("f32", "f16"):
        out[f"cm_over_bgk_time_{storage}"] = round(out[f"cm_{storage}"]["ms_per_step"] /
                                                   out[f"bgk_{storage}"]["ms_per_step"], 3)
    return out


def cpu_baseline(rho, u, n, budget_s=20.0):
    """FP64 oracle on a 256 x 256 x 32 periodic slab of the same field (about
    10-20 s of host work)."""
    import numpy as np

    from oracle import oracle as O
    nz = 32
    S = O.OracleSim(n, n, nz, 1e-4)
    S.init_equilibrium(rho[:nz].astype(np.float64), u[:, :nz].astype(np.float64))
    steps, t0 = 0, time.perf_counter()
    while steps < 8:
        S.step(1)
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    cells = n * n * nz
    return {"value": round(cells * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} step(s) of the FP64 oracle on a {n}x{n}x{nz} periodic slab of the same "
                      f"turbulence field ({cells} cells, {dt:.1f} s)"}


def step_roofline(cells, storage, band, samples, scalar, t_step):
    """HBM roofline of one whole step: algorithmic bytes per step (27 reads +
    27 writes per node; per band node its pulled populations, (rho, u) and
    force; per sample its position, velocity, area, gain, cell and spreading
    share; the scalar's read and write) over the measured step time."""
    b = 4 if storage == "f32" else 8 if storage == "f64" else 2
    byts = cells * 54 * b + band * (27 * b + 16 + 12) + samples * 52 + (8 * cells if scalar else 0)
    achieved = byts / t_step / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_step": int(byts),
            "scope": "whole step (all kernels)"}


def health(s, c0):
    """Mass drift since c0 and the non-finite check of the stored state."""
    from paper_2101_11856_amd import lbm
    try:
        c1 = s.conserved()
    except lbm.LbmError as e:
        return {"finite": False, "error": str(e)}
    return {"finite": True, "mass_drift_rel": float(abs(c1[0] - c0[0]) / c0[0])}


def sphere_workload(steps, warmup, storage="f32", n_sphere=13000, n_random=200000):
    import torch

    from paper_2101_11856_amd import lbm, synth
    nx, ny, nz = 512, 128, 128
    s = lbm.Solver(nx, ny, nz, 5e-5, faces=(lbm.INLET, lbm.OUTFLOW, 0, 0, 0, 0), u_in=(0.05, 0.0, 0.0),
                   storage=storage)
    rho, u = synth.uniform(nx, ny, nz, (0.05, 0.0, 0.0))
    s.init_equilibrium(rho, u)
    xyz, ub, area, gain = synth.sphere_scene(n_sphere=n_sphere, n_random=n_random)
    s.set_solids(xyz, ub, area, gain)
    band = int((s.solid_maps()[0] & 1).sum())
    c0 = s.conserved()
    t = timed_steps(s, steps, warmup)
    F = s.ib_force()
    what = f"{n_sphere} sphere + {n_random} random samples" if n_random else f"{n_sphere} sphere samples"
    out = {"workload": f"flow past an immersed sphere 512x128x128, inlet/outflow, {what}, {storage.upper()}",
           "value": round(nx * ny * nz * steps / t / 1e6, 1),
           "unit": "MLUPS", "ms_per_step": round(1e3 * t / steps, 4), "samples": int(xyz.shape[1]),
           "band_nodes": band, "drag_x": float(-F[0]),
           "roofline": step_roofline(nx * ny * nz, storage, band, int(xyz.shape[1]), False, t / steps),
           "health": health(s, c0)}
    del s
    torch.cuda.empty_cache()
    return out


def dense_sphere_workload(steps, warmup, n_sphere=150000):
    """The sphere of the sphere workload sampled at the paper's density
    (Sec. 3.1: 10-100 samples per near-boundary cell): 150,000 Fibonacci
    samples, no random box.  Timed with the default wavefront-scan spreading
    and with one lane per run, next to the same grid with no samples; the
    run-length statistics are those of the sorted samples."""
    import numpy as np
    import torch

    from paper_2101_11856_amd import lbm, synth
    nx, ny, nz = 512, 128, 128
    xyz, ub, area, gain = synth.sphere_scene(n_sphere=n_sphere, n_random=0)
    rho, u = synth.uniform(nx, ny, nz, (0.05, 0.0, 0.0))

    def run(samples, lane_per_run=False):
        old = os.environ.pop("LBM_IB_LANE_PER_RUN", None)
        if lane_per_run:
            os.environ["LBM_IB_LANE_PER_RUN"] = "1"
        try:
            s = lbm.Solver(nx, ny, nz, 5e-5, faces=(lbm.INLET, lbm.OUTFLOW, 0, 0, 0, 0), u_in=(0.05, 0.0, 0.0))
        finally:
            os.environ.pop("LBM_IB_LANE_PER_RUN", None)
            if old is not None:
                os.environ["LBM_IB_LANE_PER_RUN"] = old
        s.init_equilibrium(rho, u)
        info = {}
        if samples:
            s.set_solids(xyz, ub, area, gain)
            fl, cell, perm = (t.cpu().numpy() for t in s.solid_maps())
            info["band"] = int((fl & 1).sum())
            sc = cell[perm]                                   # base cell of each sorted sample
            _, counts = np.unique(sc, return_counts=True)
            info["per_cell"] = counts
            starts = np.r_[0, np.flatnonzero(np.diff(sc)) + 1]
            lens = np.diff(np.r_[starts, sc.size])            # samples per cell in sorted order
            w = lens[: lens.size // 64 * 64].reshape(-1, 64)  # 64 cells per wavefront of the lane-per-run form
            info["wave_max_over_mean"] = float((w.max(axis=1) / w.mean(axis=1)).mean())
            info["F"] = None
        t = timed_steps(s, steps, warmup)
        if samples:
            info["F"] = s.ib_force()
        del s
        torch.cuda.empty_cache()
        return t / steps, info

    t_plain, _ = run(False)
    t_seg, info = run(True)
    t_lpr, info2 = run(True, lane_per_run=True)
    pc = info["per_cell"]
    return {"workload": f"immersed sphere 512x128x128 at the paper's sampling density, {n_sphere} samples, FP32",
            "value": round(nx * ny * nz / t_seg / 1e6, 1), "unit": "MLUPS", "ms_per_step": round(1e3 * t_seg, 4),
            "samples": int(xyz.shape[1]), "band_nodes": info["band"],
            "samples_per_base_cell": {"mean": round(float(pc.mean()), 1), "max": int(pc.max()),
                                      "p10": float(np.percentile(pc, 10)), "p90": float(np.percentile(pc, 90))},
            "lane_per_run_wave_max_over_mean_run": round(info["wave_max_over_mean"], 2),
            "no_samples_ms_per_step": round(1e3 * t_plain, 4),
            "ib_share_of_step": round((t_seg - t_plain) / t_seg, 4),
            "lane_per_run_ms_per_step": round(1e3 * t_lpr, 4),
            "lane_per_run_ib_share_of_step": round((t_lpr - t_plain) / t_lpr, 4),
            "drag_x": float(-info["F"][0]), "drag_x_lane_per_run": float(-info2["F"][0]),
            "roofline": step_roofline(nx * ny * nz, "f32", info["band"], int(xyz.shape[1]), False, t_seg)}


def city_workload(steps, warmup, storage="f32"):
    """City blocks 1200x250x840 (252M cells): inlet wind, no-slip ground,
    free-slip top, periodic z, 400 boxes with 3.86M samples, passive scalar."""
    import torch

    from paper_2101_11856_amd import lbm, synth
    nx, ny, nz = 1200, 250, 840
    s = lbm.Solver(nx, ny, nz, 1e-5, faces=(lbm.INLET, lbm.OUTFLOW, lbm.NOSLIP, lbm.FREESLIP, 0, 0),
                   u_in=(0.05, 0.0, 0.0), storage=storage, scalar=True, scalar_inlet_height=50)
    rho = torch.ones((nz, ny, nx), dtype=torch.float32, device="cuda")
    u = torch.zeros((3, nz, ny, nx), dtype=torch.float32, device="cuda")
    u[0] = 0.05
    s.init_equilibrium(rho, u)
    del rho, u
    s.set_scalar(torch.zeros((nz, ny, nx), dtype=torch.float32, device="cuda"))
    xyz, ub, area, gain = synth.city_markers(synth.city_boxes())
    s.set_solids(xyz, ub, area, gain)
    band = int((s.solid_maps()[0] & 1).sum())
    c0 = s.conserved()
    t = timed_steps(s, steps, warmup)
    cells = nx * ny * nz
    out = {"workload": f"city blocks 1200x250x840, {xyz.shape[1]} samples, passive scalar, {storage.upper()}",
           "value": round(cells * steps / t / 1e6, 1), "unit": "MLUPS", "ms_per_step": round(1e3 * t / steps, 3),
           "samples": int(xyz.shape[1]), "band_nodes": band, "cells": cells,
           "population_bytes": 2 * 27 * cells * (4 if storage == "f32" else 2),
           "roofline": step_roofline(cells, storage, band, int(xyz.shape[1]), True, t / steps),
           "health": dict(health(s, c0), steps=warmup + steps)}
    del s
    torch.cuda.empty_cache()
    return out


def moving_torus_workload(steps, warmup):
    """Rotating torus in air, 400x200x400 periodic (the paper's rotating-torus
    scene size): torus major radius 48, minor 16, 273k samples, tilted 0.5 rad
    about x and turning about its own axis at rim speed 0.05.  Every step
    places the samples at the new pose (rigid update, re-sort, re-band) and
    then advances; timed by the host clock around whole steps (a device
    synchronisation on both sides).  The same scene held still gives the
    share of the re-placement."""
    import numpy as np
    import torch

    from paper_2101_11856_amd import lbm, synth
    nx, ny, nz = 400, 200, 400
    X, area = synth.torus_body(48.0, 16.0)
    n = X.shape[1]
    ub = np.zeros((3, n), np.float32)
    gain = np.ones(n, np.float32)
    tilt = synth.rotation((1.0, 0.0, 0.0), 0.5)
    axis = tilt @ np.array([0.0, 0.0, 1.0])
    rate = 0.05 / 64.0
    o = (200.0, 100.0, 200.0)
    w = rate * axis

    def pose(t):
        return synth.rotation(axis, rate * t) @ tilt, o, (0.0, 0.0, 0.0), w

    s = lbm.Solver(nx, ny, nz, 1e-4)
    rho, u = synth.uniform(nx, ny, nz)
    s.init_equilibrium(rho, u)
    s.set_body(X, ub, area, gain, *pose(0))
    band0 = int((s.solid_maps()[0] & 1).sum())
    t_static = timed_steps(s, steps, warmup)
    for k in range(warmup):
        s.set_pose(*pose(k))
        s.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        s.set_pose(*pose(warmup + k))
        s.step(1)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    T = s.ib_torque()
    cells = nx * ny * nz
    out = {"workload": f"rotating torus 400x200x400, {n} samples re-placed, re-sorted and re-banded every step, FP32",
           "value": round(cells * steps / t / 1e6, 1), "unit": "MLUPS", "ms_per_step": round(1e3 * t / steps, 4),
           "static_ms_per_step": round(1e3 * t_static / steps, 4),
           "replace_ms_per_step": round(1e3 * (t - t_static) / steps, 4),
           "samples": n, "band_nodes_at_start": band0, "torque_on_fluid": [float(x) for x in T],
           "roofline": dict(step_roofline(cells, "f32", band0, n, False, t / steps),
                            scope="whole moving step (re-placement included, its bytes not counted)"),
           "roofline_static": step_roofline(cells, "f32", band0, n, False, t_static / steps)}
    del s
    torch.cuda.empty_cache()
    return out


def oracle_errors(steps=100, n=64):
    """Part of the CPU-baseline leg (the only leg that runs the oracle): error
    of each storage form against the FP64 oracle, on the same seeded inputs:
    the turbulence generator on an n^3 periodic box (the headline's field at
    reduced size), and an immersed-boundary scene at the paper's sampling
    density (70x18x16 channel, inlet/outflow, no-slip and free-slip walls; a
    sphere with about 44 samples per base cell plus a cluster of about 375 per
    cell).  rel-L2 over all nodes after `steps` steps."""
    import numpy as np
    import torch

    from oracle import oracle as O
    from paper_2101_11856_amd import lbm, synth

    def rel(a, b):
        return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))

    out = {}
    rho, u = synth.turbulence(n)
    S = O.OracleSim(n, n, n, 1e-4)
    S.init_equilibrium(rho.astype(np.float64), u.astype(np.float64))
    S.step(steps)
    r_ref, u_ref = S.macros()
    res = {}
    for storage in ("f32", "f16", "bf16"):
        sv = lbm.Solver(n, n, n, 1e-4, storage=storage)
        sv.init_equilibrium(rho, u)
        sv.step(steps)
        r, uu = (t.cpu().double().numpy() for t in sv.macros())
        res[storage] = {"u_rel_l2": rel(uu, u_ref), "rho_rel_l2": rel(r, r_ref)}
        del sv
    out["turbulence"] = {"case": f"turbulence {n}^3 periodic, nu=1e-4, {steps} steps", **res}

    nx, ny, nz = 70, 18, 16
    faces = (lbm.INLET, lbm.OUTFLOW, lbm.NOSLIP, lbm.FREESLIP, 0, 0)
    rng = np.random.default_rng(31)
    sph = synth.fibonacci_sphere(20000, 5.0, (14.3, ny / 2 + 0.2, nz / 2 - 0.1))
    clu = synth.random_box(3000, (40.0, 8.0, 7.0), (42.0, 10.0, 9.0), 32)
    xyz = np.concatenate([sph, clu], axis=1)
    m = xyz.shape[1]
    ub = np.zeros((3, m), np.float32)
    area = np.concatenate([np.full(20000, 4 * np.pi * 25.0 / 20000), np.full(3000, 8.0 / 3000)]).astype(np.float32)
    gain = np.ones(m, np.float32)
    rho = (1.0 + 1e-3 * rng.standard_normal((nz, ny, nx))).astype(np.float32)
    u = np.zeros((3, nz, ny, nx), np.float32)
    u[0] = 0.03
    S = O.OracleSim(nx, ny, nz, 1e-3, faces=faces, u_in=(0.03, 0, 0))
    S.set_markers(xyz, ub.astype(np.float64), area.astype(np.float64), gain.astype(np.float64))
    S.init_equilibrium(rho.astype(np.float64), u.astype(np.float64))
    S.step(steps)
    r_ref, u_ref = S.macros()
    F_ref = S.last_force()
    res = {}
    for storage in ("f32", "f16", "bf16"):
        sv = lbm.Solver(nx, ny, nz, 1e-3, storage=storage, faces=faces, u_in=(0.03, 0, 0))
        sv.set_solids(xyz, ub, area, gain)
        sv.init_equilibrium(rho, u)
        sv.step(steps)
        r, uu = (t.cpu().double().numpy() for t in sv.macros())
        res[storage] = {"u_rel_l2": rel(uu, u_ref), "rho_rel_l2": rel(r, r_ref),
                        "force_rel": rel(sv.ib_force(), F_ref)}
        del sv
    torch.cuda.empty_cache()
    out["immersed_dense"] = {"case": f"70x18x16 channel, {m} samples (sphere ~44 per base cell, cluster ~375 per "
                                     f"cell), nu=1e-3, {steps} steps", **res}
    out["note"] = "the gate of the 16-bit forms is u rel-L2 <= 1e-3 in these terms; FP32 <= 1e-5"
    return out


def adjoint_workload(steps=2000, every=100):
    """Adjoint channel 128x64x64, cylinder samples: forward with checkpoints,
    then the reverse sweep (segment recompute + adjoint steps)."""
    import torch

    from paper_2101_11856_amd import synth
    from paper_2101_11856_amd.adjoint import AdjointRun, ChannelProblem
    p = ChannelProblem(steps=steps, checkpoint_every=every)
    a = torch.tensor(synth.inlet_coefficients(seed=2105), dtype=torch.float64, device="cuda", requires_grad=True)
    g = torch.ones(p.n, dtype=torch.float64, device="cuda", requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    drag, probe = AdjointRun.apply(p, a, g)
    J = p.objective(drag, probe)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    cells = p.nx * p.ny * p.nz
    return {"workload": f"adjoint channel 128x64x64, {p.n} cylinder samples, {steps} steps, checkpoint every {every}, "
                        "FP32", "forward_ms_per_step": round(1e3 * (t1 - t0) / steps, 4),
            "backward_ms_per_step": round(1e3 * (t2 - t1) / steps, 4),
            "backward_MLUPS": round(cells * steps / (t2 - t1) / 1e6, 1),
            "note": "backward = segment recompute with tape + adjoint step; wall clock incl. host launch overhead",
            "J": float(J), "grad_norm_coeffs": float(a.grad.norm())}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed steps (the turbulence workload's 1000)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="grid edge of the turbulence workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the 16-bit and sphere runs")
    ap.add_argument("--storage", default="f32", help="population storage of --profile-pass")
    ap.add_argument("--profile-pass", action="store_true",
                    help="profiler pass: the workload only, then 3 state copies of known size (calibration)")
    ap.add_argument("--workload", default="turbulence",
                    choices=["turbulence", "sphere", "sphere_dense", "city", "moving_torus", "adjoint"],
                    help="workload of --profile-pass")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1 "
                                   "(the multi-GPU slab decomposition is a design, not a measured path)"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2101_11856_amd import synth

    if args.profile_pass and args.workload == "sphere":
        print(json.dumps(sphere_workload(args.steps, args.warmup, args.storage)), flush=True)
        return
    if args.profile_pass and args.workload == "sphere_dense":
        print(json.dumps(dense_sphere_workload(args.steps, args.warmup)), flush=True)
        return
    if args.profile_pass and args.workload == "moving_torus":
        print(json.dumps(moving_torus_workload(args.steps, args.warmup)), flush=True)
        return
    if args.profile_pass and args.workload == "adjoint":
        print(json.dumps(adjoint_workload(args.steps, min(args.steps, 100))), flush=True)
        return
    if args.profile_pass and args.workload == "city":
        print(json.dumps(city_workload(args.steps, args.warmup, args.storage)), flush=True)
        return

    n = args.n
    log(f"generating turbulence field {n}^3")
    rho, u = synth.turbulence(n)
    cells = n ** 3

    if args.profile_pass:
        s = turbulence_solver(n, args.storage, rho, u)
        t = timed_steps(s, args.steps, args.warmup)
        snap = s.checkpoint()
        for _ in range(3):
            s.checkpoint(snap)
        torch.cuda.synchronize()
        print(json.dumps({"profile_pass": True, "storage": args.storage, "n": n, "steps": args.steps,
                          "ms_per_step": 1e3 * t / args.steps, "copy_bytes_each_way": s.state_bytes(),
                          "kernel_source_sha256_16": kernel_hash()}), flush=True)
        return

    log("fp32 run")
    s = turbulence_solver(n, "f32", rho, u)
    c0 = s.conserved()
    torch.cuda.synchronize()
    t = timed_steps(s, args.steps, args.warmup)
    c1 = s.conserved()
    _, u32 = s.macros()
    u32 = u32.cpu().numpy()
    mlups = cells * args.steps / t / 1e6
    copy_gbs = measured_copy(s)
    t_launch = t / args.steps          # only the fused kernel runs in this workload
    bytes_launch = 27 * 2 * 4 * cells  # algorithmic: read + write 27 FP32 per cell
    achieved = bytes_launch / t_launch / 1e9
    traffic = measured_traffic()
    result = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_launch, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"decaying turbulence {n}^3 periodic, no solids, FP32 populations, nu=1e-4",
                   "cells": cells, "nu": 1e-4, "storage": "f32"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / t_launch / 1e9, 1),
                     "kernel": "k_fused<f32>", "algorithmic_bytes_per_launch": bytes_launch,
                     "copy_measured_GBs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)},
        "mass_drift_rel": float(abs(c1[0] - c0[0]) / c0[0]),
    }
    del s
    torch.cuda.empty_cache()

    if not args.no_extras:
        def u_after(storage, k):
            sk = turbulence_solver(n, storage, rho, u)
            sk.step(k)
            uk = sk.macros()[1].cpu().numpy()
            del sk
            torch.cuda.empty_cache()
            return uk
        u32_100 = u_after("f32", 100)
        for storage in ("f16", "bf16"):
            log(f"{storage} run")
            s = turbulence_solver(n, storage, rho, u)
            t16 = timed_steps(s, args.steps, args.warmup)
            _, u16 = s.macros()
            u16 = u16.cpu().numpy()
            m16 = cells * args.steps / t16 / 1e6
            err = float(np.linalg.norm(u16 - u32) / np.linalg.norm(u32))
            del s
            torch.cuda.empty_cache()
            u16_100 = u_after(storage, 100)
            err100 = float(np.linalg.norm(u16_100 - u32_100) / np.linalg.norm(u32_100))
            result[f"{storage}_storage"] = {
                "value": round(m16, 1), "unit": "MLUPS", "ratio_vs_f32": round(m16 / mlups, 3),
                "ms_per_step": round(1e3 * t16 / args.steps, 4),
                "achieved_GBs": round(27 * 2 * 2 * cells / (t16 / args.steps) / 1e9, 1),
                "vel_rel_l2_vs_f32_gpu_100_steps": err100,
                f"vel_rel_l2_vs_f32_gpu_{args.warmup + args.steps}_steps": err,
                "error_note": "u of this storage form against the FP32 run from the same initial state (the FP32 "
                              "run matches the FP64 oracle to <= 1e-5); the gate's terms are 100 steps"}
        log("collision models")
        result["collision_models"] = collision_models(n, rho, u, args.steps, args.warmup)
        log("sphere run")
        result["ib_sphere"] = sphere_workload(min(args.steps, 2000), min(args.warmup, 10))
        result["ib_sphere_f16"] = sphere_workload(min(args.steps, 2000), min(args.warmup, 10), "f16")
        result["ib_sphere_f16"]["ratio_vs_f32"] = round(result["ib_sphere_f16"]["value"] / result["ib_sphere"]["value"], 3)
        log("dense sphere run")
        result["ib_sphere_dense"] = dense_sphere_workload(min(args.steps, 2000), min(args.warmup, 10))
        for storage in ("f32", "f16"):
            log(f"city run {storage}")
            result[f"city_{storage}"] = city_workload(min(args.steps, 100), min(args.warmup, 5), storage)
        result["city_f16"]["ratio_vs_f32"] = round(result["city_f16"]["value"] / result["city_f32"]["value"], 3)
        log("moving torus run")
        result["moving_torus"] = moving_torus_workload(min(args.steps, 300), min(args.warmup, 10))
        log("adjoint run")
        result["adjoint_channel"] = adjoint_workload()

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(rho, u, n)
        if not args.no_extras:
            log("errors against the FP64 oracle (cpu baseline leg)")
            result["errors_vs_fp64_oracle"] = oracle_errors()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
