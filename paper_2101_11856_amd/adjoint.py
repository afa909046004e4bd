"""Gradients of a channel-flow objective through the hand-written adjoint of
lbm_step, exposed as a torch.autograd.Function.

Configuration (the adjoint channel): a 128 x 64 x 64 channel, no-slip walls in
y and z, inlet at -x with u_x(y, z) = 0.04 + sum_pq a_pq phi_pq(y, z) (16
sin-sin modes), outflow at +x, nu = 1e-3; a cylinder of radius 8 along z at
(32, 32) carried by immersed-boundary samples with per-sample gains gamma_s.

Objective (reading of the configuration, both terms on the final state):
  J = -F_x + sum over the probe plane x = 100 of |u0 - u_tgt|^2,
with F the total penalty force the next step would apply (force on the fluid,
so -F_x is the drag on the cylinder) and u0 = j / rho from lbm_macros.

Forward: n steps with a checkpoint every K steps (lbm_checkpoint).  Backward:
seeds on the final state, then for each segment in reverse: restore its
checkpoint, record the K forward states on a tape, and run lbm_adjoint_step.
Parameter gradients accumulate in FP64 on the device.  The mode synthesis of
the inlet profile and its transpose are the objective's parameterisation (two
small tensor contractions), not part of the solver.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lbm, synth


class ChannelProblem:
    def __init__(self, nx=128, ny=64, nz=64, nu=1e-3, steps=2000, checkpoint_every=100, storage="f32",
                 probe_x=100, u_tgt=(0.04, 0.0, 0.0), base=0.04, radius=8.0, center=(32.0, 32.0),
                 n_around=50, mode_length=64.0, device="cuda"):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.steps, self.K = steps, checkpoint_every
        self.probe_x, self.base = probe_x, base
        self.device = torch.device(device)
        self.u_tgt = torch.tensor(u_tgt, dtype=torch.float64, device=self.device)
        faces = (lbm.INLET, lbm.OUTFLOW, lbm.NOSLIP, lbm.NOSLIP, lbm.NOSLIP, lbm.NOSLIP)
        self.real = torch.float64 if storage == "f64" else torch.float32
        prof = np.zeros((3, nz, ny))
        prof[0] = base
        self.solver = lbm.Solver(nx, ny, nz, nu, faces=faces, inlet_profile=prof, storage=storage,
                                 device=device)
        xyz, ub, area, gain = synth.cylinder_markers(radius, center, nz, n_around)
        keep = xyz[2] < nz - 1          # stencils stay off the z walls
        self.xyz, self.ub, self.area = xyz[:, keep], ub[:, keep], area[keep]
        self.n = int(self.xyz.shape[1])
        self.solver.set_solids(self.xyz, self.ub, self.area, np.ones(self.n, np.float32))
        self.B = torch.as_tensor(synth.inlet_mode_basis(ny, nz, length=mode_length), dtype=torch.float64,
                                 device=self.device)                     # [16, nz, ny]
        rho, u = synth.uniform(nx, ny, nz, (base, 0.0, 0.0), dtype=np.float64)   # rounded to the storage type by the solver
        self._rho0, self._u0 = rho, u
        self.solver.adjoint_init()

    # parameterisation -------------------------------------------------------
    def profile(self, coeffs: torch.Tensor) -> torch.Tensor:
        prof = torch.zeros((3, self.nz, self.ny), dtype=torch.float64, device=self.device)
        prof[0] = self.base + torch.tensordot(coeffs.to(torch.float64), self.B, dims=1)
        return prof

    def set_params(self, coeffs, gains):
        self.solver.set_inlet_profile(self.profile(torch.as_tensor(coeffs, device=self.device)))
        self.solver.set_gains(torch.as_tensor(gains, device=self.device).to(torch.float32))

    # forward ------------------------------------------------------------------
    def run_forward(self, coeffs, gains, keep_checkpoints=True):
        """Run the forward steps from the equilibrium initial state.  Returns
        (drag, probe u0, record); the record holds what the reverse sweep of
        this run needs (its parameters, its checkpoints and its final state),
        so later forward runs on the same problem do not disturb it."""
        s = self.solver
        coeffs = torch.as_tensor(coeffs, device=self.device).detach().clone()
        gains = torch.as_tensor(gains, device=self.device).detach().clone()
        self.set_params(coeffs, gains)
        s.init_equilibrium(self._rho0, self._u0)
        checkpoints = []
        done = 0
        while done < self.steps:
            k = min(self.K, self.steps - done)
            if keep_checkpoints:
                checkpoints.append((s.checkpoint(), k))
            s.step(k)
            done += k
        F = s.ib_force_eval()
        _, u = s.macros()
        probe = u[:, :, :, self.probe_x].to(torch.float64)
        drag = torch.tensor(-F[0], dtype=torch.float64, device=self.device)
        record = ForwardRecord(coeffs, gains, checkpoints, s.checkpoint() if keep_checkpoints else None)
        return drag, probe, record

    def objective(self, drag, probe):
        return drag + ((probe - self.u_tgt[:, None, None]) ** 2).sum()

    # backward -----------------------------------------------------------------
    def run_backward(self, record: "ForwardRecord", g_drag: float, g_probe: torch.Tensor):
        """Reverse sweep of the forward run that produced `record`: its
        parameters and final state are put back first, then the seeds, then the
        segments in reverse order."""
        if record.final is None or not record.checkpoints:
            raise RuntimeError("this forward run kept no checkpoints (keep_checkpoints=False): no reverse sweep")
        s = self.solver
        nz, ny, nx = s.shape
        self.set_params(record.coeffs, record.gains)
        s.restore(record.final)
        g_inlet = s.new_grad_inlet()
        g_gain = s.new_grad_gain()
        s.adjoint_init()                                  # lambda = 0
        g_u = torch.zeros((3, nz, ny, nx), dtype=self.real, device=self.device)
        g_u[:, :, :, self.probe_x] = g_probe.to(self.real)
        s.adjoint_seed_macros(None, g_u, g_inlet)
        s.adjoint_seed_force((-float(g_drag), 0.0, 0.0), g_inlet, g_gain)
        tape = torch.empty((self.K, s.state_bytes()), dtype=torch.uint8, device=self.device)
        for snap, k in reversed(record.checkpoints):
            s.restore(snap)
            tape = s.record_tape(k, tape)
            s.adjoint_step(k, tape, g_inlet, g_gain)
        g_coeffs = torch.tensordot(self.B, g_inlet[0], dims=([1, 2], [0, 1]))
        return g_coeffs, g_gain[: self.n]


class ForwardRecord:
    """Parameters, checkpoints [(snapshot, steps)] and final-state snapshot of
    one forward run (device tensors owned by the record)."""

    def __init__(self, coeffs, gains, checkpoints, final):
        self.coeffs, self.gains = coeffs, gains
        self.checkpoints, self.final = checkpoints, final


class AdjointRun(torch.autograd.Function):
    """(inflow coefficients [16], sample gains [n]) -> (drag, probe-plane u0 [3, nz, ny]).

    Each application keeps its own forward record in the autograd context, so
    several forward runs on one problem may be taken before their backward
    passes, in any order."""

    @staticmethod
    def forward(ctx, problem: ChannelProblem, coeffs: torch.Tensor, gains: torch.Tensor):
        drag, probe, record = problem.run_forward(coeffs.detach(), gains.detach())
        ctx.problem = problem
        ctx.record = record
        ctx.dtypes = (coeffs.dtype, gains.dtype)
        return drag, probe

    @staticmethod
    def backward(ctx, g_drag, g_probe):
        p = ctx.problem
        gd = 0.0 if g_drag is None else float(g_drag)
        gp = torch.zeros((3, p.nz, p.ny), dtype=torch.float64, device=p.device) if g_probe is None else g_probe
        g_coeffs, g_gain = p.run_backward(ctx.record, gd, gp)
        ctx.record = None
        return None, g_coeffs.to(ctx.dtypes[0]), g_gain.to(ctx.dtypes[1])
