"""Test infrastructure, not product code: a second FP64 model of the time
step, written in plain PyTorch CPU ops so that ``torch.autograd`` can
differentiate it exactly.  Only tests may import it.

It is independent of both the C oracle and the HIP library: its own
velocity order (a plain product order), dense per-node moment matrices
T(u) solved with ``torch.linalg.solve``, and index-gather streaming.  It
covers what the adjoint tests need: pull streaming with the face rules,
Eq. (2) macros, the immersed-boundary interpolation, penalty and
spreading of Eqs. (6)-(8), the central-moment collision of Eqs. (4)-(5)
with Guo forcing in moment space, and the channel objective (drag plus
probe-plane velocity mismatch, both on the final state).

The readings are the same as the oracle's:
  * faces: no-slip = halfway bounce-back, inlet (-x) = bounce-back plus
    2 w_i (c_i . u_in) / cs^2, outflow (+x) = the value pulled one node
    inward, free-slip = specular reflection; precedence no-slip > inlet >
    outflow > free-slip > periodic (Sec. 4.3.3);
  * second-order moments relax as the deviatoric combinations at s_nu and
    the trace at s_bulk; orders 3..6 at s_high[order - 3]; orders 0 and 1
    are conserved; u = (j + F/2) / rho; u0 = j / rho for the immersed
    boundary (Sec. 2.1 and 2.2);
  * the force moments are F_a cs^(2 * number of twos) for exponent vectors
    with exactly one 1, zero otherwise.
"""
import itertools

import torch

PERIODIC, NOSLIP, FREESLIP, INLET, OUTFLOW = 0, 1, 2, 3, 4
_RANK = {PERIODIC: 0, FREESLIP: 1, OUTFLOW: 2, INLET: 3, NOSLIP: 4}
CS2 = 1.0 / 3.0
DT = torch.float64

# velocities: index = (cx+1) + 3 (cy+1) + 9 (cz+1); the opposite of i is 26 - i
CV = torch.tensor([(cx, cy, cz) for cz, cy, cx in itertools.product((-1, 0, 1), repeat=3)], dtype=DT)
_W1 = {-1: 1.0 / 6.0, 0: 2.0 / 3.0, 1: 1.0 / 6.0}
W = torch.tensor([_W1[int(a)] * _W1[int(b)] * _W1[int(c)] for a, b, c in CV.tolist()], dtype=DT)
# moment exponents (a_x, a_y, a_z) in {0,1,2}^3
EXPO = torch.tensor([(ax, ay, az) for az, ay, ax in itertools.product((0, 1, 2), repeat=3)], dtype=torch.long)


def _index(c):
    return (c[0] + 1) + 3 * (c[1] + 1) + 9 * (c[2] + 1)


def _relaxation_matrix(s_nu, s_bulk, s_high):
    """S = C^-1 D C: the rates act on combinations of the central moments
    (the order-2 trace and deviators, everything else one moment each)."""
    order = EXPO.sum(1)
    comb = torch.eye(27, dtype=DT)
    rate = torch.zeros(27, dtype=DT)
    for m in range(27):
        o = int(order[m])
        if o >= 3:
            rate[m] = s_high[o - 3]
    idx = {tuple(EXPO[m].tolist()): m for m in range(27)}
    a, b, c = idx[(2, 0, 0)], idx[(0, 2, 0)], idx[(0, 0, 2)]
    comb[a] = 0.0
    comb[a, [a, b, c]] = 1.0                       # trace
    comb[b] = 0.0
    comb[b, a], comb[b, b] = 1.0, -1.0             # k200 - k020
    comb[c] = 0.0
    comb[c, a], comb[c, c] = 1.0, -1.0             # k200 - k002
    rate[a], rate[b], rate[c] = s_bulk, s_nu, s_nu
    for e in ((1, 1, 0), (1, 0, 1), (0, 1, 1)):
        rate[idx[e]] = s_nu
    return torch.linalg.solve(comb, torch.diag(rate) @ comb)


class Channel:
    """Grid, faces and immersed samples of one problem; ``run`` maps
    (inlet profile, gains) to the objective as a differentiable graph."""

    def __init__(self, nx, ny, nz, nu, faces, xyz, ub, area, s_bulk=1.0, s_high=(1.0, 1.0, 1.0, 1.0)):
        self.n = (nx, ny, nz)
        self.N = nx * ny * nz
        self.faces = tuple(faces)
        self.S = _relaxation_matrix(1.0 / (3.0 * nu + 0.5), s_bulk, s_high)
        self._build_pull()
        self._build_markers(xyz, ub, area)
        e = EXPO
        nones = (e == 1).sum(1)
        ntwos = (e == 2).sum(1)
        self.eq_mask = torch.where(nones == 0, CS2 ** ntwos.to(DT), torch.zeros((), dtype=DT))
        # force moment m picks F along the axis whose exponent is 1
        self.force_axis = torch.where(nones == 1, (e == 1).to(torch.long).argmax(1), torch.full_like(nones, -1))
        self.force_scale = torch.where(nones == 1, CS2 ** ntwos.to(DT), torch.zeros((), dtype=DT))

    # -- streaming --------------------------------------------------------------
    def _pull_rule(self, i, p):
        """(source direction, source node, inlet node (y, z) or None, direction of the inlet term)."""
        c = [int(v) for v in CV[i].tolist()]
        src = [p[a] - c[a] for a in range(3)]
        best, brank, baxis, bside = PERIODIC, 0, -1, 0
        crossed = [False] * 3
        for a in range(3):
            if 0 <= src[a] < self.n[a]:
                continue
            side = 0 if src[a] < 0 else 1
            fc = self.faces[2 * a + side]
            if fc == PERIODIC:
                src[a] %= self.n[a]
                continue
            crossed[a] = True
            if _RANK[fc] > brank:
                best, brank, baxis, bside = fc, _RANK[fc], a, side
        lin = lambda q: q[0] + self.n[0] * (q[1] + self.n[1] * q[2])
        if best == PERIODIC:
            return i, lin(src), None
        if best == NOSLIP:
            return 26 - i, lin(p), None
        if best == INLET:
            return 26 - i, lin(p), (p[1], p[2])
        if best == OUTFLOW:
            q = list(p)
            q[baxis] += -1 if bside else 1
            return self._pull_rule(i, q)
        cr = [(-c[a] if crossed[a] else c[a]) for a in range(3)]
        q = [(p[a] if crossed[a] else src[a]) for a in range(3)]
        return _index(cr), lin(q), None

    def _build_pull(self):
        nx, ny, nz = self.n
        N = self.N
        gather = torch.empty((27, N), dtype=torch.long)
        inlet_dir, inlet_node, inlet_yz = [], [], []
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    k = x + nx * (y + ny * z)
                    for i in range(27):
                        d, s, yz = self._pull_rule(i, (x, y, z))
                        gather[i, k] = d * N + s
                        if yz is not None:
                            inlet_dir.append(i)
                            inlet_node.append(k)
                            inlet_yz.append(yz[0] + ny * yz[1])
        self.gather = gather.reshape(-1)
        self.inlet_dir = torch.tensor(inlet_dir, dtype=torch.long)
        self.inlet_flat = self.inlet_dir * N + torch.tensor(inlet_node, dtype=torch.long)
        self.inlet_yz = torch.tensor(inlet_yz, dtype=torch.long)

    def pull(self, f, u_in):
        """f*_i(x) = f_i(x - c_i) with the face rules; u_in is [3, nz*ny]."""
        fs = f.reshape(-1)[self.gather]
        if self.inlet_flat.numel():
            cu = (CV[self.inlet_dir] * u_in[:, self.inlet_yz].T).sum(1)
            fs = fs.index_add(0, self.inlet_flat, 2.0 * W[self.inlet_dir] * cu / CS2)
        return fs.reshape(27, self.N)

    # -- immersed boundary ----------------------------------------------------------
    def _build_markers(self, xyz, ub, area):
        """Base cells, trilinear weights and stencil nodes; positions are FP32."""
        p = torch.as_tensor(xyz, dtype=torch.float32)
        b = torch.floor(p)
        t = (p - b).to(DT)
        b = b.to(torch.long)
        nodes, weights = [], []
        for dz, dy, dx in itertools.product((0, 1), repeat=3):
            d = (dx, dy, dz)
            wt = torch.ones(p.shape[1], dtype=DT)
            q = []
            for a in range(3):
                wt = wt * (1.0 - (t[a] - d[a]).abs())
                q.append((b[a] + d[a]) % self.n[a])
            nodes.append(q[0] + self.n[0] * (q[1] + self.n[1] * q[2]))
            weights.append(wt)
        self.m_node = torch.stack(nodes)           # [8, n]
        self.m_w = torch.stack(weights)            # [8, n]
        self.ub = torch.as_tensor(ub, dtype=DT)
        self.area = torch.as_tensor(area, dtype=DT)

    def penalty(self, rho, u0, gain):
        """Eqs. (6)-(7): g_s = gain_s rho_s (u_b - u_s)."""
        rs = (self.m_w * rho[self.m_node]).sum(0)
        us = (self.m_w[None] * u0[:, self.m_node]).sum(1)
        return gain * rs * (self.ub - us)

    def spread(self, G):
        """Eq. (8): g(x_f) = sum_s a_s K_s(x_f) g_s."""
        src = (self.area * G)[:, None, :] * self.m_w[None]             # [3, 8, n]
        return torch.zeros((3, self.N), dtype=DT).index_add(1, self.m_node.reshape(-1), src.reshape(3, -1))

    # -- collision --------------------------------------------------------------------
    def collide(self, fs, rho, j, F):
        u = (j + 0.5 * F) / rho
        d = CV.T[None, :, :] - u.T[:, :, None]                             # [N, 3(axis), 27(i)]
        powers = torch.stack([torch.ones_like(d), d, d * d], dim=-1)       # [N, 3, 27, 3]
        T = torch.ones((self.N, 27, 27), dtype=DT)
        for a in range(3):
            T = T * powers[:, a][:, :, EXPO[:, a]].transpose(1, 2)        # [N, m, i]
        kappa = torch.einsum("nmi,in->nm", T, fs)
        keq = rho[:, None] * self.eq_mask[None]
        Fm = torch.where(self.force_axis[None] >= 0,
                         F.T[:, self.force_axis.clamp(min=0)] * self.force_scale[None], torch.zeros((), dtype=DT))
        kpost = kappa - (kappa - keq) @ self.S.T + Fm - 0.5 * (Fm @ self.S.T)
        return torch.linalg.solve(T, kpost.unsqueeze(-1)).squeeze(-1).T    # [27, N]

    # -- driver -------------------------------------------------------------------------
    def equilibrium(self, rho, u):
        """f_i = rho prod_a phi_{c_ia}(u_a): phi_0 = 2/3 - u^2, phi_{+-1} = (1/3 +- u + u^2)/2."""
        f = rho[None].expand(27, -1).clone()
        for a in range(3):
            c = CV[:, a][:, None]
            ua = u[a][None]
            phi = torch.where(c == 0, 2.0 / 3.0 - ua * ua, 0.5 * (1.0 / 3.0 + c * ua + ua * ua))
            f = f * phi
        return f

    def macros(self, fs):
        rho = fs.sum(0)
        j = CV.T @ fs
        return rho, j

    def step(self, f, u_in, gain):
        fs = self.pull(f, u_in)
        rho, j = self.macros(fs)
        G = self.penalty(rho, j / rho, gain)
        F = self.spread(G)
        return self.collide(fs, rho, j, F)

    def objective(self, f, u_in, gain, probe_x, u_tgt):
        """-F_x of the next step's immersed-boundary force, plus the squared
        mismatch of u0 on the plane x = probe_x; both from the state f."""
        fs = self.pull(f, u_in)
        rho, j = self.macros(fs)
        u0 = j / rho
        G = self.penalty(rho, u0, gain)
        Fx = (self.area * G[0]).sum()
        nx, ny, nz = self.n
        probe = u0.reshape(3, nz, ny, nx)[:, :, :, probe_x]
        tgt = torch.as_tensor(u_tgt, dtype=DT)[:, None, None]
        return -Fx + ((probe - tgt) ** 2).sum()

    def run(self, u_in, gain, steps, rho0, u0, probe_x, u_tgt=(0.04, 0.0, 0.0)):
        f = self.equilibrium(torch.as_tensor(rho0, dtype=DT).reshape(-1),
                             torch.as_tensor(u0, dtype=DT).reshape(3, -1))
        for _ in range(steps):
            f = self.step(f, u_in, gain)
        return self.objective(f, u_in, gain, probe_x, u_tgt)
