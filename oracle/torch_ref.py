"""Differentiable FP64 twin of the oracle's ADR step in plain PyTorch-CPU ops
(test infrastructure only).

It exists to obtain reference gradients d eps / d k(x) by autograd on small
grids.  The step is the same scheme as ``lbref.c`` (paper Eqs. LBE_ADE, BGK,
the second-order equilibrium, source_lbm applied to the populations that stream
into a catalytic node, Eq. BC at the inlet/outlet, half-way bounce-back at
solids), written with whole-array tensor operations instead of loops; the
CPU tests cross-check the two to round-off.

Objective: starting from a fixed pre-collision state g0, take T steps and
evaluate eps (Eq. A-B) from the outlet fluxes of the last streaming.
"""
from __future__ import annotations

import numpy as np
import torch
from torch.utils.checkpoint import checkpoint

CX = (0, 1, 0, -1, 0)
CY = (0, 0, 1, 0, -1)
WQ = (1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6)
OPP = (0, 3, 4, 1, 2)


def _shift(a, dx, dy):
    """b[..., y, x] = a[..., y - dy, x - dx], zero where the source is outside."""
    ny, nx = a.shape[-2:]
    b = torch.zeros_like(a)
    ys0, ys1 = max(0, dy), min(ny, ny + dy)
    xs0, xs1 = max(0, dx), min(nx, nx + dx)
    b[..., ys0:ys1, xs0:xs1] = a[..., ys0 - dy:ys1 - dy, xs0 - dx:xs1 - dx]
    return b


class Scheme:
    """Precomputed masks of one geometry; ``step`` is differentiable in k."""

    def __init__(self, node_type, ux, uy, nspecies, tau, c_in=1.0, vel_scale=1.0, xf=None):
        t = torch.as_tensor(np.asarray(node_type), dtype=torch.uint8)
        self.ny, self.nx = t.shape
        self.ns = nspecies
        self.tau = float(tau)
        self.c_in = float(c_in)
        self.xf = self.nx - 3 if xf is None else xf
        fluid = t == 0
        self.fluid = fluid.to(torch.float64)
        u = vel_scale * torch.as_tensor(np.asarray(ux), dtype=torch.float64)
        v = vel_scale * torch.as_tensor(np.asarray(uy), dtype=torch.float64)
        uu = u * u + v * v
        # equilibrium factor e_i(x) = w_i (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u)
        self.e = torch.stack([WQ[i] * (1 + 3 * (CX[i] * u + CY[i] * v)
                                       + 4.5 * (CX[i] * u + CY[i] * v) ** 2 - 1.5 * uu)
                              for i in range(5)])
        # links into catalysts: cat[i][type] is 1 at fluid x whose neighbour
        # x + c_i has that catalyst type
        tt = t.to(torch.int64)
        self.cat1, self.cat2 = [], []
        for i in range(5):
            nb = _shift(tt + 100, -CX[i], -CY[i]) - 100  # type of x + c_i (-100 outside)
            self.cat1.append(((nb == 2) & fluid).to(torch.float64))
            self.cat2.append(((nb == 3) & fluid & (nspecies == 3)).to(torch.float64))
        # streaming source classes for direction i at each fluid node
        xs = torch.arange(self.nx).expand(self.ny, self.nx)
        self.src_fluid, self.src_solid = [], []
        for i in range(5):
            sfl = _shift(fluid.to(torch.int64) + 10, CX[i], CY[i]) - 10  # fluid flag of x - c_i
            inside_x = (xs - CX[i] >= 0) & (xs - CX[i] < self.nx)
            self.src_fluid.append(((sfl == 1) & fluid & inside_x).to(torch.float64))
            self.src_solid.append(((sfl != 1) & fluid & inside_x).to(torch.float64))
        self.inlet = torch.zeros(self.ny, self.nx, dtype=torch.float64)
        self.inlet[:, 0] = self.fluid[:, 0]
        self.outlet = torch.zeros(self.ny, self.nx, dtype=torch.float64)
        self.outlet[:, -1] = self.fluid[:, -1]

    def step(self, g, k):
        """One step from pre-collision g [ns, 5, ny, nx] with rate map k [ny, nx]."""
        c = g.sum(1)                                        # [ns, ny, nx]
        post = g - (g - self.e.unsqueeze(0) * c.unsqueeze(1)) / self.tau
        post = post * self.fluid
        post = list(post.unbind(0))
        post = [list(p.unbind(0)) for p in post]
        for i in range(1, 5):
            k_nb = _shift(k, -CX[i], -CY[i])                 # k at x + c_i
            r1 = k_nb * WQ[i] * c[0] * self.cat1[i]
            post[0][i] = post[0][i] - r1
            post[1][i] = post[1][i] + r1
            if self.ns == 3:
                r2 = k_nb * WQ[i] * c[1] * self.cat2[i]
                post[1][i] = post[1][i] - r2
                post[2][i] = post[2][i] + r2
        out = []
        for s in range(self.ns):
            ps = post[s]
            cb = sum(ps)
            rows = [ps[0]]
            for i in range(1, 5):
                val = (self.src_fluid[i] * _shift(ps[i], CX[i], CY[i])
                       + self.src_solid[i] * ps[OPP[i]])
                if i == 1:  # E: inlet
                    if s == 0:
                        val = val + self.inlet * (-ps[3] + 2 * WQ[1] * self.c_in)
                    else:
                        val = val + self.inlet * ps[3]
                if i == 3:  # W: outlet, C_w = C_b
                    val = val + self.outlet * (-ps[1] + 2 * WQ[3] * cb)
                rows.append(val)
            out.append(torch.stack(rows))
        return torch.stack(out) * self.fluid

    def fluxes(self, g):
        """N_s of the last streaming through the face xf + 1/2."""
        a, b = self.xf, self.xf + 1
        both = self.fluid[:, a] * self.fluid[:, b]
        return ((g[:, 1, :, b] - g[:, 3, :, a]) * both).sum(-1)

    def efficiency(self, g):
        n = self.fluxes(g)
        return n[-1] / n.sum()


def eps_and_grad(node_type, k, ux, uy, g0, nspecies, tau, T, c_in=1.0, vel_scale=1.0,
                 segment=200):
    """eps after T steps from the fixed pre-collision state g0, and d eps / d k
    over the whole rate map (autograd, recomputing each segment of steps)."""
    sch = Scheme(node_type, ux, uy, nspecies, tau, c_in, vel_scale)
    kt = torch.tensor(np.asarray(k, dtype=np.float64), requires_grad=True)
    g = torch.as_tensor(np.asarray(g0, dtype=np.float64))

    def run(gs, kk, n):
        for _ in range(n):
            gs = sch.step(gs, kk)
        return gs

    done = 0
    while done < T:
        n = min(segment, T - done)
        g = checkpoint(run, g, kt, n, use_reentrant=False)
        done += n
    eps = sch.efficiency(g)
    eps.backward()
    return float(eps.detach()), kt.grad.numpy().copy(), g.detach().numpy()
