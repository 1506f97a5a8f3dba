"""Steady state of the ADR lattice-Boltzmann scheme by a direct sparse solve
(test infrastructure only).

For a frozen velocity field and fixed rates, one step of the scheme (paper
Eqs. LBE_ADE, BGK, source_lbm with Eq. BC at the inlet and outlet) is an
affine map of the pre-collision populations,

    g(t+1) = A g(t) + b,    A = S L,

with L block-diagonal (collision + reaction, one (5 ns)x(5 ns) block per
fluid node) and S the streaming operator with its boundary rules (bounce-back
at solids, anti-bounce-back at the inlet for A / bounce-back for B, C,
anti-bounce-back with C_w = C_b at the outlet).  The steady state solves
(I - A) g = b.  The matrix is assembled here from the formulas, independently
of the time-stepping loop in ``lbref.c``, so that the two can pin each other.

The steady adjoint gives d eps / d k(sigma) at the fixed point:
(I - A)^T lam = d eps / d g, then d eps / d k = lam^T (dA/dk) g.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

CX = np.array([0, 1, 0, -1, 0])
CY = np.array([0, 0, 1, 0, -1])
WQ = np.array([1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6])
OPP = np.array([0, 3, 4, 1, 2])


class System:
    """Affine one-step map of the ADR scheme restricted to fluid nodes."""

    def __init__(self, node_type, k, ux, uy, nspecies, tau, c_in=1.0, vel_scale=1.0,
                 xf=None):
        t = np.asarray(node_type)
        self.t = t
        self.ny, self.nx = t.shape
        self.ns = nspecies
        self.tau = tau
        self.c_in = c_in
        self.xf = self.nx - 3 if xf is None else xf
        fy, fx = np.nonzero(t == 0)
        self.fy, self.fx = fy, fx
        self.nf = len(fx)
        self.node_index = np.full(t.shape, -1, dtype=np.int64)
        self.node_index[fy, fx] = np.arange(self.nf)
        self.k = np.asarray(k, dtype=np.float64)
        self.u = vel_scale * np.asarray(ux, dtype=np.float64)[fy, fx]
        self.v = vel_scale * np.asarray(uy, dtype=np.float64)[fy, fx]
        self.nu = self.ns * 5 * self.nf
        self._links = self._catalytic_links()
        self.L = self._collision_reaction()
        self.S, self.b = self._streaming()
        self.A = (self.S @ self.L).tocsr()

    def idx(self, s, i, j):
        """Unknown index of population i of species s at fluid node j."""
        return (s * 5 + i) * self.nf + j

    def _catalytic_links(self):
        """(fluid node j, direction i, solid node y, x, src, prod) for each
        population that streams into a catalytic node."""
        out = []
        for i in range(1, 5):
            sx, sy = self.fx + CX[i], self.fy + CY[i]
            ok = (sx >= 0) & (sx < self.nx) & (sy >= 0) & (sy < self.ny)
            for j in np.nonzero(ok)[0]:
                ty = self.t[sy[j], sx[j]]
                if ty == 2:
                    out.append((j, i, sy[j], sx[j], 0, 1))
                elif ty == 3 and self.ns == 3:
                    out.append((j, i, sy[j], sx[j], 1, 2))
        return out

    def _collision_reaction(self):
        rows, cols, vals = [], [], []
        j = np.arange(self.nf)
        uu = self.u ** 2 + self.v ** 2
        for s in range(self.ns):
            for i in range(5):
                cu = CX[i] * self.u + CY[i] * self.v
                e = WQ[i] * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
                for jj in range(5):
                    val = e / self.tau + ((1 - 1 / self.tau) if jj == i else 0.0)
                    rows.append(self.idx(s, i, j)); cols.append(self.idx(s, jj, j)); vals.append(val)
        for (jn, i, sy, sx, src, prod) in self._links:
            kr = self.k[sy, sx] * WQ[i]
            for jj in range(5):
                rows += [self.idx(src, i, jn), self.idx(prod, i, jn)]
                cols += [self.idx(src, jj, jn)] * 2
                vals += [-kr, kr]
        rows = np.concatenate([np.atleast_1d(r) for r in rows])
        cols = np.concatenate([np.atleast_1d(c) for c in cols])
        vals = np.concatenate([np.atleast_1d(v) for v in vals])
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.nu, self.nu))

    def _streaming(self):
        rows, cols, vals = [], [], []
        b = np.zeros(self.nu)
        for s in range(self.ns):
            for j in range(self.nf):
                x, y = self.fx[j], self.fy[j]
                rows.append(self.idx(s, 0, j)); cols.append(self.idx(s, 0, j)); vals.append(1.0)
                for i in range(1, 5):
                    r = self.idx(s, i, j)
                    sx, sy = x - CX[i], y - CY[i]
                    if sx < 0:
                        if s == 0:
                            rows.append(r); cols.append(self.idx(s, 3, j)); vals.append(-1.0)
                            b[r] += 2 * WQ[1] * self.c_in
                        else:
                            rows.append(r); cols.append(self.idx(s, 3, j)); vals.append(1.0)
                    elif sx >= self.nx:
                        rows.append(r); cols.append(self.idx(s, 1, j)); vals.append(-1.0)
                        for jj in range(5):
                            rows.append(r); cols.append(self.idx(s, jj, j)); vals.append(2 * WQ[3])
                    elif sy < 0 or sy >= self.ny or self.t[sy, sx] != 0:
                        rows.append(r); cols.append(self.idx(s, OPP[i], j)); vals.append(1.0)
                    else:
                        rows.append(r); cols.append(self.idx(s, i, self.node_index[sy, sx])); vals.append(1.0)
        S = sp.csr_matrix((vals, (rows, cols)), shape=(self.nu, self.nu))
        return S, b

    # ------------------------------------------------------------------ solves
    def flux_functionals(self):
        """Row vectors l_s with N_s = l_s . g (net flux through the face between
        columns xf and xf+1), and l_in with inflow_A = l_in . g + const."""
        ls = np.zeros((self.ns, self.nu))
        for y in range(self.ny):
            a, c = self.node_index[y, self.xf], self.node_index[y, self.xf + 1]
            if a < 0 or c < 0:
                continue
            for s in range(self.ns):
                ls[s, self.idx(s, 1, c)] += 1.0
                ls[s, self.idx(s, 3, a)] -= 1.0
        return ls

    def steady(self):
        """Fixed point g of g = A g + b; returns (g, N, eps)."""
        M = (sp.identity(self.nu, format="csr") - self.A).tocsc()
        g = spla.spsolve(M, self.b)
        ls = self.flux_functionals()
        N = ls @ g
        return g, N, float(N[-1] / N.sum())

    def concentration(self, g):
        c = np.zeros((self.ns, self.ny, self.nx))
        for s in range(self.ns):
            cs = sum(g[self.idx(s, i, 0): self.idx(s, i, 0) + self.nf] for i in range(5))
            c[s, self.fy, self.fx] = cs
        return c

    def steady_gradient(self):
        """d eps / d k at every node (non-zero at catalytic nodes) at the
        steady state, by the adjoint of the fixed-point equation."""
        g, N, eps = self.steady()
        ls = self.flux_functionals()
        tot = N.sum()
        deps_dN = -N[-1] / tot ** 2 * np.ones(self.ns)
        deps_dN[-1] += 1.0 / tot
        rhs = ls.T @ deps_dN
        M = (sp.identity(self.nu, format="csr") - self.A).T.tocsc()
        lam = spla.spsolve(M, rhs)
        lam_post = self.S.T @ lam          # sensitivity to post-collision values
        c = self.concentration(g)
        grad = np.zeros((self.ny, self.nx))
        for (jn, i, sy, sx, src, prod) in self._links:
            csrc = c[src, self.fy[jn], self.fx[jn]]
            grad[sy, sx] += WQ[i] * csrc * (lam_post[self.idx(prod, i, jn)]
                                            - lam_post[self.idx(src, i, jn)])
        return grad, eps
