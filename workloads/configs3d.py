"""3D workloads: the paper's randomly oriented fibre membranes (Sec. "System
geometry: Single reaction" and "Cascade reaction": a 120x100x120 box with six
R = 3 fibres for A->B, 200x60x60 with two six-fibre R = 3 membranes for the
cascade, 160x60x60 with six R = 6 side-by-side fibres).

Lattice mapping (the 3D ADR uses D3Q7 with cs^2 = 1/4):

    D = u_ref R / Pe;  if D > 1/2: D = 1/2 and u_ref = Pe D / R
    tau_g = 1/2 + 4 D,   k = Da D / R^2

The flow is driven by a uniform body force in a box periodic in every
direction, as in the paper; its entrance velocity u0 (mean x-velocity over the
fluid nodes of the plane x = 0) is measured after the flow solve and the ADR
velocity is scaled by vel_scale = u_ref / u0 (linear Stokes scaling).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .geometry3d import CAT1, CAT2, FLUID, membrane, side_by_side_membrane

U_REF = 0.05     # ADR entrance velocity before the Pe clamp
TAU_F = 0.8
FORCE = 1e-6     # body force of the flow solve (the paper's value)
C_IN = 1.0
LENGTH = 40      # fibre length (flat caps)


@dataclass(frozen=True)
class LatticeParams3D:
    pe: float
    da: float
    r: int
    d: float
    tau_g: float
    k: float
    u_ref: float


def lattice_params3d(pe: float, da: float, r: int, u_ref: float = U_REF) -> LatticeParams3D:
    d = u_ref * r / pe
    if d > 0.5:
        d = 0.5
        u_ref = pe * d / r
    return LatticeParams3D(pe, da, r, d, 0.5 + 4.0 * d, da * d / (r * r), u_ref)


@dataclass
class Workload3D:
    name: str
    node_type: np.ndarray            # uint8 [nz, ny, nx]
    k: np.ndarray                    # float64 [nz, ny, nx]
    nspecies: int
    params: LatticeParams3D
    real: str = "f32"
    tau_f: float = TAU_F
    force: float = FORCE
    c_in: float = C_IN

    @property
    def shape(self):
        return self.node_type.shape

    @property
    def nx(self) -> int:
        return self.node_type.shape[2]

    @property
    def ny(self) -> int:
        return self.node_type.shape[1]

    @property
    def nz(self) -> int:
        return self.node_type.shape[0]

    @property
    def tau_g(self) -> float:
        return self.params.tau_g

    def n_catalytic(self) -> int:
        return int((self.node_type >= CAT1).sum())

    def vel_scale(self, ux) -> float:
        """u_ref over the entrance velocity of a flow field ux [nz, ny, nx]."""
        plane = np.asarray(ux)[:, :, 0][self.node_type[:, :, 0] == FLUID]
        return self.params.u_ref / float(plane.mean())


def _rates(t, k):
    return np.where(t >= CAT1, k, 0.0)


def make_workload3d(name: str, pe: float | None = None, da: float | None = None,
                    real: str | None = None) -> Workload3D:
    """M3a   120x100x120 (nx, ny, nz), six R = 3 type-1 fibres in x in [20, 100),
             seed 31, A->B, Pe 10, Da 1.
    M3c   200x60x60, six R = 3 type-1 fibres in [30, 95) and six type-2 in
          [105, 170), seed 32, cascade, Pe 10, Da 5.
    M3s   160x60x60, six R = 6 side-by-side fibres in [30, 130), seed 33,
          cascade, Pe 10, Da 5.
    M3c2  M3c doubled in every direction (400x120x120, 48 + 48 fibres, seed 34).
    M3t   40x24x20, one type-1 and one type-2 fibre R = 3, length 16, seed 35:
          the oracle-sized parity case.
    All fibres are 40 nodes long (16 for M3t), gap 2."""
    if name == "M3a":
        shape, r = (120, 100, 120), 3
        t = membrane(shape, [(20, 100)], [6], [CAT1], r, LENGTH, 31)
        ns, pe, da = 2, pe or 10.0, da or 1.0
    elif name == "M3c":
        shape, r = (60, 60, 200), 3
        t = membrane(shape, [(30, 95), (105, 170)], [6, 6], [CAT1, CAT2], r, LENGTH, 32)
        ns, pe, da = 3, pe or 10.0, da or 5.0
    elif name == "M3s":
        shape, r = (60, 60, 160), 6
        t = side_by_side_membrane(shape, (30, 130), 6, r, LENGTH, 33)
        ns, pe, da = 3, pe or 10.0, da or 5.0
    elif name == "M3c2":
        shape, r = (120, 120, 400), 3
        t = membrane(shape, [(60, 190), (210, 340)], [48, 48], [CAT1, CAT2], r, LENGTH, 34)
        ns, pe, da = 3, pe or 10.0, da or 5.0
    elif name == "M3t":
        shape, r = (20, 24, 40), 3
        t = membrane(shape, [(8, 20), (22, 34)], [1, 1], [CAT1, CAT2], r, 16, 35)
        ns, pe, da = 3, pe or 5.0, da or 10.0
    else:
        raise KeyError(name)
    p = lattice_params3d(pe, da, r)
    return Workload3D(name, t, _rates(t, p.k), ns, p, real=real or "f32")


CONFIGS3D = ("M3a", "M3c", "M3s", "M3c2", "M3t")
