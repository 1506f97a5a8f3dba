"""Workload definitions: geometry + lattice parameters for each configuration.

Dimensionless numbers (paper Sec. "System parameters and dimensionless
numbers"): Pe = u0 R / D with u0 the centre-line inlet velocity, Da = k R^2 / D.
Lattice mapping used here (one flow field per geometry, driven at u0 = 0.05 and
scaled linearly for the ADR, as the paper does with its Stokes flows):

    D = u0 R / Pe;  if D > 1/2:  D = 1/2 and vel_scale = Pe D / (u0 R)
    tau_g = 1/2 + 3 D      (D = cs^2 (tau_g - 1/2), cs^2 = 1/3)
    k = Da D / R^2

Both the GPU library and the oracle receive tau_g, vel_scale and the per-node
rate map k as inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .geometry import CAT1, CAT2, FLUID, channel, classify_surface, place_discs, rasterize

U0 = 0.05      # centre-line inlet velocity of the flow solve
TAU_F = 0.8    # D2Q9 BGK relaxation time
C_IN = 1.0     # inlet concentration of species A


@dataclass(frozen=True)
class LatticeParams:
    pe: float
    da: float
    r: int
    d: float
    tau_g: float
    k: float
    vel_scale: float


def lattice_params(pe: float, da: float, r: int, u0: float = U0) -> LatticeParams:
    d = u0 * r / pe
    vel_scale = 1.0
    if d > 0.5:
        d = 0.5
        vel_scale = pe * d / (u0 * r)
    return LatticeParams(pe, da, r, d, 0.5 + 3.0 * d, da * d / (r * r), vel_scale)


@dataclass
class Workload:
    name: str
    node_type: np.ndarray            # uint8 [ny, nx]
    k: np.ndarray                    # float64 [ny, nx], non-zero at catalytic nodes
    nspecies: int
    params: LatticeParams
    real: str = "f32"                # arithmetic of the GPU path: "f32" or "f64"
    u0: float = U0
    tau_f: float = TAU_F
    c_in: float = C_IN
    flow_steps: int | None = None    # fixed flow step count (None: run to tolerance)
    flow_tol: float | None = None    # max|du| over check interval <= tol*u0 (None: by precision)
    adr_tol: float = 1e-8            # relative change of eps over check interval
    check_every: int = 1000
    centres: list = field(default_factory=list)
    boundary: int = 0                # 0 channel with inlet/outlet, 1 periodic box (no flow)

    @property
    def nx(self) -> int:
        return self.node_type.shape[1]

    @property
    def ny(self) -> int:
        return self.node_type.shape[0]

    @property
    def flow_tolerance(self) -> float:
        """Flow convergence tolerance: 1e-6 u0 in FP64; 1e-5 u0 with FP32
        storage, whose rounding keeps max|du| over 1000 steps near 4e-6 u0 on
        the C1/C2 lattices however long the flow runs."""
        if self.flow_tol is not None:
            return self.flow_tol
        return 1e-5 if self.real == "f32" else 1e-6

    @property
    def tau_g(self) -> float:
        return self.params.tau_g

    @property
    def vel_scale(self) -> float:
        return self.params.vel_scale

    @property
    def xf(self) -> int:
        return self.nx - 3

    def n_catalytic(self) -> int:
        return int((self.node_type >= CAT1).sum())


def _finish(node_type, owner, surface, types_per_fibre, k_value):
    """Assign a catalyst type to every surface node and fill the rate map."""
    t = node_type
    k = np.zeros(t.shape, dtype=np.float64)
    ys, xs = np.nonzero(surface)
    for y, x in zip(ys, xs):
        ty = types_per_fibre(owner[y, x], x, y)
        t[y, x] = ty
        k[y, x] = k_value
    return t, k


def _membranes(nx, ny, r, bands, counts, seed, gap=2):
    """Two-membrane cascade geometry: fibres of membrane 1 carry catalyst
    type 1, fibres of membrane 2 catalyst type 2."""
    rng = np.random.default_rng(seed)
    centres, kinds = [], []
    for band, cnt, kind in zip(bands, counts, (CAT1, CAT2)):
        c = place_discs(rng, cnt, r, band, ny, gap, existing=centres)
        centres += c
        kinds += [kind] * len(c)
    t = channel(nx, ny)
    owner = rasterize(t, centres, r)
    surf = classify_surface(t, owner)
    return t, owner, surf, centres, kinds


def _cascade(name, nx, ny, r, bands, counts, seed, pe, da, real="f32"):
    p = lattice_params(pe, da, r)
    t, owner, surf, centres, kinds = _membranes(nx, ny, r, bands, counts, seed)
    t, k = _finish(t, owner, surf, lambda f, x, y: kinds[f], p.k)
    return Workload(name, t, k, 3, p, real=real, centres=centres)


def _side_by_side(name, nx, ny, r, band, count, seed, pe, da, gap=2, real="f32"):
    """One band of fibres, each carrying catalyst type 1 on the half of its
    surface facing -(cos th, sin th) and type 2 on the other half; th is drawn
    uniformly in [0, 2 pi) per fibre (th = 0: type 1 on the upstream half)."""
    p = lattice_params(pe, da, r)
    rng = np.random.default_rng(seed)
    centres = place_discs(rng, count, r, band, ny, gap)
    theta = rng.uniform(0.0, 2.0 * np.pi, size=count)
    t = channel(nx, ny)
    owner = rasterize(t, centres, r)
    surf = classify_surface(t, owner)

    def kind(f, x, y):
        cx, cy = centres[f]
        s = (x - cx) * np.cos(theta[f]) + (y - cy) * np.sin(theta[f])
        return CAT1 if s < 0 else CAT2

    t, k = _finish(t, owner, surf, kind, p.k)
    w = Workload(name, t, k, 3, p, real=real, centres=centres)
    return w


def _single_disc(name, nx, ny, r, centre, pe, da, kind=CAT1, nspecies=2, real="f64",
                 flow_steps=None):
    p = lattice_params(pe, da, r)
    t = channel(nx, ny)
    owner = rasterize(t, [centre], r)
    surf = classify_surface(t, owner)
    t, k = _finish(t, owner, surf, lambda f, x, y: kind, p.k)
    return Workload(name, t, k, nspecies, p, real=real, flow_steps=flow_steps,
                    centres=[centre])


def _two_discs(name, nx, ny, r, c1, c2, pe, da, real="f64"):
    p = lattice_params(pe, da, r)
    t = channel(nx, ny)
    owner = rasterize(t, [c1, c2], r)
    surf = classify_surface(t, owner)
    t, k = _finish(t, owner, surf, lambda f, x, y: (CAT1, CAT2)[f], p.k)
    return Workload(name, t, k, 3, p, real=real, centres=[c1, c2])


def box_workload(morphology: str = "pair", da: float = 150.0, d: float = 0.1, n: int = 300,
                 xi: int = 100, real: str = "f64") -> Workload:
    """Pure-diffusion cascade in an n x n box periodic in x and y (paper Sec.
    "Pure diffusion case"): no flow, A fills the fluid homogeneously at t = 0,
    and the totals of A, B, C are followed in time.

    morphology "pair": two fibres R = 5 on the centre row, centres xi apart,
    the left one carrying catalyst type 1 and the right one type 2 (the
    "individual" arrangement).  "side": one fibre R = 10 at the centre, type 1
    on its left half (x < cx) and type 2 on the right half (side-by-side).
    D = (tau_g - 1/2)/3 is fixed by ``d``; k = Da D / R^2 with the fibre's R."""
    t = np.zeros((n, n), dtype=np.uint8)
    c = n // 2
    if morphology == "pair":
        r = 5
        centres = [(c - xi // 2, c), (c + xi - xi // 2, c)]
        kind = lambda f, x, y: (CAT1, CAT2)[f]
    elif morphology == "side":
        r = 10
        centres = [(c, c)]
        kind = lambda f, x, y: CAT1 if x < c else CAT2
    else:
        raise KeyError(morphology)
    k = da * d / (r * r)
    p = LatticeParams(0.0, da, r, d, 0.5 + 3.0 * d, k, 0.0)
    owner = rasterize(t, centres, r)
    surf = classify_surface(t, owner)
    t, kmap = _finish(t, owner, surf, kind, k)
    return Workload(f"box-{morphology}", t, kmap, 3, p, real=real, centres=centres, boundary=1)


def make_workload(name: str, pe: float | None = None, da: float | None = None,
                  real: str | None = None) -> Workload:
    """Build one of the named workloads (optionally overriding Pe, Da, precision).

    C0      200x100, one type-1 disc R = 10 at (60, 50), A->B, FP64, Pe 10, Da 1,
            10,000 flow steps, ADR until the relative change of eps < 1e-8.
    C1      2048x512 cascade: 20 type-1 discs in x in [400, 800], 20 type-2
            discs in [1000, 1400], R = 8, gap 2, seed 1, Pe 100, Da 10, FP32.
    C1q     C1 at a quarter of its linear size (512x128, 5 + 5 discs, R = 8).
    C2      4096x1024, 200 side-by-side discs R = 6 in [1000, 3000], seed 2,
            Pe in {1, 10, 100, 1000} (default 100), Da 5, FP32.
    C2q     C2 at a quarter of its linear size (1024x256, 12 discs).
    tiny    64x32 cascade: type-1 disc R = 3 at (20, 16), type-2 disc R = 3 at
            (36, 15), Pe 5, Da 10 -- the autograd-sized adjoint case.
    rw      96x34, one type-1 disc R = 4 at (32, 17), Pe 2, Da 1, A->B -- the
            random-walk comparison case.
    """
    if name == "C0":
        w = _single_disc("C0", 200, 100, 10, (60, 50), pe or 10.0, da or 1.0,
                         real=real or "f64", flow_steps=10000)
        return w
    if name == "C1":
        return _cascade("C1", 2048, 512, 8, [(400, 800), (1000, 1400)], [20, 20], 1,
                        pe or 100.0, da or 10.0, real=real or "f32")
    if name == "C1q":
        return _cascade("C1q", 512, 128, 8, [(100, 200), (250, 350)], [5, 5], 11,
                        pe or 100.0, da or 10.0, real=real or "f32")
    if name == "C2":
        return _side_by_side("C2", 4096, 1024, 6, (1000, 3000), 200, 2, pe or 100.0,
                             da or 5.0, real=real or "f32")
    if name == "C2q":
        return _side_by_side("C2q", 1024, 256, 6, (250, 750), 12, 22, pe or 100.0,
                             da or 5.0, real=real or "f32")
    if name == "tiny":
        return _two_discs("tiny", 64, 32, 3, (20, 16), (36, 15), pe or 5.0, da or 10.0,
                          real=real or "f64")
    if name == "rw":
        return _single_disc("rw", 96, 34, 4, (32, 17), pe or 2.0, da or 1.0,
                            real=real or "f64")
    raise KeyError(name)


CONFIGS = ("C0", "C1", "C1q", "C2", "C2q", "tiny", "rw")


def batch_instances(n: int = 64, seed: int = 3, ny: int = 256, nx_range=(512, 2048),
                    pe_range=(0.1, 1000.0), da_range=(0.01, 100.0), r: int = 8,
                    fibres: int = 20):
    """Instances of the batched Pe x Da sweep: two-membrane cascades like C1
    with length nx_i ~ U{512..2048}, height 256, bands scaled by nx_i/2048,
    Pe log-uniform in [0.1, 1000], Da log-uniform in [0.01, 100].  The master
    seed draws (nx_i, Pe_i, Da_i); instance i's geometry uses seed 3000 + i."""
    rng = np.random.default_rng(seed)
    nxs = rng.integers(nx_range[0], nx_range[1] + 1, size=n)
    pes = 10.0 ** rng.uniform(np.log10(pe_range[0]), np.log10(pe_range[1]), size=n)
    das = 10.0 ** rng.uniform(np.log10(da_range[0]), np.log10(da_range[1]), size=n)
    out = []
    for i in range(n):
        nx = int(nxs[i])
        s = nx / 2048.0
        bands = [(int(round(400 * s)), int(round(800 * s))),
                 (int(round(1000 * s)), int(round(1400 * s)))]
        w = _cascade(f"C3[{i}]", nx, ny, r, bands, [fibres, fibres], 3000 + i,
                     float(pes[i]), float(das[i]))
        out.append(w)
    return out
