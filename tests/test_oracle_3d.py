"""Pins of the 3D oracle (D3Q19 forced flow, D3Q7 ADR) against what the
mathematics fixes: exact uniform acceleration under Guo forcing, the exact
plate-Poiseuille profile of BGK with half-way bounce-back at the relaxation
time where its wall error vanishes, second-order convergence elsewhere, mass
conservation, mirror symmetry, the 3D Gaussian hill, exact homogeneous
decay, first-step link removal, steady mass balances and linearity."""
import numpy as np
import pytest

from oracle import lbref3d as R
from workloads.geometry3d import CAT1, CAT2, cylinder_voxels, classify_surface

TAU_MAGIC = 0.5 + np.sqrt(3.0) / 4.0   # (tau - 1/2)^2 = 3/16


def _plates(nx, ny, nz):
    t = np.zeros((nz, ny, nx), np.uint8)
    t[:, 0, :] = 1
    t[:, -1, :] = 1
    return t


def test_uniform_acceleration_is_exact():
    # empty periodic box: each step adds F to the momentum, u(t) = F (t + 1/2)
    t = np.zeros((3, 4, 5), np.uint8)
    F = (2e-5, -1e-5, 3e-6)
    for steps in (0, 1, 7):
        u, rho = R.flow(t, 0.8, F, steps)
        for a in range(3):
            assert np.abs(u[a] - F[a] * (steps + 0.5)).max() < 1e-15
        assert np.abs(rho - 1.0).max() < 1e-14


def _poiseuille(ny, tau, F=1e-5, steps=None):
    t = _plates(4, ny, 2)
    nu = (tau - 0.5) / 3.0
    H = ny - 2
    steps = steps or int(25 * H * H / nu)
    u, _ = R.flow(t, tau, (F, 0.0, 0.0), steps)
    y = np.arange(1, ny - 1)
    exact = F / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
    return u[0][0, 1:-1, 0], exact, u


def test_plate_poiseuille_exact_at_magic_tau():
    num, exact, u = _poiseuille(10, TAU_MAGIC)
    assert np.abs(num - exact).max() < 1e-9 * exact.max()
    assert np.abs(u[1]).max() < 1e-15 and np.abs(u[2]).max() < 1e-15


def test_plate_poiseuille_second_order_at_other_tau():
    errs = []
    for ny in (8, 14):
        num, exact, _ = _poiseuille(ny, 0.8)
        errs.append(np.abs(num - exact).max() / exact.max())
    assert errs[0] > 1e-4                     # a real wall error at tau = 0.8 ...
    assert errs[0] / errs[1] > 3.0            # ... that falls ~ (H1/H2)^-2 = 4


def _fibre_box(nx=24, ny=12, nz=10, centre=(11.5, 5.5, 4.5), axis=(0.0, 0.6, 0.8), r=2.5,
               length=8, kind=CAT1):
    t = np.zeros((nz, ny, nx), np.uint8)
    z, y, x, _ = cylinder_voxels(t.shape, np.array(centre), np.array(axis) / np.linalg.norm(axis),
                                 r, length)
    t[z, y, x] = 1
    surf = classify_surface(t == 1)
    t[surf] = kind
    return t


def test_flow_mass_conserved_and_mirror_symmetric():
    # axis in the y-z plane with the fibre centred in z: mirror z -> nz-1-z
    t = np.zeros((10, 12, 24), np.uint8)
    t[3:7, 4:8, 10:14] = 1                  # a block symmetric about z = 4.5
    f = R.flow_init(t)
    m0 = f.sum()
    R.flow_run(t, f, 0.8, (1e-5, 0, 0), 300)
    assert abs(f.sum() - m0) < 1e-11 * m0
    u, _ = R.flow_velocity(t, f, (1e-5, 0, 0))
    um = np.abs(u[0]).max()
    assert um > 1e-4
    # exact up to the summation order of the mirrored populations
    assert np.abs(u[0] - u[0][::-1]).max() < 1e-12 * um
    assert np.abs(u[2] + u[2][::-1]).max() < 1e-12 * um


def _hill(n, s0, tau, T):
    t = np.zeros((n, n, n), np.uint8)
    c = (n - 1) / 2.0
    zz, yy, xx = np.meshgrid(np.arange(n) - c, np.arange(n) - c, np.arange(n) - c, indexing="ij")
    r2 = xx ** 2 + yy ** 2 + zz ** 2
    c0 = np.exp(-r2 / (2 * s0 * s0))
    g = np.zeros((2, 7, n, n, n))
    w = [0.25] + [0.125] * 6
    for i in range(7):
        g[0, i] = w[i] * c0
    out = []
    for steps in (T // 2, T - T // 2):
        R.adr_run(t, np.zeros(t.shape), np.zeros((3, n, n, n)), g, tau, steps, mode=R.NODE,
                  bc=R.PERIODIC_X)
        out.append(R.adr_concentration(t, g)[0])
    return out, r2, xx, c0


def test_gaussian_hill_3d_closed_form():
    # periodic box, u = 0: C(r, t) = (s0^2/s^2)^(3/2) exp(-r^2 / (2 s^2)),
    # s^2 = s0^2 + 2 D t, D = (tau - 1/2)/4 for D3Q7 with cs^2 = 1/4.  D3Q7 at
    # cs^2 = 1/4 is not isotropic at fourth order, so the hill carries an
    # O(1/s^2) shape error: it must fall ~4x when s0 doubles (with 2 D t / s0^2
    # fixed).  A wrong D would leave an O(1) error in the width.
    tau = 0.9
    D = (tau - 0.5) / 4.0
    errs = []
    for n, s0 in ((24, 2.0), (44, 4.0)):
        T = int(round(1.5 * s0 * s0 / (2 * D)))
        (half, conc), r2, xx, c0 = _hill(n, s0, tau, T)
        s2 = s0 * s0 + 2 * D * T
        exact = (s0 * s0 / s2) ** 1.5 * np.exp(-r2 / (2 * s2))
        errs.append(np.abs(conc - exact).max() / exact.max())
        assert abs(conc.sum() - c0.sum()) < 1e-10 * c0.sum()
    assert errs[1] < 6e-3
    assert errs[0] / errs[1] > 3.0


@pytest.mark.parametrize("k", [0.01, 1.0])
def test_homogeneous_decay_exact(k):
    t = np.zeros((3, 4, 5), np.uint8)
    z = np.zeros((3,) + t.shape)
    g = R.adr_init(t, z, 2)
    for step in range(1, 6):
        R.adr_run(t, np.full(t.shape, k), z, g, 0.8, 1, mode=R.NODE, bc=R.PERIODIC_X)
        tot = R.adr_totals(t, g)
        assert abs(tot[0] - (1 - k) ** step * t.size) < 1e-12 * t.size
        assert abs(tot.sum() - t.size) < 1e-12 * t.size


def test_first_step_link_removal_exact():
    t = _fibre_box()
    k = np.where(t == CAT1, 0.3, 0.0)
    z = np.zeros((3,) + t.shape)
    g = np.zeros((2, 7) + t.shape)
    w = [0.25] + [0.125] * 6
    for i in range(7):
        g[0, i] = np.where(t == 0, w[i], 0.0)
    a0 = g[0].sum()
    R.adr_run(t, k, z, g, 0.9, 1, bc=R.PERIODIC_X)
    nz, ny, nx = t.shape
    links = 0
    for (zz, yy, xx) in zip(*np.nonzero(t == 0)):
        for dz, dy, dx in ((0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)):
            links += t[(zz + dz) % nz, (yy + dy) % ny, (xx + dx) % nx] == CAT1
    assert links > 20
    assert abs((a0 - g[0].sum()) - 0.3 * 0.125 * links) < 1e-12
    assert abs(g[1].sum() - 0.3 * 0.125 * links) < 1e-12


@pytest.fixture(scope="module")
def fibre_flow():
    t = _fibre_box(nx=20, ny=8, nz=8, centre=(9.5, 3.5, 3.5), axis=(0.0, 1.0, 0.3), r=2.2, length=5)
    u, _ = R.flow(t, 0.8, (2e-5, 0, 0), 1500)
    return t, u


def test_da0_outflow_equals_inflow_3d(fibre_flow):
    t, u = fibre_flow
    g = R.adr_init(t, u, 2, vel_scale=30.0)
    R.adr_run(t, np.zeros(t.shape), u, g, 0.7, 6000, vel_scale=30.0)
    flux, inflow = R.adr_observe(t, g)
    assert abs(flux.sum() - inflow) < 1e-8 * abs(inflow)
    assert abs(flux[1]) < 1e-14


def test_cascade_mass_balance_and_linearity_3d(fibre_flow):
    t0, u = fibre_flow
    t = t0.copy()
    t[:, :, 10:][t[:, :, 10:] == CAT1] = CAT2        # downstream half of the fibre: type 2
    k = np.where(t >= CAT1, 0.05, 0.0)
    out = []
    for c_in in (1.0, 2.5):
        g = R.adr_init(t, u, 3, c_in=c_in, vel_scale=30.0)
        R.adr_run(t, k, u, g, 0.7, 6000, c_in=c_in, vel_scale=30.0)
        flux, inflow = R.adr_observe(t, g, c_in=c_in)
        assert abs(flux.sum() - inflow) < 1e-7 * abs(inflow)
        out.append((R.efficiency(flux), R.adr_concentration(t, g)))
    assert out[0][0] > 0
    assert abs(out[0][0] - out[1][0]) < 1e-12
    assert np.abs(2.5 * out[0][1] - out[1][1]).max() < 1e-12 * 2.5 * out[0][1].max()
