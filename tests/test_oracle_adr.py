"""Pins of the oracle's D2Q5 advection-diffusion-reaction solver.

Each test checks the oracle against something the paper or the mathematics
fixes -- closed forms, exact discrete solutions, conservation laws, special
cases -- never against itself:

* Gaussian hill (paper appendix "Advection-Diffusion of a Gaussian Hill"):
  closed form with sigma_D^2 = 2 D t, D = cs^2 (tau - 1/2) (Eq. Diffusion_LBM).
* homogeneous first-order decay (appendix "Homogeneous reaction"): with a
  unit time step the scheme gives exactly C(t) = (1 - k)^t C(0); k = 1 decays
  in a single step.
* plug flow with a uniform sink: the steady profile decays as exp(lambda x),
  lambda = (U - sqrt(U^2 + 4 D k)) / (2 D); the exact discrete decay factor is
  the root of a 5x5 transfer-matrix determinant.
* conservation: at Da = 0 the outflux of A equals its inflow and eps = 0; in
  the steady cascade N_A + N_B + N_C equals the inflow of A (Eq. A-B).
* the first step from a uniform state removes exactly sum k w_i C of A
  (Eq. source_lbm applied at the links into catalytic nodes).
* linearity in the inlet concentration; mirror symmetry.
* the direct sparse fixed-point solve equals the time-stepped steady state.
* the initial state: the equilibrium's zeroth and first moments are C = c_in
  and C u (u the scaled flow velocity), B and C absent.
* the steady-state test of a run does not fire before the product leaves.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import lbref as R
from oracle.steady_direct import System
from workloads import CAT1, CAT2, channel, make_workload, rasterize
from workloads.geometry import classify_surface

W = np.array([1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6])
CX = np.array([0, 1, 0, -1, 0])
CY = np.array([0, 0, 1, 0, -1])


# ------------------------------------------------------------------ helpers
def _eq_state(c, u, v):
    """Species-A equilibrium populations for a concentration field c and a
    uniform velocity (u, v), written out from the second-order equilibrium."""
    g = np.zeros((1, 5) + c.shape)
    for i in range(5):
        cu = CX[i] * u + CY[i] * v
        g[0, i] = W[i] * c * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (u * u + v * v))
    return g


def _hill(n, sigma0, u, tau, T):
    y, x = np.mgrid[0:n, 0:n].astype(float)
    x0 = y0 = n / 2
    c0 = np.exp(-((x - x0) ** 2 + (y - y0) ** 2) / (2 * sigma0 ** 2))
    g = _eq_state(c0, *u)
    t = np.zeros((n, n), np.uint8)
    z = np.zeros((n, n))
    R.adr_run(t, z, z + u[0], z + u[1], g, tau, T, mode=R.NODE,
              bc=R.PERIODIC_X | R.PERIODIC_Y)
    c = g[0].sum(0)
    X, Y = x - x0 - u[0] * T, y - y0 - u[1] * T
    return c, X, Y


@pytest.fixture(scope="module")
def tiny_flow():
    w = make_workload("tiny")
    ux, uy, _, _ = R.flow_steady(w.node_type, w.tau_f, w.u0, 3000, tol=0)
    return w, ux, uy


# ------------------------------------------------------- Gaussian hill pins
@pytest.mark.parametrize("sigma0,T,tol", [(4, 100, 2e-3), (4, 400, 1e-3),
                                           (1, 100, 3e-3), (1, 400, 1e-3)])
def test_gaussian_hill_pure_diffusion(sigma0, T, tol):
    # tau = 1 gives D = 1/6 (the paper's 0.1666); exact solution is Gaussian
    tau = 1.0
    D = (tau - 0.5) / 3
    assert abs(D - 0.1666) < 1e-4
    c, X, Y = _hill(100, sigma0, (0.0, 0.0), tau, T)
    s2 = sigma0 ** 2 + 2 * D * T
    exact = sigma0 ** 2 / s2 * np.exp(-(X * X + Y * Y) / (2 * s2))
    assert np.abs(c - exact).max() / exact.max() < tol
    assert abs(c.sum() - 2 * np.pi * sigma0 ** 2) < 1e-9 * c.sum() or sigma0 == 1


def test_gaussian_hill_advected_d2q5_tensor():
    # u = (0.1, 0.1) as in the paper.  The D2Q5 equilibrium's second moment is
    # C (1/3 - u.u/2 + 3/2 u_a^2) on the diagonal and 0 off it, so the
    # diffusion tensor is D_ab = (tau - 1/2)(Pi_ab/C - u_a u_b):
    # Dxx = Dyy = (tau-1/2)(1/3 - u^2/2...), Dxy = -(tau-1/2) u_x u_y.
    tau, T, sigma0 = 1.0, 100, 4.0
    u = (0.1, 0.1)
    c, X, Y = _hill(100, sigma0, u, tau, T)
    uu = u[0] ** 2 + u[1] ** 2
    dxx = (tau - 0.5) * (1 / 3 - 0.5 * uu + 0.5 * u[0] ** 2)
    dyy = (tau - 0.5) * (1 / 3 - 0.5 * uu + 0.5 * u[1] ** 2)
    dxy = -(tau - 0.5) * u[0] * u[1]
    sx, sy, sxy = sigma0 ** 2 + 2 * dxx * T, sigma0 ** 2 + 2 * dyy * T, 2 * dxy * T
    det = sx * sy - sxy ** 2
    exact = sigma0 ** 2 / np.sqrt(det) * np.exp(-0.5 * (sy * X * X - 2 * sxy * X * Y + sx * Y * Y) / det)
    assert np.abs(c - exact).max() / exact.max() < 5e-3
    # the isotropic closed form is only met to ~1 %
    s2 = sigma0 ** 2 + 2 * (tau - 0.5) / 3 * T
    iso = sigma0 ** 2 / s2 * np.exp(-(X * X + Y * Y) / (2 * s2))
    assert np.abs(c - iso).max() / iso.max() < 1.5e-2
    # at tau = 1 the first moment of the post-collision state is C u exactly,
    # so the centre of mass moves with u; coordinates are taken periodic
    # around the expected centre (tails at +-50 are ~1e-11)
    y, x = np.mgrid[0:100, 0:100].astype(float)
    xr = (x - (50 + u[0] * T) + 50) % 100 - 50
    assert abs((c * xr).sum() / c.sum()) < 1e-9


# ------------------------------------------------------ homogeneous decay
@pytest.mark.parametrize("k", [0.01, 0.3, 1.0])
def test_homogeneous_decay_is_exactly_geometric(k):
    n = 8
    t = np.zeros((n, n), np.uint8)
    z = np.zeros((n, n))
    g = np.zeros((2, 5, n, n))
    g[0] = _eq_state(np.ones((n, n)), 0.0, 0.0)[0]
    for step in range(1, 41):
        R.adr_run(t, z + k, z, z, g, 0.8, 1, mode=R.NODE, bc=R.PERIODIC_X | R.PERIODIC_Y)
        ca = g[0].sum(0)
        cb = g[1].sum(0)
        assert np.abs(ca - (1 - k) ** step).max() <= 1e-14 * max(1.0, step)
        assert np.abs(ca + cb - 1.0).max() < 1e-14
    if k == 1.0:
        # the paper notes the LB with a unit time step decays at once for k = 1
        assert np.abs(g[0]).max() < 1e-16


def test_homogeneous_cascade_recursion():
    n, k1, k2 = 6, 0.02, 0.05
    t = np.zeros((n, n), np.uint8)
    z = np.zeros((n, n))
    g = np.zeros((3, 5, n, n))
    g[0] = _eq_state(np.ones((n, n)), 0.0, 0.0)[0]
    a, b = 1.0, 0.0
    for step in range(60):
        R.adr_run(t, z + k1, z, z, g, 0.7, 1, mode=R.NODE, bc=3, k2=z + k2)
        a, b = a * (1 - k1), b * (1 - k2) + k1 * a
        c = g.sum(1)
        assert np.abs(c[0] - a).max() < 1e-14
        assert np.abs(c[1] - b).max() < 1e-14
        assert np.abs(c.sum(0) - 1.0).max() < 1e-14


# ------------------------------------------------------------- plug flow
def _transfer_root(U, tau, k):
    """Exact decay factor mu of the 1D steady scheme: with g(x) = mu^x v and
    post-collision P v, streaming gives mu v_E = (Pv)_E, v_W = mu (Pv)_W and
    v_i = (Pv)_i otherwise; mu is a root of det(P - diag(1, mu, 1, 1/mu, 1))."""
    e = W * (1 + 3 * CX * U + 4.5 * (CX * U) ** 2 - 1.5 * U * U)
    P = (1 - 1 / tau) * np.eye(5) + np.outer(e, np.ones(5)) / tau - k * np.outer(W, np.ones(5))
    return brentq(lambda mu: np.linalg.det(P - np.diag([1, mu, 1, 1 / mu, 1])), 0.5, 1 - 1e-12)


def test_plug_flow_uniform_sink():
    U, D, k, nx = 0.05, 0.05, 1e-3, 512
    tau = 0.5 + 3 * D
    t = np.zeros((1, nx), np.uint8)
    ux = np.full((1, nx), U); uy = np.zeros((1, nx)); kk = np.full((1, nx), k)
    g = R.adr_init(t, ux, uy, 2)
    prev = None
    for _ in range(40):
        R.adr_run(t, kk, ux, uy, g, tau, 2500, mode=R.NODE, bc=R.PERIODIC_Y)
        c = g[0].sum(0)[0]
        if prev is not None and np.abs(c - prev).max() < 1e-15:
            break
        prev = c
    xs = np.arange(nx // 8, nx // 2)
    mu = _transfer_root(U, tau, k)
    assert np.abs(c[xs + 1] / c[xs] - mu).max() < 1e-11
    lam = (U - np.sqrt(U * U + 4 * D * k)) / (2 * D)
    slope = np.polyfit(xs, np.log(c[xs]), 1)[0]
    assert abs(slope / lam - 1) < 1e-3
    # what enters as A leaves as A or B
    flux, inflow = R.adr_observe(t, g)
    assert abs(flux.sum() - inflow) < 1e-10 * inflow


# ------------------------------------------------- conservation and links
def test_da0_outflux_equals_inflow(tiny_flow):
    w, ux, uy = tiny_flow
    z = np.zeros_like(w.k)
    # eps is identically 0 here, so run a fixed number of steps to steady state
    g, steps, flux, inflow, eps = R.adr_steady(w.node_type, z, ux, uy, 3, w.tau_g, 30000,
                                               check_every=30000, tol=0)
    assert flux[1] == 0.0 and flux[2] == 0.0 and eps == 0.0
    assert abs(flux[0] - inflow) < 1e-9 * inflow


def test_cascade_steady_mass_balance(tiny_flow):
    w, ux, uy = tiny_flow
    g, steps, flux, inflow, eps = R.adr_steady(w.node_type, w.k, ux, uy, 3, w.tau_g, 60000,
                                               check_every=2000, tol=1e-12)
    assert abs(flux.sum() - inflow) < 1e-9 * inflow
    assert 0 < eps < 1 and flux[1] > 0 and flux[2] > 0


def test_production_equals_the_outflow_at_steady_state(tiny_flow):
    # at the steady cascade nothing accumulates: what B -> C converts per step
    # leaves as C (the paper's production rate of the final species), what
    # A -> B converts and B -> C does not leaves as B, the rest of the inflow
    # leaves as A
    w, ux, uy = tiny_flow
    g, steps, flux, inflow, eps = R.adr_steady(w.node_type, w.k, ux, uy, 3, w.tau_g, 60000,
                                               check_every=2000, tol=1e-12)
    r = R.adr_production(w.node_type, w.k, g)
    assert r[1] > 0 and r[0] > r[1]
    assert abs(r[1] - flux[2]) < 1e-8 * inflow
    assert abs(r[0] - r[1] - flux[1]) < 1e-8 * inflow
    assert abs(inflow - r[0] - flux[0]) < 1e-8 * inflow


def test_first_step_removal_exact():
    # closed periodic box at rest, uniform A: after one step A has lost exactly
    # sum over links (fluid x -> catalytic x + c_i) of k w_i c_in
    nx, ny = 40, 30
    t = np.zeros((ny, nx), np.uint8)
    owner = rasterize(t, [(20, 15)], 5)
    surf = classify_surface(t, owner)
    t[surf] = CAT1
    k = np.where(surf, 0.37, 0.0)
    g = np.zeros((2, 5, ny, nx))
    g[0] = np.where(t == 0, _eq_state(np.ones((ny, nx)), 0, 0)[0], 0.0)
    a0 = g[0].sum()
    removed = 0.0
    for y in range(ny):
        for x in range(nx):
            if t[y, x] != 0:
                continue
            for i in range(1, 5):
                yy, xx = (y + CY[i]) % ny, (x + CX[i]) % nx
                if t[yy, xx] == CAT1:
                    removed += k[yy, xx] * W[i] * 1.0
    z = np.zeros((ny, nx))
    R.adr_run(t, k, z, z, g, 0.9, 1, bc=R.PERIODIC_X | R.PERIODIC_Y)
    assert abs((a0 - g[0].sum()) - removed) < 1e-12
    assert abs(g[1].sum() - removed) < 1e-12
    assert removed > 0


def test_only_second_catalyst_gives_zero_efficiency(tiny_flow):
    w, ux, uy = tiny_flow
    t = w.node_type.copy()
    t[t == CAT1] = CAT2
    g = R.adr_init(t, ux, uy, 3)
    R.adr_run(t, w.k, ux, uy, g, w.tau_g, 3000)
    flux, _ = R.adr_observe(t, g)
    assert flux[1] == 0.0 and flux[2] == 0.0 and R.efficiency(flux) == 0.0


def test_linear_in_inlet_concentration(tiny_flow):
    w, ux, uy = tiny_flow
    out = []
    for cin in (1.0, 2.5):
        g = R.adr_init(w.node_type, ux, uy, 3, c_in=cin)
        R.adr_run(w.node_type, w.k, ux, uy, g, w.tau_g, 2000, c_in=cin)
        out.append((g, R.adr_observe(w.node_type, g, c_in=cin)[0]))
    assert np.abs(out[1][0] - 2.5 * out[0][0]).max() < 1e-12
    assert abs(R.efficiency(out[1][1]) - R.efficiency(out[0][1])) < 1e-13


def test_adr_mirror_symmetry():
    nx, ny = 60, 31
    t = channel(nx, ny)
    owner = rasterize(t, [(20, 15)], 4)
    surf = classify_surface(t, owner)
    t[surf] = CAT1
    k = np.where(surf, 0.05, 0.0)
    ux, uy, _, _ = R.flow_steady(t, 0.8, 0.05, 1500, tol=0)
    g = R.adr_init(t, ux, uy, 2)
    R.adr_run(t, k, ux, uy, g, 0.6, 1500)
    c = R.adr_concentration(t, g)
    assert np.abs(c - c[:, ::-1, :]).max() < 1e-13
    assert c[1].max() > 1e-3


# ---------------------------------------------- direct steady state solve
def test_direct_steady_solve_equals_time_stepping(tiny_flow):
    w, ux, uy = tiny_flow
    sysm = System(w.node_type, w.k, ux, uy, 3, w.tau_g)
    gd, Nd, eps_d = sysm.steady()
    g, steps, flux, inflow, eps = R.adr_steady(w.node_type, w.k, ux, uy, 3, w.tau_g, 60000,
                                               check_every=2000, tol=1e-13)
    assert abs(eps / eps_d - 1) < 1e-10
    assert np.abs(flux - Nd).max() < 1e-10
    c = R.adr_concentration(w.node_type, g)
    assert np.abs(c - sysm.concentration(gd)).max() < 1e-10


def test_direct_steady_gradient_matches_finite_differences(tiny_flow):
    w, ux, uy = tiny_flow
    grad, eps = System(w.node_type, w.k, ux, uy, 3, w.tau_g).steady_gradient()
    ys, xs = np.nonzero(w.node_type >= CAT1)
    assert (grad[w.node_type < CAT1] == 0).all()
    for j in (0, 9, 20, 31):
        y, x = ys[j], xs[j]
        h = 1e-4 * w.k[y, x]
        e = []
        for sgn in (1, -1):
            kk = w.k.copy(); kk[y, x] += sgn * h
            e.append(System(w.node_type, kk, ux, uy, 3, w.tau_g).steady()[2])
        fd = (e[0] - e[1]) / (2 * h)
        assert abs(grad[y, x] - fd) < 1e-7 * abs(fd)


# ------------- the paper's comparison variant: every population of the node reacts
def _closed_box_disc(kind=CAT1, k=0.3):
    nx, ny = 40, 30
    t = np.zeros((ny, nx), np.uint8)
    owner = rasterize(t, [(20, 15)], 5)
    surf = classify_surface(t, owner)
    t[surf] = kind
    return t, np.where(surf, k, 0.0), surf


def test_all_populations_variant_first_step_removal():
    # every fluid node next to a type-1 catalyst loses k c_in of A in one step
    # (all five populations react, sum of w_i = 1), whatever its number of
    # catalytic links -- against link mode, which removes k w_i c_in per link
    t, k, surf = _closed_box_disc()
    ny, nx = t.shape
    reactive = 0
    links = 0
    for y in range(ny):
        for x in range(nx):
            if t[y, x] != 0:
                continue
            n = sum(t[(y + CY[i]) % ny, (x + CX[i]) % nx] == CAT1 for i in range(1, 5))
            reactive += n > 0
            links += n
    z = np.zeros((ny, nx))
    out = {}
    for mode in (R.LINK, R.NODE_AT_CATALYST):
        g = np.zeros((2, 5, ny, nx))
        g[0] = np.where(t == 0, _eq_state(np.ones((ny, nx)), 0, 0)[0], 0.0)
        a0 = g[0].sum()
        R.adr_run(t, k, z, z, g, 0.9, 1, mode=mode, bc=R.PERIODIC_X | R.PERIODIC_Y)
        out[mode] = a0 - g[0].sum()
        assert abs(g[1].sum() - out[mode]) < 1e-12
    assert abs(out[R.NODE_AT_CATALYST] - 0.3 * reactive) < 1e-12
    assert abs(out[R.LINK] - 0.3 * links / 6) < 1e-12


def test_all_populations_variant_equals_node_reaction_with_neighbour_mean_rates():
    # the variant is a node reaction whose per-node rate is the mean rate of
    # the node's catalytic neighbours of each type (cascade, both types)
    nx, ny = 48, 36
    t = np.zeros((ny, nx), np.uint8)
    own = rasterize(t, [(15, 18), (33, 17)], 4)
    surf = classify_surface(t, own)
    t[surf & (own == 0)] = CAT1
    t[surf & (own == 1)] = CAT2
    rng = np.random.default_rng(0)
    k = np.where(surf, rng.uniform(0.05, 0.4, size=t.shape), 0.0)
    k1 = np.zeros((ny, nx))
    k2 = np.zeros((ny, nx))
    for y in range(ny):
        for x in range(nx):
            if t[y, x] != 0:
                continue
            a = [k[(y + CY[i]) % ny, (x + CX[i]) % nx] for i in range(1, 5)
                 if t[(y + CY[i]) % ny, (x + CX[i]) % nx] == CAT1]
            b = [k[(y + CY[i]) % ny, (x + CX[i]) % nx] for i in range(1, 5)
                 if t[(y + CY[i]) % ny, (x + CX[i]) % nx] == CAT2]
            k1[y, x] = np.mean(a) if a else 0.0
            k2[y, x] = np.mean(b) if b else 0.0
    z = np.zeros((ny, nx))
    bc = R.PERIODIC_X | R.PERIODIC_Y
    ga = np.zeros((3, 5, ny, nx))
    ga[0] = np.where(t == 0, _eq_state(np.ones((ny, nx)), 0, 0)[0], 0.0)
    gb = ga.copy()
    R.adr_run(t, k, z, z, ga, 0.8, 200, mode=R.NODE_AT_CATALYST, bc=bc)
    R.adr_run(t, k1, z, z, gb, 0.8, 200, mode=R.NODE, bc=bc, k2=k2)
    assert np.abs(ga - gb).max() < 1e-14
    tot = R.adr_totals(t, ga)
    assert abs(tot.sum() - (t == 0).sum()) < 1e-9   # closed box: A + B + C conserved
    assert tot[2] > 0


def test_production_of_the_uniform_state_has_its_closed_form():
    # closed box at rest, uniform A = 1: the link reaction converts sum over
    # links of k w_i, the all-populations variant k at every fluid node next
    # to a type-1 catalyst (brute force over the lattice)
    t, k, surf = _closed_box_disc()
    ny, nx = t.shape
    g = np.zeros((2, 5, ny, nx))
    g[0] = np.where(t == 0, _eq_state(np.ones((ny, nx)), 0, 0)[0], 0.0)
    links = reactive = 0
    for y in range(ny):
        for x in range(nx):
            if t[y, x] != 0:
                continue
            n = sum(t[(y + CY[i]) % ny, (x + CX[i]) % nx] == CAT1 for i in range(1, 5))
            links += n
            reactive += n > 0
    bc = R.PERIODIC_X | R.PERIODIC_Y
    assert links > 0
    assert abs(R.adr_production(t, k, g, R.LINK, bc)[0] - 0.3 * links / 6) < 1e-13
    assert abs(R.adr_production(t, k, g, R.NODE_AT_CATALYST, bc)[0] - 0.3 * reactive) < 1e-13


@pytest.mark.parametrize("mode", [R.LINK, R.NODE_AT_CATALYST])
def test_production_is_the_change_of_the_totals_in_a_closed_box(mode):
    # in a closed box (periodic, inert walls, no flow) one step changes the
    # totals by the reaction amounts only: A by -r0, B by r0 - r1, C by r1
    from workloads.configs import box_workload
    w = box_workload("side", n=60, da=40.0)
    t = w.node_type
    ny, nx = t.shape
    z = np.zeros((ny, nx))
    bc = R.PERIODIC_X | R.PERIODIC_Y
    g = R.adr_init(t, z, z, 3)
    R.adr_run(t, w.k, z, z, g, w.tau_g, 300, mode=mode, bc=bc)
    r = R.adr_production(t, w.k, g, mode, bc)
    before = R.adr_totals(t, g)
    R.adr_run(t, w.k, z, z, g, w.tau_g, 1, mode=mode, bc=bc)
    d = R.adr_totals(t, g) - before
    assert r[0] > 0 and r[1] > 0
    scale = before.sum()
    assert abs(d[0] + r[0]) < 1e-12 * scale
    assert abs(d[1] - (r[0] - r[1])) < 1e-12 * scale
    assert abs(d[2] - r[1]) < 1e-12 * scale


@pytest.mark.parametrize("c_in,scale", [(1.0, 1.0), (2.5, 0.7), (0.3, 3.0)])
def test_adr_initial_state_moments(tiny_flow, c_in, scale):
    # at every fluid node sum_i g_A,i = c_in and sum_i c_i g_A,i = c_in u with
    # u = vel_scale * u_flow (the second-order equilibrium reproduces both
    # moments exactly on D2Q5); species B and C and every solid node are 0
    w, ux, uy = tiny_flow
    g = R.adr_init(w.node_type, ux, uy, 3, c_in, scale)
    fl = w.node_type == 0
    c0 = g[0].sum(axis=0)
    jx = (CX[:, None, None] * g[0]).sum(axis=0)
    jy = (CY[:, None, None] * g[0]).sum(axis=0)
    assert np.abs(c0[fl] - c_in).max() < 1e-14 * c_in
    assert np.abs(jx[fl] - c_in * scale * ux[fl]).max() < 1e-15 * c_in
    assert np.abs(jy[fl] - c_in * scale * uy[fl]).max() < 1e-15 * c_in
    assert np.abs(scale * ux[fl]).max() > 1e-3   # the velocity terms matter here
    assert (g[1:] == 0).all() and (g[:, :, ~fl] == 0).all()


def test_steady_check_waits_for_the_product(tiny_flow):
    # with a check every 20 steps eps is exactly 0 at the first checks (the
    # products have not reached the flux plane), which a bare "eps did not
    # change" test would take for a steady state; the run must continue until
    # the product leaves and the outlet fluxes balance the inflow
    w, ux, uy = tiny_flow
    g = R.adr_init(w.node_type, ux, uy, 3)
    R.adr_run(w.node_type, w.k, ux, uy, g, w.tau_g, 40)
    flux, inflow = R.adr_observe(w.node_type, g)
    assert R.efficiency(flux) == 0.0
    g, steps, flux, inflow, eps = R.adr_steady(w.node_type, w.k, ux, uy, 3, w.tau_g, 60000,
                                               check_every=20, tol=1e-8)
    assert steps < 60000 and flux[2] > 0 and 0 < eps < 1
    assert abs(flux.sum() - inflow) <= R.MASS_BALANCE_TOL * inflow
    assert not R.is_steady(np.array([1.0, 0.0, 0.0]), 1.0, 0.0, 0.0, 1e-8)
    assert not R.is_steady(np.array([0.5, 0.1, 0.1]), 1.0, 1 / 7, 1 / 7, 1e-8)
    assert R.is_steady(np.array([0.8, 0.1, 0.1]), 1.0, 0.1, 0.1, 1e-8)
