"""GPU path vs the FP64 oracle for the reaction variant (every population of a
fluid node next to catalysts reacts, mean neighbour rate per type) and for the
pure-diffusion periodic box, with the species totals.

Bars as in the channel parity tests: FP64 within 1e-10, FP32 storage within
1e-4 (fields relative to their maximum, totals relative to the initial
amount).  Both sides get the same velocity (the oracle's steady flow, rounded
to the GPU storage precision) so the comparison isolates the ADR step.
"""
import numpy as np
import pytest
import torch

from oracle import lbref as R
from workloads import box_workload, make_workload

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-4}


def _lbf():
    import paper_2109_04455_amd as L
    return L


def _field_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _rounded(a, real):
    return a.astype(np.float32).astype(np.float64) if real == "f32" else a


def _gpu_adr(w, real, mode, ux, uy, steps):
    L = _lbf()
    p = L.params(w.nx, w.ny, real=real, nspecies=w.nspecies, tau_f=w.tau_f, u0=w.u0,
                 tau_g=w.tau_g, c_in=w.c_in, vel_scale=w.vel_scale, reaction_mode=mode,
                 boundary=w.boundary)
    c = L.Context(p)
    c.set_geometry(w.node_type)
    c.set_rates(w.k)
    dt = torch.float32 if real == "f32" else torch.float64
    c.set_velocity(torch.from_numpy(ux).to(dt), torch.from_numpy(uy).to(dt))
    c.adr_init()
    c.adr_run(steps, check_every=steps, tol=0)
    conc = np.stack([c.concentration(s).double().cpu().numpy() for s in range(w.nspecies)])
    return c, conc, c.totals()


def _oracle_adr(w, mode, ux, uy, steps):
    bc = (R.PERIODIC_X | R.PERIODIC_Y) if w.boundary == 1 else 0
    omode = R.NODE_AT_CATALYST if mode == 1 else R.LINK
    g = R.adr_init(w.node_type, ux, uy, w.nspecies, w.c_in, w.vel_scale)
    R.adr_run(w.node_type, w.k, ux, uy, g, w.tau_g, steps, w.c_in, w.vel_scale, mode=omode, bc=bc)
    return g, R.adr_concentration(w.node_type, g), R.adr_totals(w.node_type, g)


@pytest.mark.parametrize("real", ["f64", "f32"])
@pytest.mark.parametrize("morph,mode", [("pair", 0), ("side", 0), ("side", 1)])
def test_periodic_box_parity_and_totals(real, morph, mode):
    # 130 x 130 box (2 + ragged tiles of 256 x 1 per row, odd padding)
    w = box_workload(morph, real=real, n=130, xi=40)
    z = np.zeros((w.ny, w.nx))
    steps = 800
    print(f"box {morph} mode {mode} {real} steps {steps}", flush=True)
    c, conc, tot = _gpu_adr(w, real, mode, z, z, steps)
    _, oconc, otot = _oracle_adr(w, mode, z, z, steps)
    for s in range(3):
        e = _field_err(conc[s], oconc[s])
        assert e <= TOL[real], f"species {s} field error {e:.3e}"
    n0 = float((w.node_type == 0).sum()) * w.c_in
    assert np.abs(tot - otot).max() <= TOL[real] * n0
    # closed box: reactions move mass between species, bounce-back keeps it
    assert abs(tot.sum() - n0) <= (1e-12 if real == "f64" else 1e-5) * n0
    assert otot[2] > 0 and tot[2] > 0
    c.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_periodic_box_catalyst_across_both_seams(mode):
    # the same periodic problem, rolled so that one fibre sits on the corner
    # (x = 0 and y = 0 seams): links, reactions and bounce-back all wrap
    w = box_workload("pair", real="f64", n=130, xi=40)
    cx, cy = w.centres[0]
    w.node_type = np.ascontiguousarray(np.roll(w.node_type, (-cy, -cx), axis=(0, 1)))
    w.k = np.ascontiguousarray(np.roll(w.k, (-cy, -cx), axis=(0, 1)))
    z = np.zeros((w.ny, w.nx))
    c, conc, tot = _gpu_adr(w, "f64", mode, z, z, 600)
    _, oconc, otot = _oracle_adr(w, mode, z, z, 600)
    for s in range(3):
        assert _field_err(conc[s], oconc[s]) <= 1e-10
    assert np.abs(tot - otot).max() <= 1e-10 * otot.sum()
    # and equal to the unrolled problem (translation invariance of the box)
    w0 = box_workload("pair", real="f64", n=130, xi=40)
    _, oconc0, otot0 = _oracle_adr(w0, mode, z, z, 600)
    assert np.abs(np.roll(oconc0, (-cy, -cx), axis=(1, 2)) - oconc).max() <= 1e-12
    c.close()


@pytest.mark.parametrize("real", ["f64", "f32"])
def test_reaction_variant_channel_parity(real):
    w = make_workload("tiny")
    ux, uy, _, _ = R.flow_steady(w.node_type, w.tau_f, w.u0, 6000, tol=0)
    ux, uy = _rounded(ux, real), _rounded(uy, real)
    steps = 3000
    c, conc, tot = _gpu_adr(w, real, 1, ux, uy, steps)
    g, oconc, otot = _oracle_adr(w, 1, ux, uy, steps)
    for s in range(3):
        e = _field_err(conc[s], oconc[s])
        assert e <= TOL[real], f"species {s} field error {e:.3e}"
    eps, N, inflow = c.efficiency()
    flux, oinflow = R.adr_observe(w.node_type, g, w.c_in)
    assert abs(eps - R.efficiency(flux)) <= TOL[real] * abs(R.efficiency(flux))
    assert np.abs(N - flux).max() <= TOL[real] * abs(oinflow)
    assert np.abs(tot - otot).max() <= TOL[real] * otot.sum()
    # the variant differs from link reactions on this geometry
    _, _, ltot = _oracle_adr(w, 0, ux, uy, steps)
    assert abs(ltot[2] - otot[2]) > 0.5 * otot[2]
    c.close()


@pytest.mark.parametrize("morph", ["pair", "side"])
def test_full_box_totals_conserved_and_monotone(morph):
    # the paper's 300 x 300 box, Da 150: no oracle at this length; properties
    # that hold at any size -- conservation of A + B + C, A falls, C rises
    w = box_workload(morph, real="f32")
    z = np.zeros((w.ny, w.nx))
    print(f"full box {morph}", flush=True)
    c, _, tot = _gpu_adr(w, "f32", 0, z, z, 1)
    n0 = float((w.node_type == 0).sum()) * w.c_in
    prev = tot
    for _ in range(10):
        c.adr_run(2000, check_every=2000, tol=0)
        tot = c.totals()
        assert abs(tot.sum() - n0) <= 1e-5 * n0
        assert tot[0] < prev[0] and tot[2] > prev[2]
        prev = tot
    c.close()


def test_totals_match_oracle_in_channel():
    w = make_workload("C0")
    ux, uy, _, _ = R.flow_steady(w.node_type, w.tau_f, w.u0, 3000, tol=0)
    c, _, tot = _gpu_adr(w, "f64", 0, ux, uy, 700)
    _, _, otot = _oracle_adr(w, 0, ux, uy, 700)
    assert np.abs(tot - otot).max() <= 1e-10 * otot.sum()
    c.close()


@pytest.mark.parametrize("real", ["f64", "f32"])
@pytest.mark.parametrize("case,mode", [("box", 0), ("box", 1), ("channel", 0), ("channel", 1)])
def test_production_matches_oracle(real, case, mode):
    # reaction production after n steps against the oracle's from its state
    # after n steps: 130 x 130 side-by-side box and the 64 x 32 cascade
    # channel with its flow, both reaction forms
    if case == "box":
        w = box_workload("side", real=real, n=130, xi=40)
        ux = uy = np.zeros((w.ny, w.nx))
    else:
        w = make_workload("tiny")
        ux, uy, _, _ = R.flow_steady(w.node_type, w.tau_f, w.u0, 3000, tol=0)
        ux, uy = _rounded(ux, real), _rounded(uy, real)
    steps = 600
    print(f"production {case} mode {mode} {real}", flush=True)
    c, _, _ = _gpu_adr(w, real, mode, ux, uy, steps)
    r = c.production()
    c.close()
    g, _, _ = _oracle_adr(w, mode, ux, uy, steps)
    bc = (R.PERIODIC_X | R.PERIODIC_Y) if w.boundary == 1 else 0
    ro = R.adr_production(w.node_type, w.k, g, R.NODE_AT_CATALYST if mode == 1 else R.LINK, bc)
    assert r.shape == ro.shape == (w.nspecies - 1,)
    assert (ro > 0).all()
    assert np.abs(r - ro).max() <= TOL[real] * ro.max()


@pytest.mark.parametrize("mode", [0, 1])
def test_production_is_the_change_of_the_totals_in_a_closed_box(mode):
    # one GPU step changes the totals of A, B, C by -r0, r0 - r1, r1
    w = box_workload("side", real="f64", n=130, xi=40)
    z = np.zeros((w.ny, w.nx))
    c, _, before = _gpu_adr(w, "f64", mode, z, z, 500)
    r = c.production()
    c.adr_run(1, check_every=1, tol=0)
    d = c.totals() - before
    c.close()
    scale = before.sum()
    assert r[0] > 0 and r[1] > 0
    assert abs(d[0] + r[0]) <= 1e-12 * scale
    assert abs(d[1] - (r[0] - r[1])) <= 1e-12 * scale
    assert abs(d[2] - r[1]) <= 1e-12 * scale


def test_production_equals_the_product_outflow_at_steady_state():
    # C0 run to a tight steady state: the A -> B conversion per step equals
    # the B leaving through the outlet face (the paper's production rate),
    # and the inflow minus it the A leaving
    L = _lbf()
    w = make_workload("C0")
    p = L.params(w.nx, w.ny, real="f64", nspecies=w.nspecies, tau_f=w.tau_f, u0=w.u0,
                 tau_g=w.tau_g, c_in=w.c_in, vel_scale=w.vel_scale)
    c = L.Context(p)
    c.set_geometry(w.node_type)
    c.set_rates(w.k)
    c.flow_init()
    c.flow_run(10000)
    c.adr_init()
    steps, conv = c.adr_run(400000, check_every=1000, tol=1e-11)
    eps, N, inflow = c.efficiency()
    r = c.production()
    c.close()
    print("C0 steady", steps, conv, r, N, inflow, flush=True)
    assert conv and r.shape == (1,)
    assert abs(r[0] - N[1]) <= 1e-7 * inflow
    assert abs(inflow - r[0] - N[0]) <= 1e-7 * inflow


def test_periodic_box_rejects_channel_only_calls():
    L = _lbf()
    w = box_workload("pair", real="f64", n=64, xi=20)
    z = np.zeros((w.ny, w.nx))
    c, _, _ = _gpu_adr(w, "f64", 0, z, z, 10)
    with pytest.raises(L.LbfError):
        c.flow_init()
    with pytest.raises(L.LbfError):
        c.efficiency()
    with pytest.raises(L.LbfError):
        c.adr_run(100, check_every=10, tol=1e-6)
    with pytest.raises(L.LbfError):
        c.adjoint(5, ckpt_every=5)
    c.close()
