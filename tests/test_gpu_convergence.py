"""GPU convergence loops, the velocity hand-off and the Pe range of the
side-by-side membrane, against the FP64 oracle.

* flow to a tolerance (max |u(t) - u(t - 1000)| <= tol u0): the GPU stops at
  the oracle's step count with the oracle's velocity;
* the steady-state test of the ADR run: with short checks it must not stop
  while the product is still upstream of the flux plane; the stop step of
  the oracle's run is stored in tests/golden/c0_short_checks.json;
* the ADR velocity is the flow velocity scaled by vel_scale (the paper's
  linear scaling of one Stokes flow), checked at scales below and above 1 and
  on a low-Pe sweep instance whose scale comes from the (Pe, Da) mapping;
* the side-by-side membrane at a quarter of its size over the paper's Pe
  range 1 ... 1000 (tau_g 1.4 ... 0.5009), FP32 state against the oracle's
  stored results (tests/golden/c2q_pe<Pe>.json, written by make_golden.py).
  After 500 flow steps the velocity still carries the start-up transient
  (weakly compressible, so C_A rises above c_in in places) and after 3000 ADR
  steps the products have barely reached the flux plane: the comparison is of
  the arithmetic on the fields, the fluxes and the totals, not of a steady
  efficiency.
"""
import dataclasses
import json
import os

import numpy as np
import pytest
import torch

from oracle import lbref as R
from workloads import batch_instances, make_workload

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _ctx(w, real, **kw):
    import paper_2109_04455_amd as L
    p = L.params(w.nx, w.ny, real=real, nspecies=w.nspecies, tau_f=w.tau_f, u0=w.u0,
                 tau_g=w.tau_g, c_in=w.c_in, vel_scale=w.vel_scale, **kw)
    c = L.Context(p)
    c.set_geometry(w.node_type)
    c.set_rates(w.k)
    return c


def _with_scale(w, scale):
    return dataclasses.replace(w, params=dataclasses.replace(w.params, vel_scale=scale))


# ------------------------------------------------------- flow convergence
def test_flow_steady_stops_where_the_oracle_stops():
    w = make_workload("rw")
    ux, uy, steps, res = R.flow_steady(w.node_type, w.tau_f, w.u0, 100000, check_every=1000,
                                       tol=1e-6)
    assert steps < 100000
    c = _ctx(w, "f64")
    c.flow_init()
    s, r, conv = c.flow_steady(100000, 1000, 1e-6)
    print("oracle", steps, res / w.u0, "gpu", s, r / w.u0, flush=True)
    assert conv and s == steps
    assert abs(r - res) <= 1e-9 * w.u0
    gx, gy = c.get_velocity()
    du = max(np.abs(gx.cpu().numpy() - ux).max(), np.abs(gy.cpu().numpy() - uy).max())
    assert du <= 1e-10 * w.u0


def test_flow_steady_reports_not_converged_within_budget():
    w = make_workload("rw")
    c = _ctx(w, "f64")
    c.flow_init()
    s, r, conv = c.flow_steady(3000, 1000, 1e-6)
    assert not conv and s == 3000 and r > 1e-6 * w.u0


# ------------------------------------------------- ADR steady-state test
def test_short_checks_do_not_stop_before_the_product_leaves():
    ref = json.load(open(os.path.join(HERE, "golden", "c0_short_checks.json")))
    w = make_workload("C0")
    c = _ctx(w, "f64")
    c.flow_init()
    c.flow_run(ref["flow_steps"])
    c.adr_init()
    steps, conv = c.adr_run(400000, check_every=ref["check_every"], tol=ref["tol"])
    eps, N, inflow = c.efficiency()
    print("gpu", steps, eps, "oracle", ref["adr_steps"], ref["eps"], flush=True)
    assert conv and steps == ref["adr_steps"]
    assert N[-1] > 0 and abs(N.sum() - inflow) <= 1e-3 * inflow
    assert abs(eps / ref["eps"] - 1) < 1e-9


def test_no_product_never_counts_as_steady():
    # only type-2 catalysts with two species: the product flux stays 0, so no
    # check is steady and the run reports that it did not converge
    import paper_2109_04455_amd as L
    w = make_workload("tiny")
    k = w.k.copy()
    k[w.node_type == 2] = 0.0
    w2 = dataclasses.replace(w, k=k)
    c = _ctx(w2, "f64")
    c.flow_init()
    c.flow_run(500)
    c.adr_init()
    steps, conv = c.adr_run(3000, check_every=100, tol=1e-6)
    assert not conv and steps == 3000
    with pytest.raises(L.LbfNotConverged):
        c.adr_run(200, check_every=100, tol=1e-6, raise_not_converged=True)


# ------------------------------------------------------ velocity hand-off
@pytest.mark.parametrize("scale", [0.2, 3.0])
@pytest.mark.parametrize("real,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_scaled_velocity_parity(scale, real, tol):
    w = _with_scale(make_workload("tiny"), scale)
    ux, uy, _, _ = R.flow_steady(w.node_type, w.tau_f, w.u0, 1500, tol=0)
    g = R.adr_init(w.node_type, ux, uy, 3, w.c_in, scale)
    R.adr_run(w.node_type, w.k, ux, uy, g, w.tau_g, 2000, w.c_in, scale)
    cref = R.adr_concentration(w.node_type, g)
    flux, inflow = R.adr_observe(w.node_type, g, w.c_in)
    c = _ctx(w, real)
    c.flow_init()
    c.flow_run(1500)
    c.adr_init()
    c.adr_run(2000, tol=0)
    eps, N, gin = c.efficiency()
    for s in range(3):
        e = np.abs(c.concentration(s).double().cpu().numpy() - cref[s]).max() / np.abs(cref[s]).max()
        assert e <= tol, f"species {s}: {e:.2e}"
    assert np.abs(N - flux).max() <= tol * abs(inflow)
    # the scale really enters: the unscaled run is far off
    if real == "f64":
        g1 = R.adr_init(w.node_type, ux, uy, 3, w.c_in, 1.0)
        R.adr_run(w.node_type, w.k, ux, uy, g1, w.tau_g, 2000, w.c_in, 1.0)
        assert np.abs(R.adr_concentration(w.node_type, g1)[1] - cref[1]).max() > 1e-3 * np.abs(cref[1]).max()


def test_low_peclet_sweep_instance_parity():
    # instance 57 of the 64-instance sweep: Pe = 0.16, so D is clamped at 1/2
    # (tau_g = 2) and the ADR runs on 0.20 x the flow; FP32 state
    w = batch_instances()[57]
    assert 0.19 < w.vel_scale < 0.21 and w.tau_g == 2.0
    ux, uy, _, _ = R.flow_steady(w.node_type, w.tau_f, w.u0, 300, tol=0)
    g = R.adr_init(w.node_type, ux, uy, 3, w.c_in, w.vel_scale)
    R.adr_run(w.node_type, w.k, ux, uy, g, w.tau_g, 600, w.c_in, w.vel_scale)
    cref = R.adr_concentration(w.node_type, g)
    flux, inflow = R.adr_observe(w.node_type, g, w.c_in)
    c = _ctx(w, "f32")
    c.flow_init()
    c.flow_run(300)
    c.adr_init()
    c.adr_run(600, tol=0)
    eps, N, gin = c.efficiency()
    for s in range(3):
        ref = cref[s]
        if np.abs(ref).max() == 0:
            continue
        e = np.abs(c.concentration(s).double().cpu().numpy() - ref).max() / np.abs(ref).max()
        assert e <= 1e-4, f"species {s}: {e:.2e}"
    assert np.abs(N - flux).max() <= 1e-5 * abs(inflow)
    assert abs(gin - inflow) <= 1e-5 * abs(inflow)


# ------------------------------------- side-by-side membrane over Pe
@pytest.mark.parametrize("pe", [1, 10, 100, 1000])
def test_c2_quarter_pe_range_parity(pe):
    ref = json.load(open(os.path.join(HERE, "golden", f"c2q_pe{pe}.json")))
    w = make_workload("C2q", pe=float(pe))
    assert abs(w.tau_g - ref["tau_g"]) < 1e-15
    c = _ctx(w, "f32")
    c.flow_init()
    c.flow_run(ref["flow_steps"])
    c.adr_init()
    steps, _ = c.adr_run(ref["adr_steps"], tol=0)
    assert ref["finite"], "the oracle itself diverged"
    eps, N, inflow = c.efficiency()
    tot = c.totals()
    conc = [c.concentration(s).double().cpu().numpy() for s in range(3)]
    nodes = np.asarray(ref["nodes"])
    print(f"Pe {pe} tau_g {w.tau_g:.4f}: eps {eps:.6e} (oracle {ref['eps']:.6e})", flush=True)
    for s in range(3):
        cmax = ref["cmax"][s]
        if cmax == 0:
            assert np.abs(conc[s]).max() == 0
            continue
        got = conc[s][nodes[:, 0], nodes[:, 1]]
        e = np.abs(got - np.asarray(ref["c_nodes"][s])).max() / cmax
        assert e <= 1e-4, f"species {s} sampled-node error {e:.2e}"
        a = ref["argmax"][s]
        assert abs(conc[s][a[0], a[1]] - ref["c_argmax"][s][s]) <= 1e-4 * cmax
        assert abs(np.abs(conc[s]).max() - cmax) <= 1e-4 * cmax
        assert abs(tot[s] - ref["totals"][s]) <= 1e-4 * abs(ref["totals"][0])
    assert np.abs(N - np.asarray(ref["N"])).max() <= 1e-5 * abs(ref["inflow"])
    assert abs(inflow - ref["inflow"]) <= 1e-5 * abs(ref["inflow"])
    if ref["eps"] > 1e-6:
        assert abs(eps / ref["eps"] - 1) <= 1e-4
