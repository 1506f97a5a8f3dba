"""3D GPU path (D3Q19 forced flow, D3Q7 ADR) vs the FP64 3D oracle, element
by element on the same seeded inputs.  Bars: FP64 within 1e-10 (fields
relative to their maximum, fluxes relative to the inflow, eps); FP32 storage
within 1e-4."""
import numpy as np
import pytest
import torch

from oracle import lbref3d as R
from workloads.configs3d import make_workload3d

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-4}


def _lbf():
    import paper_2109_04455_amd as L
    return L


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _ctx(w, real, vel_scale=1.0, **kw):
    L = _lbf()
    p = L.params3d(w.nx, w.ny, w.nz, real=real, nspecies=w.nspecies, tau_f=w.tau_f,
                   force_x=w.force, tau_g=w.tau_g, c_in=w.c_in, vel_scale=vel_scale, **kw)
    c = L.Context3D(p)
    c.set_geometry(w.node_type)
    c.set_rates(w.k)
    return c


def _oracle(w, flow_steps, adr_steps, vel_scale, u=None):
    if u is None:
        u, _ = R.flow(w.node_type, w.tau_f, (w.force, 0.0, 0.0), flow_steps)
    g = R.adr_init(w.node_type, u, w.nspecies, w.c_in, vel_scale)
    R.adr_run(w.node_type, w.k, u, g, w.tau_g, adr_steps, w.c_in, vel_scale)
    flux, inflow = R.adr_observe(w.node_type, g, w.c_in)
    return {"u": u, "c": R.adr_concentration(w.node_type, g), "N": flux, "inflow": inflow,
            "eps": R.efficiency(flux), "tot": R.adr_totals(w.node_type, g)}


def _gpu(w, real, flow_steps, adr_steps, vel_scale, u=None, **kw):
    c = _ctx(w, real, vel_scale, **kw)
    if u is None:
        c.flow_init()
        c.flow_run(flow_steps)
    else:
        c.set_velocity(torch.from_numpy(u))
    ug = c.get_velocity().double().cpu().numpy()
    c.adr_init()
    c.adr_run(adr_steps, check_every=max(adr_steps, 1), tol=0)
    eps, N, inflow = c.efficiency()
    conc = np.stack([c.concentration(s).double().cpu().numpy() for s in range(w.nspecies)])
    return {"u": ug, "c": conc, "N": N, "inflow": inflow, "eps": eps, "tot": c.totals(), "ctx": c}


def _compare(g, o, tol, check_u=True):
    if check_u:
        assert _rel(g["u"], o["u"]) <= tol, f"velocity error {_rel(g['u'], o['u']):.3e}"
    for s in range(len(o["N"])):
        e = _rel(g["c"][s], o["c"][s])
        assert e <= tol, f"species {s} field error {e:.3e}"
    dn = np.abs(np.asarray(g["N"]) - o["N"]).max() / abs(o["inflow"])
    assert dn <= tol, f"flux error {dn:.3e}"
    assert abs(g["inflow"] - o["inflow"]) <= tol * abs(o["inflow"])
    # eps = N_last / sum N moves by ~ dN / sum N, bounded by the flux check
    assert abs(g["eps"] - o["eps"]) <= tol * max(abs(o["eps"]), 1e-2)
    assert np.abs(g["tot"] - o["tot"]).max() <= tol * o["tot"].sum()


@pytest.fixture(scope="module")
def m3t_oracle():
    w = make_workload3d("M3t", real="f64")
    return w, _oracle(w, 400, 800, 150.0)


@pytest.mark.parametrize("real", ["f64", "f32"])
def test_m3t_flow_and_adr_parity(m3t_oracle, real):
    w, o = m3t_oracle
    print(f"M3t {real}", flush=True)
    g = _gpu(w, real, 400, 800, 150.0)
    assert o["eps"] > 1e-4 and np.abs(o["u"][0]).max() > 1e-2 / 150.0
    _compare(g, o, TOL[real])
    g["ctx"].close()


def test_m3t_adr_on_imported_velocity_fp32():
    # the same ADR on the oracle's FP32-rounded velocity: isolates the ADR step
    w = make_workload3d("M3t")
    u, _ = R.flow(w.node_type, w.tau_f, (w.force, 0.0, 0.0), 400)
    u = u.astype(np.float32).astype(np.float64)
    o = _oracle(w, 0, 600, 40.0, u=u)
    g = _gpu(w, "f32", 0, 600, 40.0, u=u)
    _compare(g, o, TOL["f32"], check_u=False)
    g["ctx"].close()


def test_multi_tile_ragged_box_fp64():
    # 300 nodes per row: two 256-node tiles, the second ragged; odd ny, nz
    w = make_workload3d("M3t", real="f64")
    t = np.zeros((7, 9, 300), np.uint8)
    t[:, :, :40] = w.node_type[:7, :9, :]
    t[:, :, 150:190] = w.node_type[:7, :9, :]
    w.node_type = t
    w.k = np.where(t >= 2, w.params.k, 0.0)
    o = _oracle(w, 200, 250, 40.0)
    g = _gpu(w, "f64", 200, 250, 40.0)
    _compare(g, o, TOL["f64"])
    g["ctx"].close()


@pytest.mark.parametrize("name", ["M3c", "M3s"])
def test_paper_boxes_short_run_fp32(name):
    # the paper's 200x60x60 and 160x60x60 membranes at full size, a short run
    w = make_workload3d(name)
    print(f"{name} full size", flush=True)
    o = _oracle(w, 20, 20, 20.0)
    g = _gpu(w, "f32", 20, 20, 20.0)
    _compare(g, o, TOL["f32"])
    g["ctx"].close()


def test_streaming_cached_and_graph_paths_bit_identical():
    w = make_workload3d("M3t")
    outs = []
    for flags, chunks in ((2, [300]), (64, [300]), (2, [5] * 60)):
        c = _ctx(w, "f32", 40.0, flags=flags)
        c.flow_init()
        for n in chunks:
            c.flow_run(n)
        c.adr_init()
        for n in chunks:
            c.adr_run(n, check_every=n, tol=0)
        outs.append([c.concentration(s).cpu() for s in range(3)] + [c.get_velocity().cpu()])
        c.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert torch.equal(a, b)


def test_velocity_roundtrip_and_error_paths():
    L = _lbf()
    w = make_workload3d("M3t")
    c = _ctx(w, "f32")
    with pytest.raises(L.LbfError):
        c.efficiency()                       # no ADR step yet
    with pytest.raises(L.LbfError):
        c.set_rates(np.where(w.node_type >= 2, 2.0, 0.0))
    u = torch.randn((3,) + w.shape, dtype=torch.float32) * 1e-3
    u[:, torch.from_numpy(w.node_type) != 0] = 0
    c.set_velocity(u)
    assert torch.equal(c.get_velocity().cpu(), u)
    c.close()
