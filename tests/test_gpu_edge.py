"""Degenerate inputs of the 2D path against the oracle: no reaction (Da = 0),
a channel blocked by a solid wall (nothing reaches the outlet: eps is NaN by
the ABI's contract), the narrowest channel (one fluid row) and the smallest
accepted width."""
import numpy as np
import pytest
import torch

from oracle import lbref as R
from workloads import channel, make_workload

pytestmark = pytest.mark.gpu


def _lbf():
    import paper_2109_04455_amd as L
    return L


def _run(node_type, k, real, flow_steps, adr_steps, nspecies=3, velocity=None, tau_g=0.7):
    L = _lbf()
    ny, nx = node_type.shape
    p = L.params(nx, ny, real=real, nspecies=nspecies, tau_g=tau_g)
    c = L.Context(p)
    c.set_geometry(node_type)
    c.set_rates(k)
    if velocity is None:
        c.flow_init()
        c.flow_run(flow_steps)
    else:
        dt = torch.float64 if real == "f64" else torch.float32
        c.set_velocity(torch.from_numpy(velocity[0]).to(dt), torch.from_numpy(velocity[1]).to(dt))
    c.adr_init()
    c.adr_run(adr_steps, check_every=adr_steps, tol=0)
    conc = np.stack([c.concentration(s).double().cpu().numpy() for s in range(nspecies)])
    return c, conc


def _oracle(node_type, k, flow_steps, adr_steps, nspecies=3, velocity=None, tau_g=0.7):
    if velocity is None:
        ux, uy, _, _ = R.flow_steady(node_type, 0.8, 0.05, flow_steps, tol=0)
    else:
        ux, uy = velocity
    g = R.adr_init(node_type, ux, uy, nspecies)
    R.adr_run(node_type, k, ux, uy, g, tau_g, adr_steps)
    flux, inflow = R.adr_observe(node_type, g)
    return g, R.adr_concentration(node_type, g), flux, inflow


def test_no_reaction_gives_exactly_zero_products():
    w = make_workload("C0")
    k = np.zeros_like(w.k)
    c, conc = _run(w.node_type, k, "f64", 2000, 3000, nspecies=2)
    eps, N, inflow = c.efficiency()
    assert N[1] == 0.0 and eps == 0.0
    assert np.all(conc[1] == 0.0)
    _, oc, flux, _ = _oracle(w.node_type, k, 2000, 3000, nspecies=2)
    assert np.abs(conc[0] - oc[0]).max() <= 1e-10 * np.abs(oc[0]).max()
    c.close()


def test_blocked_channel_reaches_nothing_and_eps_is_nan():
    t = channel(48, 12)
    t[:, 20] = 1                           # a solid wall across the channel
    t[5, 19] = 2                           # a catalyst on its upstream face
    k = np.where(t == 2, 0.2, 0.0)
    z = np.zeros(t.shape)
    c, conc = _run(t, k, "f64", 0, 2000, velocity=(z, z))
    eps, N, inflow = c.efficiency()
    # A starts uniform on both sides of the wall; without flow the part
    # beyond it stays uniform, so nothing crosses the outlet face and B, C
    # never get there (eps is NaN when sum N = 0, else 0)
    assert np.abs(N).max() <= 1e-14 and (np.isnan(eps) or eps == 0.0)
    assert np.all(conc[1:, :, 21:] == 0.0)
    _, oc, flux, _ = _oracle(t, k, 0, 2000, velocity=(z, z))
    assert np.all(flux == 0.0)
    for s in range(3):
        assert np.abs(conc[s] - oc[s]).max() <= 1e-10 * max(np.abs(oc[s]).max(), 1e-300)
    assert conc[1].max() > 0                # B is made at the catalyst
    c.close()


@pytest.mark.parametrize("nx,ny", [(16, 3), (8, 5)])
def test_smallest_channels_match_oracle(nx, ny):
    t = channel(nx, ny)
    if ny > 3:
        t[ny // 2, nx // 2] = 2            # one catalytic node in the middle
    k = np.where(t == 2, 0.3, 0.0)
    c, conc = _run(t, k, "f64", 300, 400)
    eps, N, inflow = c.efficiency()
    _, oc, flux, oinflow = _oracle(t, k, 300, 400)
    for s in range(3):
        assert np.abs(conc[s] - oc[s]).max() <= 1e-10 * max(np.abs(oc[s]).max(), 1e-300)
    assert np.abs(N - flux).max() <= 1e-10 * abs(oinflow)
    c.close()
