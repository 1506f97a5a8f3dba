"""The two-step launch by marching wavefronts (flags bit 9) against the
LDS-tile two-step kernel (the default) and against single steps (flags
bit 8), on lattices whose width leaves a one-column last strip, puts
the outlet at a strip's first or last lane, and whose height leaves a ragged
last strip row; both reaction types, catalysts touching strip edges.  Node
arithmetic is shared, so FP32 fields agree bit for bit."""
import numpy as np
import pytest
import torch

from workloads import CAT1, CAT2, channel, rasterize
from workloads.configs import Workload, lattice_params
from workloads.geometry import classify_surface

pytestmark = pytest.mark.gpu


def _workload(nx, ny, centres, r=3, pe=3.0, da=5.0):
    t = channel(nx, ny)
    own = rasterize(t, centres, r)
    surf = classify_surface(t, own)
    t[surf & (own % 2 == 0)] = CAT1
    t[surf & (own % 2 == 1)] = CAT2
    rng = np.random.default_rng(nx * 1000 + ny)
    k = np.where(t >= CAT1, rng.uniform(0.05, 0.4, size=t.shape), 0.0)
    return Workload(f"m{nx}x{ny}", t, k, 3, lattice_params(pe, da, r), real="f32")


SHAPES = [
    (65, 23, [(20, 11), (60, 12)]),            # last strip: one column, the outlet
    (75, 23, [(20, 11), (45, 12), (63, 10)]),  # disc across the strip edge x = 64
    (128, 40, [(30, 20), (64, 18), (100, 25)]),  # outlet at the last lane of a strip
    (129, 37, [(10, 18), (63, 9), (66, 28)]),  # one-column last strip, ragged rows
    (200, 100, [(60, 50), (127, 30), (128, 70)]),
]


def _run(w, flags, flow_steps=300, blocks=(1, 2, 3, 5, 17, 300, 1001)):
    import paper_2109_04455_amd as L
    p = L.params(w.nx, w.ny, real="f32", nspecies=3, tau_f=w.tau_f, u0=w.u0, tau_g=w.tau_g,
                 c_in=w.c_in, vel_scale=w.vel_scale, flags=flags)
    c = L.Context(p)
    c.set_geometry(w.node_type)
    c.set_rates(w.k)
    c.flow_init()
    c.flow_run(flow_steps)
    c.adr_init()
    for n in blocks:
        c.adr_run(n, check_every=n, tol=0)
    eps, N, inflow = c.efficiency()
    out = [c.concentration(s) for s in range(3)], N, inflow, c.adr_steps()
    c.close()
    return out


@pytest.mark.parametrize("nx,ny,centres", SHAPES)
def test_march_equals_lds_tile_and_single_steps(nx, ny, centres):
    w = _workload(nx, ny, centres)
    march = _run(w, 512)
    tile = _run(w, 0)
    single = _run(w, 256)
    assert march[3] == tile[3] == single[3] == 1329
    for s in range(3):
        assert torch.equal(march[0][s], tile[0][s]), f"species {s} march != LDS tile"
        d = (march[0][s].double() - single[0][s].double()).abs().max().item()
        assert d <= 1e-6 * single[0][s].double().abs().max().item()
        assert march[0][s].abs().max().item() > 0 or s == 2
    assert np.array_equal(march[1], tile[1]) and march[2] == tile[2]


@pytest.mark.parametrize("name", ["C1q", "C2q"])
def test_march_equals_lds_tile_on_scaled_configs(name):
    from workloads import make_workload
    w = make_workload(name)
    a = _run(w, 512, flow_steps=500, blocks=(999,))
    b = _run(w, 0, flow_steps=500, blocks=(999,))
    for s in range(3):
        assert torch.equal(a[0][s], b[0][s])


def test_march_two_species():
    w = _workload(200, 60, [(50, 30), (120, 28)])
    import dataclasses
    w2 = dataclasses.replace(w, nspecies=2)
    import paper_2109_04455_amd as L
    res = []
    for flags in (0, 512):
        p = L.params(w2.nx, w2.ny, real="f32", nspecies=2, tau_g=w2.tau_g, vel_scale=w2.vel_scale,
                     flags=flags)
        c = L.Context(p)
        c.set_geometry(w2.node_type)
        c.set_rates(w2.k)
        c.flow_init()
        c.flow_run(300)
        c.adr_init()
        c.adr_run(777, tol=0)
        res.append([c.concentration(s) for s in range(2)])
        c.close()
    for s in range(2):
        assert torch.equal(res[0][s], res[1][s])
