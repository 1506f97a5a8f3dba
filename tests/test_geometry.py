"""Input-generator checks: seeded fibre placement, rasterisation, surface
classification and the (Pe, Da) -> lattice mapping (paper Sec. "System
parameters and dimensionless numbers", Sec. "Membrane generation")."""
import numpy as np
import pytest

from workloads import (CAT1, CAT2, FLUID, SOLID, batch_instances, lattice_params,
                       make_workload, surface_counts)


def _brute_surface(r):
    # integer points inside the disc with a 4-neighbour outside it
    n = 0
    for x in range(-r - 1, r + 2):
        for y in range(-r - 1, r + 2):
            if x * x + y * y > r * r:
                continue
            if any((x + dx) ** 2 + (y + dy) ** 2 > r * r
                   for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1))):
                n += 1
    return n


@pytest.mark.parametrize("r", [3, 4, 6, 8, 10])
def test_surface_counts(r):
    assert surface_counts(r) == _brute_surface(r)


def test_known_surface_counts():
    assert [surface_counts(r) for r in (3, 6, 8, 10)] == [16, 32, 44, 56]


def test_lattice_params_paper_consistency():
    # the paper's isolated fibre: R = 5, Da = 150 <-> k = 1 and Da = 1.5 <->
    # k = 0.01 with tau_g = 1 (D = 1/6)
    d = 1.0 / 6.0
    assert abs(150 * d / 25 - 1.0) < 1e-12 and abs(1.5 * d / 25 - 0.01) < 1e-12
    p = lattice_params(10.0, 1.0, 10)
    assert abs(p.d - 0.05) < 1e-15 and abs(p.tau_g - 0.65) < 1e-15 and abs(p.k - 5e-4) < 1e-15
    p = lattice_params(0.1, 1.0, 8)          # D would be 4 -> clamped, flow scaled
    assert p.d == 0.5 and p.tau_g == 2.0 and abs(p.vel_scale - 0.125) < 1e-15
    # Pe is preserved by the scaling: Pe = (s u0) R / D
    assert abs(p.vel_scale * 0.05 * 8 / p.d - 0.1) < 1e-12


def test_c0_geometry():
    w = make_workload("C0")
    assert (w.nx, w.ny) == (200, 100)
    assert (w.node_type[0] == SOLID).all() and (w.node_type[-1] == SOLID).all()
    assert (w.node_type == CAT1).sum() == 56 and (w.node_type == CAT2).sum() == 0
    assert (w.k[w.node_type == CAT1] == 5e-4).all() and (w.k[w.node_type < CAT1] == 0).all()
    assert w.node_type[50, 60] == SOLID  # disc centre (interior node is inert)


def test_c1_geometry_deterministic_and_valid():
    a = make_workload("C1")
    b = make_workload("C1")
    assert (a.node_type == b.node_type).all() and a.centres == b.centres
    assert len(a.centres) == 40
    r, gap = 8, 2
    for i, (x1, y1) in enumerate(a.centres):
        band = (400, 800) if i < 20 else (1000, 1400)
        assert band[0] + r <= x1 <= band[1] - r
        assert r + gap + 1 <= y1 <= a.ny - 2 - r - gap
        for (x2, y2) in a.centres[:i]:
            assert (x1 - x2) ** 2 + (y1 - y2) ** 2 >= (2 * r + gap + 1) ** 2
    assert (a.node_type == CAT1).sum() == 20 * 44 and (a.node_type == CAT2).sum() == 20 * 44
    assert a.nspecies == 3 and a.real == "f32"


def test_c2_side_by_side_split():
    w = make_workload("C2q")
    n1, n2 = (w.node_type == CAT1).sum(), (w.node_type == CAT2).sum()
    assert n1 + n2 == 12 * 32
    assert 0.35 < n1 / (n1 + n2) < 0.65


def test_batch_instances():
    inst = batch_instances(n=4)
    again = batch_instances(n=4)
    for a, b in zip(inst, again):
        assert (a.node_type == b.node_type).all() and a.params == b.params
        assert a.ny == 256 and 512 <= a.nx <= 2048
        assert 0.1 <= a.params.pe <= 1000 and 0.01 <= a.params.da <= 100
        assert 0.5 < a.params.tau_g <= 2.0
        assert (a.node_type == FLUID).sum() > 0.8 * a.nx * (a.ny - 2)
