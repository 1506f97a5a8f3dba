"""64-bit population offsets where they are needed.  A channel whose flow
lattice exceeds 4 GiB (11000 x 11000 nodes, 9 FP32 planes of 121 M nodes)
takes the 64-bit instantiations of the node updates by itself.  An empty
channel whose bottom wall alternates A -> B and B -> C catalysts is periodic
along x (period 2) away from the inlet and the outlet, so after a few steps
its middle column equals, bit for bit, the middle column of a 64-node-wide
channel run the same way with 32-bit offsets (both middles at even x)."""
import numpy as np
import pytest
import torch

from workloads import channel

pytestmark = pytest.mark.gpu

NY = 11000
FLOW_STEPS, ADR_STEPS = 4, 5  # the inlet and outlet reach < 16 nodes inward


def _middle_columns(nx):
    import paper_2109_04455_amd as L
    t = channel(nx, NY)
    t[0, 0::2] = 2
    t[0, 1::2] = 3
    k = np.zeros(t.shape)
    k[0, :] = 0.1
    c = L.Context(L.params(nx, NY, real="f32", nspecies=3))
    c.set_geometry(t)
    c.set_rates(k)
    del t, k
    c.flow_init()
    c.flow_run(FLOW_STEPS)
    mid = nx // 2
    ux, uy = c.get_velocity()
    cols = [ux[:, mid].cpu(), uy[:, mid].cpu()]
    del ux, uy
    c.adr_init()
    c.adr_run(ADR_STEPS, check_every=ADR_STEPS, tol=0)   # two-step launches + a single step
    for s in range(3):
        cols.append(c.concentration(s)[:, mid].cpu())
    c.close()
    torch.cuda.empty_cache()
    return cols


def test_lattice_beyond_4gib_matches_narrow_channel():
    big = _middle_columns(11000)
    small = _middle_columns(64)
    for name, a, b in zip(("ux", "uy", "A", "B", "C"), big, small):
        assert torch.isfinite(a).all(), name
        assert torch.equal(a, b), name
    assert big[3][1].item() > 0 and big[4][1].item() > 0   # both reactions ran
