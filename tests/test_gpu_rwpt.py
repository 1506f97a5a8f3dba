"""GPU random-walk particle tracker vs the oracle's tracker.  Both draw their
random numbers from the same counter-based generator (splitmix64 keyed by
particle id, step and draw), each written from its published definition, so a
particle's path is a deterministic function of its id and start: the two must
agree trajectory by trajectory (positions to round-off, species exactly) and,
over a whole run with insertion and removal, in the crossing counts.  The only
allowed differences come from the last-bit differences of the two sides'
sin/cos, which may flip a reflection or reaction decision of a particle that
sits within an ulp of a face."""
import numpy as np
import pytest
import torch

from oracle import lbref as R
from oracle import rwpt
from workloads import make_workload

pytestmark = pytest.mark.gpu


def _lbf():
    import paper_2109_04455_amd as L
    return L


@pytest.fixture(scope="module")
def flows():
    out = {}
    for name, da in (("rw", 5.0), ("tiny", 10.0)):
        w = make_workload(name, da=da)
        ux, uy, _, _ = R.flow_steady(w.node_type, w.tau_f, w.u0, 4000, tol=0)
        out[name] = (w, ux, uy)
    return out


def _start(w, n, seed):
    rng = np.random.default_rng(seed)
    fy, fx = np.nonzero(w.node_type == 0)
    pick = rng.integers(0, fx.size, size=n)
    x = fx[pick] - 0.5 + rng.random(n)
    y = fy[pick] - 0.5 + rng.random(n)
    ids = rng.integers(0, 2 ** 62, size=n, dtype=np.int64).astype(np.uint64)
    return ids, x, y


@pytest.mark.parametrize("name,ns,vel_scale", [("rw", 2, 1.0), ("tiny", 3, 4.0), ("tiny", 3, 60.0)])
def test_trajectories_match_oracle(flows, name, ns, vel_scale):
    # vel_scale 60: advection moves up to 1.5 cells per step, beyond the 5 x 5
    # window of cell types the GPU step reads at once, so its direct reads of
    # the cells outside the window are exercised as well
    L = _lbf()
    w, ux, uy = flows[name]
    D = w.params.d
    ids, x, y = _start(w, 20000, 5)
    sp = np.zeros(x.size, np.uint8)
    kw = dict(vel_scale=vel_scale * w.vel_scale, rate_w=1.0 / 6.0, dt=0.5, zone=1.0, wall_mode=1,
              seed=77)
    steps = 400
    xo, yo, so = rwpt.walk(w.node_type, ux, uy, w.k * 20.0, ns, D, ids, x, y, sp, 3, steps, **kw)
    p = L.rw_params(w.nx, w.ny, nspecies=ns, D=D, dt=0.5, zone=1.0, rate_w=1.0 / 6.0,
                    vel_scale=vel_scale * w.vel_scale, seed=77, wall_mode=1)
    r = L.RandomWalk(p)
    r.set_fields(w.node_type, ux, uy, w.k * 20.0)
    xg, yg, sg = r.walk(ids, x, y, sp, 3, steps)
    xg, yg, sg = xg.cpu().numpy(), yg.cpu().numpy(), sg.cpu().numpy()
    r.close()
    assert (so > 0).mean() > (0.02 if vel_scale < 10 else 0.002)  # reactions happened
    d = np.abs(xg - xo) + np.abs(yg - yo)
    off = (d > 1e-9) | (sg != so)
    assert off.mean() <= 1e-3, off.mean()
    assert np.median(d) <= 1e-12


def test_full_run_crossing_counts_match_oracle(flows):
    L = _lbf()
    w, ux, uy = flows["rw"]
    D = w.params.d
    kw = dict(vel_scale=w.vel_scale, rate_w=1.0 / 6.0, density=5.0, dt=0.5, zone=1.0,
              wall_mode=1, seed=11)
    burn, meas = 1500, 3000
    n_or = rwpt.run(w.node_type, ux, uy, w.k, 2, D, burn_steps=burn, meas_steps=meas, **kw)
    p = L.rw_params(w.nx, w.ny, nspecies=2, D=D, **kw)
    r = L.RandomWalk(p)
    r.set_fields(w.node_type, ux, uy, w.k)
    r.fill()
    r.run(burn)
    r.run(meas, measure=True)
    n_gpu, held, steps = r.counts()
    r.close()
    assert steps == meas
    crossings_gpu = np.rint(n_gpu * meas * 0.5)
    crossings_or = np.rint(np.asarray(n_or) * meas * 0.5)
    assert crossings_or[0] > 1000 and crossings_or[1] > 50
    assert np.abs(crossings_gpu - crossings_or).max() <= 3, (crossings_gpu, crossings_or)


def test_graph_blocks_do_not_change_results(flows):
    # the compactions fall at the start of every captured block and every
    # nx / 8 steps inside one (12 on this 96-wide lattice): one-step blocks
    # compact every step, the others every 7 or 12 steps, with the same
    # crossings and particle counts
    L = _lbf()
    w, ux, uy = flows["rw"]
    out = []
    for chunks in ([600], [7] * 85 + [5], [1] * 600):
        p = L.rw_params(w.nx, w.ny, nspecies=2, D=w.params.d, vel_scale=w.vel_scale, density=5.0,
                        seed=3)
        r = L.RandomWalk(p)
        r.set_fields(w.node_type, ux, uy, w.k)
        r.fill()
        for n in chunks:
            r.run(n, measure=True)
        out.append(r.counts())
        r.close()
    for o in out[1:]:
        assert np.array_equal(out[0][0], o[0]) and out[0][1] == o[1]


def test_capacity_overflow_is_reported(flows):
    L = _lbf()
    w, ux, uy = flows["rw"]
    p = L.rw_params(w.nx, w.ny, nspecies=2, D=w.params.d, vel_scale=w.vel_scale, density=5.0,
                    capacity=1000)
    r = L.RandomWalk(p)
    r.set_fields(w.node_type, ux, uy, w.k)
    r.fill()
    r.run(3)
    with pytest.raises(L.LbfError):
        r.counts()
    r.close()
