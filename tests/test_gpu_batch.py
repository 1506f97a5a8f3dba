"""Batched sweep: many uneven instances in one persistent, graph-captured
launch per step must give the same results as the single-lattice path
(bit for bit: the per-node arithmetic is the same code) and match the
oracle; converged instances leave the tile table and keep their state."""
import numpy as np
import pytest
import torch

from oracle import lbref as R
from workloads import batch_instances, make_workload

pytestmark = pytest.mark.gpu


def _params(w, real="f32", **kw):
    import paper_2109_04455_amd as L
    return L.params(w.nx, w.ny, real=real, nspecies=w.nspecies, tau_f=w.tau_f, u0=w.u0,
                    tau_g=w.tau_g, c_in=w.c_in, vel_scale=w.vel_scale, **kw)


def _single(w, flow_steps, adr_steps, real="f32", flags=0):
    # the same launch sequence as the batch: two-step launches unless flags
    # bit 8 asks for one step per launch
    import paper_2109_04455_amd as L
    c = L.Context(_params(w, real, variant=1, tile_x=256, tile_y=1, flags=flags))
    c.set_geometry(w.node_type)
    c.set_rates(w.k)
    c.flow_init()
    c.flow_run(flow_steps)
    c.adr_init()
    c.adr_run(adr_steps, tol=0)
    return c


def _agree(real, flags, fields_b, fields_s, obs_b, obs_s, inflow):
    # FP32 storage, or one step per launch: the batch and the single-lattice
    # path agree bit for bit.  Two-step launches in FP64 run the same node
    # code compiled into two kernels (multiply-adds fused per kernel): a few
    # ulps
    exact = real == "f32" or (flags & 256)
    for s, (a, b) in enumerate(zip(fields_b, fields_s)):
        d = (a.double() - b.double()).abs().max().item()
        print("species", s, "max |batch - single|", d, flush=True)
        if exact:
            assert torch.equal(a, b), s
        else:
            assert d <= 1e-12 * b.double().abs().max().item(), s
    (eb, pb), (es, ps) = obs_b, obs_s
    if exact:
        assert eb == es or (np.isnan(eb) and np.isnan(es))
        assert pb == ps
    else:
        assert abs(eb - es) <= 1e-12 * abs(es) or (np.isnan(eb) and np.isnan(es))
        assert abs(pb - ps) <= 1e-12 * abs(inflow)


def _instances(n=6, ny=48, seed=5):
    # small uneven two-membrane cascades with the sweep's Pe/Da draws
    ws = batch_instances(n=n, seed=seed, ny=ny, nx_range=(200, 400), fibres=2, r=8)
    return ws


@pytest.mark.parametrize("real,flags", [("f32", 0), ("f64", 0), ("f32", 128), ("f64", 256),
                                        ("f32", 256 | 128)])
def test_batch_equals_single_instance_path(real, flags):
    # flags bit 7: the batch addresses populations with 64-bit offsets, the
    # single-instance path with 32-bit ones; bit 8: one step per launch on
    # both sides.  The arithmetic is the same code
    import paper_2109_04455_amd as L
    ws = _instances()
    b = L.Batch([_params(w, real, flags=flags) for w in ws])
    b.set_geometry([w.node_type for w in ws], [w.k for w in ws])
    b.flow(600, check_every=600, tol=0)
    eps, prod, steps = b.run(1500, check_every=500, tol=0)
    for i, w in enumerate(ws):
        c = _single(w, 600, 1500, real, flags & 256)
        e1, N1, inflow = c.efficiency()
        assert steps[i] == 1500
        _agree(real, flags, [b.concentration(i, s) for s in range(3)],
               [c.concentration(s) for s in range(3)], (eps[i], prod[i]), (e1, N1[-1]), inflow)


def test_batch_matches_oracle():
    import paper_2109_04455_amd as L
    ws = _instances(n=3, seed=9)
    b = L.Batch([_params(w, "f64") for w in ws])
    b.set_geometry([w.node_type for w in ws], [w.k for w in ws])
    b.flow(500, check_every=500, tol=0)
    eps, prod, steps = b.run(800, check_every=800, tol=0)
    for i, w in enumerate(ws):
        ux, uy, _, _ = R.flow_steady(w.node_type, w.tau_f, w.u0, 500, tol=0)
        g = R.adr_init(w.node_type, ux, uy, 3, w.c_in, w.vel_scale)
        R.adr_run(w.node_type, w.k, ux, uy, g, w.tau_g, 800, w.c_in, w.vel_scale)
        flux, inflow = R.adr_observe(w.node_type, g, w.c_in)
        c = R.adr_concentration(w.node_type, g)
        for s in range(3):
            cg = b.concentration(i, s).cpu().numpy()
            assert np.abs(cg - c[s]).max() <= 1e-10 * max(np.abs(c[s]).max(), 1e-30)
        assert abs(prod[i] - flux[-1]) <= 1e-10 * abs(inflow)


def test_batch_convergence_drops_instances_and_keeps_their_state():
    # four small cascades that reach the steady-state test at tol 1e-7 after
    # different step counts (the oracle's stop steps and eps are stored in
    # tests/golden/batch_conv.json): each instance leaves the tile table at
    # the oracle's step, keeps its state while the others run on, and equals
    # a single-lattice run of exactly its own step count
    import json
    import os
    import paper_2109_04455_amd as L
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batch_conv.json")))
    kw = dict(ref["instances"])
    for k in ("nx_range", "pe_range", "da_range"):
        kw[k] = tuple(kw[k])
    ws = batch_instances(**kw)
    b = L.Batch([_params(w, "f64") for w in ws])
    b.set_geometry([w.node_type for w in ws], [w.k for w in ws])
    b.flow(ref["flow_steps"], check_every=ref["flow_steps"], tol=0)
    eps, prod, steps = b.run(ref["budget"], check_every=ref["check_every"], tol=ref["tol"])
    want = [r["adr_steps"] for r in ref["runs"]]
    print("batch steps", steps.tolist(), "oracle", want, flush=True)
    assert steps.tolist() == want
    assert (steps < ref["budget"]).sum() >= 2 and len(set(want)) >= 2
    for i, w in enumerate(ws):
        r = ref["runs"][i]
        c = _single(w, ref["flow_steps"], int(steps[i]), "f64")
        e1, N1, inflow = c.efficiency()
        _agree("f64", 0, [b.concentration(i, s) for s in range(w.nspecies)],
               [c.concentration(s) for s in range(w.nspecies)], (eps[i], prod[i]),
               (e1, N1[-1]), inflow)
        # converged: the product leaves and what flows in leaves as A, B or C
        assert N1[-1] > 0 and abs(N1.sum() - inflow) <= 1e-6 * inflow
        assert abs(eps[i] / r["eps"] - 1) <= 1e-9
        assert np.abs(N1 - np.asarray(r["N"])).max() <= 1e-10 * inflow
        c.close()


def test_batch_resume_equals_one_run():
    # the convergence run of the four cascades split into resumed calls of
    # 3000 steps (a multiple of the check interval) stops every instance at
    # the same step with the same state as one call
    import json
    import os
    import paper_2109_04455_amd as L
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batch_conv.json")))
    kw = dict(ref["instances"])
    for k in ("nx_range", "pe_range", "da_range"):
        kw[k] = tuple(kw[k])
    ws = batch_instances(**kw)
    out = []
    for split in (False, True):
        b = L.Batch([_params(w, "f64") for w in ws])
        b.set_geometry([w.node_type for w in ws], [w.k for w in ws])
        b.flow(ref["flow_steps"], check_every=ref["flow_steps"], tol=0)
        if split:
            with pytest.raises(L.LbfError):
                b.resume(1000, check_every=1000, tol=ref["tol"])  # no run started
            done = 4000
            res = b.run(done, check_every=1000, tol=ref["tol"])
            while not b.all_converged and done < ref["budget"]:
                res = b.resume(3000, check_every=1000, tol=ref["tol"])
                done += 3000
        else:
            res = b.run(ref["budget"], check_every=1000, tol=ref["tol"])
        assert b.all_converged
        out.append((res, [b.concentration(i, s) for i in range(len(ws)) for s in range(3)]))
        b.close()
    (r1, f1), (r2, f2) = out
    assert r1[2].tolist() == r2[2].tolist() == [r["adr_steps"] for r in ref["runs"]]
    assert (r1[0] == r2[0]).all() and (r1[1] == r2[1]).all()
    assert all(torch.equal(a, b) for a, b in zip(f1, f2))


def test_sweep_instances_full_size_short():
    # the 64-instance sweep at full size, a few steps: batch == single path
    import paper_2109_04455_amd as L
    ws = batch_instances()
    b = L.Batch([_params(w) for w in ws])
    b.set_geometry([w.node_type for w in ws], [w.k for w in ws])
    b.flow(50, check_every=50, tol=0)
    eps, prod, steps = b.run(40, check_every=40, tol=0)
    for i in (0, 17, 63):
        c = _single(ws[i], 50, 40)
        assert torch.equal(b.concentration(i, 0), c.concentration(0))
        assert prod[i] == c.efficiency()[1][-1]
