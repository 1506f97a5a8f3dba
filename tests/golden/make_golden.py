"""Write the oracle's end-to-end results that are too slow to recompute inside
a GPU test.  Calls only the oracle (and the shared input generator).

    python tests/golden/make_golden.py

c0_oracle.json -- workload C0 (200x100, one type-1 disc R = 10 at (60, 50),
A->B, Pe = 10, Da = 1): 10,000 D2Q9 flow steps, then ADR steps in blocks of
1000 until a check is steady (eps changes by <= 1e-8 of itself over a block,
the product leaves and the outlet fluxes balance the inflow).

c0_short_checks.json -- the same run with a check every 20 steps: the
convergence test must not stop while the product front is still upstream of
the flux plane (eps = 0 at consecutive checks).

c2q_pe<Pe>.json -- the side-by-side membrane at a quarter of its linear size
(1024x256, 12 fibres R = 6), Da = 5, Pe in {1, 10, 100, 1000}: 500 flow steps,
then 3000 ADR steps from the initial state.  Stored: eps, the outlet fluxes,
the inflow, the total of each species over the fluid nodes, the maximum of
each concentration field and the concentrations at 512 seeded fluid nodes
plus each field's arg-max (the GPU test compares its fields there).

batch_conv.json -- four small two-membrane cascades of the batched sweep's
generator (seed 11, 32 rows, 120 ... 200 columns, two fibres R = 5 per band,
Pe in [2, 10], Da in [1, 10]): 3000 flow steps, then ADR steps until a check
(every 1000 steps) is steady at tol 1e-7, at most 40,000.  Stored per
instance: the stop step, eps, the outlet fluxes and the inflow.

    python tests/golden/make_golden.py [c0] [c2q] [batch]
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import lbref as R  # noqa: E402
from workloads import make_workload  # noqa: E402


def c0():
    w = make_workload("C0")
    ux, uy, fsteps, fres = R.flow_steady(w.node_type, w.tau_f, w.u0, 10000, tol=0)
    g, steps, flux, inflow, eps = R.adr_steady(w.node_type, w.k, ux, uy, 2, w.tau_g, 400000,
                                               check_every=1000, tol=1e-8)
    return {"workload": "C0", "flow_steps": fsteps, "adr_steps": steps, "tol": 1e-8,
            "check_every": 1000, "eps": eps, "N": list(map(float, flux)), "inflow": inflow,
            "tau_g": w.tau_g, "k": w.params.k}


def c0_short_checks():
    w = make_workload("C0")
    ux, uy, fsteps, fres = R.flow_steady(w.node_type, w.tau_f, w.u0, 10000, tol=0)
    g, steps, flux, inflow, eps = R.adr_steady(w.node_type, w.k, ux, uy, 2, w.tau_g, 400000,
                                               check_every=20, tol=1e-8)
    return {"workload": "C0", "flow_steps": fsteps, "adr_steps": steps, "tol": 1e-8,
            "check_every": 20, "eps": eps, "N": list(map(float, flux)), "inflow": inflow}


C2Q_PE = (1.0, 10.0, 100.0, 1000.0)
C2Q_FLOW, C2Q_ADR, C2Q_SAMPLES = 500, 3000, 512


def c2q_sample_nodes(node_type, seed=7, n=C2Q_SAMPLES):
    """Seeded fluid nodes (y, x) at which the concentration fields are kept."""
    fy, fx = np.nonzero(node_type == 0)
    pick = np.random.default_rng(seed).choice(fy.size, size=n, replace=False)
    return np.stack([fy[pick], fx[pick]], axis=1)


def c2q(pe):
    w = make_workload("C2q", pe=pe)
    ux, uy, _, _ = R.flow_steady(w.node_type, w.tau_f, w.u0, C2Q_FLOW, tol=0)
    g = R.adr_init(w.node_type, ux, uy, w.nspecies, w.c_in, w.vel_scale)
    R.adr_run(w.node_type, w.k, ux, uy, g, w.tau_g, C2Q_ADR, w.c_in, w.vel_scale)
    flux, inflow = R.adr_observe(w.node_type, g, w.c_in)
    c = R.adr_concentration(w.node_type, g)
    nodes = c2q_sample_nodes(w.node_type)
    arg = [list(map(int, np.unravel_index(np.argmax(np.abs(c[s])), c[s].shape)))
           for s in range(w.nspecies)]
    return {"workload": "C2q", "pe": pe, "da": w.params.da, "tau_g": w.tau_g,
            "vel_scale": w.vel_scale, "flow_steps": C2Q_FLOW, "adr_steps": C2Q_ADR,
            "eps": R.efficiency(flux), "N": list(map(float, flux)), "inflow": inflow,
            "totals": list(map(float, R.adr_totals(w.node_type, g))),
            "finite": bool(np.isfinite(g).all()),
            "cmax": [float(np.abs(c[s]).max()) for s in range(w.nspecies)],
            "argmax": arg, "nodes": nodes.tolist(),
            "c_nodes": [[float(v) for v in c[s][nodes[:, 0], nodes[:, 1]]]
                        for s in range(w.nspecies)],
            "c_argmax": [[float(c[s][a[0], a[1]]) for a in arg] for s in range(w.nspecies)]}


BATCH_CONV = {"n": 4, "seed": 11, "ny": 32, "nx_range": [120, 200], "fibres": 2, "r": 5,
              "pe_range": [2.0, 10.0], "da_range": [1.0, 10.0]}
BATCH_FLOW, BATCH_TOL, BATCH_BUDGET = 3000, 1e-7, 40000


def batch_conv_one(i):
    from workloads import batch_instances
    kw = dict(BATCH_CONV)
    kw["nx_range"], kw["pe_range"], kw["da_range"] = (tuple(kw["nx_range"]), tuple(kw["pe_range"]),
                                                      tuple(kw["da_range"]))
    w = batch_instances(**kw)[i]
    ux, uy, _, _ = R.flow_steady(w.node_type, w.tau_f, w.u0, BATCH_FLOW, tol=0)
    g, steps, flux, inflow, eps = R.adr_steady(w.node_type, w.k, ux, uy, w.nspecies, w.tau_g,
                                               BATCH_BUDGET, 1000, BATCH_TOL, w.c_in, w.vel_scale)
    return {"nx": w.nx, "pe": w.params.pe, "da": w.params.da, "tau_g": w.tau_g,
            "adr_steps": steps, "eps": eps, "N": list(map(float, flux)), "inflow": inflow}


def batch_conv():
    with ProcessPoolExecutor(BATCH_CONV["n"]) as ex:
        runs = list(ex.map(batch_conv_one, range(BATCH_CONV["n"])))
    return {"instances": BATCH_CONV, "flow_steps": BATCH_FLOW, "tol": BATCH_TOL,
            "check_every": 1000, "budget": BATCH_BUDGET, "runs": runs}


def _write(name, out):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=0)
    print(name, {k: v for k, v in out.items() if k not in ("nodes", "c_nodes")}, flush=True)


if __name__ == "__main__":
    which = set(sys.argv[1:]) or {"c0", "c2q", "batch"}
    if "batch" in which:
        _write("batch_conv.json", batch_conv())
    if "c2q" in which:
        with ProcessPoolExecutor(len(C2Q_PE)) as ex:
            for pe, out in zip(C2Q_PE, ex.map(c2q, C2Q_PE)):
                _write(f"c2q_pe{int(pe)}.json", out)
    if "c0" in which:
        for name, fn in (("c0_oracle.json", c0), ("c0_short_checks.json", c0_short_checks)):
            _write(name, fn())
