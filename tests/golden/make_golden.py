"""Write the oracle's end-to-end results that are too slow to recompute inside
a GPU test.  Calls only the oracle (and the shared input generator).

    python tests/golden/make_golden.py

c0_oracle.json -- workload C0 (200x100, one type-1 disc R = 10 at (60, 50),
A->B, Pe = 10, Da = 1): 10,000 D2Q9 flow steps, then ADR steps in blocks of
1000 until the relative change of eps over a block is <= 1e-8.
"""
import json
import os
import sys

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


if __name__ == "__main__":
    out = c0()
    with open(os.path.join(HERE, "c0_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)
