"""Pe x Da sweep drivers: all instances through one batched launch per step,
or one after another through the single-lattice path (the serial baseline)."""
from __future__ import annotations

import time

import numpy as np
import torch


def _params(w, **kw):
    import paper_2109_04455_amd as L
    return L.params(w.nx, w.ny, real=w.real, nspecies=w.nspecies, tau_f=w.tau_f, u0=w.u0,
                    tau_g=w.tau_g, c_in=w.c_in, vel_scale=w.vel_scale, **kw)


def sweep_batched(instances, flow_steps, adr_steps, check_every=1000, tol=0.0, flow_tol=0.0,
                  tile=(256, 1), flags=0, chunk=None, progress=None):
    """Returns dict(eps, product_flux, steps, seconds, setup_seconds,
    flow_seconds, adr_seconds).  chunk: run the ADR in calls of that many
    steps (a multiple of check_every; the run resumes, so the stop steps are
    those of one call), calling progress(steps_done, active) after each."""
    import paper_2109_04455_amd as L
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = L.Batch([_params(w, tile_x=tile[0], tile_y=tile[1], flags=flags) for w in instances])
    b.set_geometry([w.node_type for w in instances], [w.k for w in instances])
    torch.cuda.synchronize()
    tf = time.perf_counter()
    b.flow(flow_steps, check_every=check_every, tol=flow_tol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if chunk:
        done = min(chunk, adr_steps)
        eps, prod, steps = b.run(done, check_every=check_every, tol=tol)
        while done < adr_steps and not b.all_converged:
            if progress:
                progress(done, int((steps == done).sum()))
            n = min(chunk, adr_steps - done)
            eps, prod, steps = b.resume(n, check_every=check_every, tol=tol)
            done += n
    else:
        eps, prod, steps = b.run(adr_steps, check_every=check_every, tol=tol)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    b.close()
    return {"eps": eps, "product_flux": prod, "steps": steps, "seconds": t2 - t0,
            "setup_seconds": tf - t0, "flow_seconds": t1 - tf, "adr_seconds": t2 - t1}


def sweep_serial(instances, flow_steps, adr_steps, check_every=1000, tol=0.0, flow_tol=0.0,
                 tile=(256, 1), flags=0):
    """The same instances one after another, each with its own context and
    captured graphs."""
    import paper_2109_04455_amd as L
    eps, prod, steps = [], [], []
    adr_s = flow_s = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for w in instances:
        c = L.Context(_params(w, tile_x=tile[0], tile_y=tile[1], flags=flags))
        c.set_geometry(w.node_type)
        c.set_rates(w.k)
        torch.cuda.synchronize()
        tf = time.perf_counter()
        c.flow_init()
        c.flow_steady(flow_steps, check_every, flow_tol)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        flow_s += ta - tf
        c.adr_init()
        n, _ = c.adr_run(adr_steps, check_every=check_every, tol=tol)
        e, N, _ = c.efficiency()
        torch.cuda.synchronize()
        adr_s += time.perf_counter() - ta
        eps.append(e)
        prod.append(N[-1])
        steps.append(n)
        c.close()
    total = time.perf_counter() - t0
    return {"eps": np.array(eps), "product_flux": np.array(prod), "steps": np.array(steps),
            "seconds": total, "setup_seconds": total - flow_s - adr_s, "flow_seconds": flow_s,
            "adr_seconds": adr_s}
