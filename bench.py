"""Benchmark: forward LB-ADR throughput (MLUPS) and HBM roofline fraction on
one MI355X, with the FP64 oracle timed on the host beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload C2|C1]

Workload (default C2): the side-by-side membrane lattice, 4096 x 1024 nodes,
200 fibres of radius 6 with both catalysts on each fibre, Pe = 100, Da = 5,
three species (A -> B -> C), FP32 populations with FP64 reductions.  Set-up
(untimed): geometry, the D2Q9 flow solved to its tolerance (capped), ADR
initial state, W warm-up steps.  A "step" is one lattice-Boltzmann time step
of the ADR over the whole lattice (all species: stream, boundary rules,
collide, link reactions); the timed region runs K steps in blocks of 1000
captured steps, each block followed by the outlet-flux / efficiency
evaluation that the convergence loop performs.  MLUPS counts every lattice
node (solid included) once per step.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "fwd/adjoint LB-ADR MLUPS & %HBM roofline; batched Pe-Da sweep vs serial"


def adr_bytes_per_step(node_type, nspecies, real_bytes):
    """Algorithmic HBM bytes of one ADR step: each fluid node reads and writes
    its 5*S populations once and reads its 2 velocity components and its 1-byte
    mask; a solid node reads only its mask."""
    fluid = int((node_type == 0).sum())
    solid = node_type.size - fluid
    per_fluid = 2 * 5 * nspecies * real_bytes + 2 * real_bytes + 1
    return fluid * per_fluid + solid * 1, per_fluid


def flow_bytes_per_step(node_type, real_bytes):
    fluid = int((node_type == 0).sum())
    return fluid * (2 * 9 * real_bytes + 2) + (node_type.size - fluid) * 2


ADR_KERNEL_SOURCES = ("kernels_adr.hip", "adr_device.hpp", "stencil.hpp", "lbf_internal.hpp")


def kernel_source_hash():
    """Hash of every source the ADR step kernel is compiled from."""
    h = hashlib.sha256()
    for name in ADR_KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2109_04455_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload):
    """HBM bytes per launch of the ADR kernel from the committed counter
    summary, or None when it is missing or was taken on other kernel source."""
    path = os.path.join(ROOT, "profiles", f"adr_step_{workload}_counters.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(w, steps=20, flow_steps=5):
    """The oracle as it stands, single-threaded FP64, on the same lattice."""
    from oracle import lbref as R
    t = w.node_type
    ux, uy, _, _ = R.flow_steady(t, w.tau_f, w.u0, flow_steps, tol=0)
    g = R.adr_init(t, ux, uy, w.nspecies, w.c_in, w.vel_scale)
    t0 = time.perf_counter()
    R.adr_run(t, w.k, ux, uy, g, w.tau_g, steps, w.c_in, w.vel_scale)
    dt = time.perf_counter() - t0
    return {"value": w.nx * w.ny * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{w.name} lattice {w.nx}x{w.ny}, {w.nspecies} species, {steps} ADR steps "
                      f"of the FP64 single-threaded oracle ({dt:.1f} s) after {flow_steps} flow steps"}


def adjoint_leg(T=20000, M=200):
    """Adjoint wall time / forward wall time on the C1 geometry (FP32 state,
    FP64 reductions and gradient), both the checkpoint-recompute path and the
    path that keeps the whole trace."""
    import torch
    import paper_2109_04455_amd as L
    from workloads import make_workload
    w = make_workload("C1")
    p = L.params(w.nx, w.ny, real="f32", nspecies=3, tau_f=w.tau_f, u0=w.u0, tau_g=w.tau_g,
                 c_in=w.c_in, vel_scale=w.vel_scale)
    c = L.Context(p)
    c.set_geometry(w.node_type)
    c.set_rates(w.k)
    c.flow_init()
    c.flow_run(20000)
    c.adr_init()
    c.adr_run(20000, tol=0)
    start = c.get_state()
    out = {"workload": "C1 geometry (2048x512, 40 fibres), T=%d, checkpoints every %d" % (T, M)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.adr_run(T, tol=0)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    out["forward_s"] = round(fwd, 4)
    # C1's two lattices (126 MB) fit the 256 MB last-level cache
    out["forward_mlups"] = round(w.nx * w.ny * T / fwd / 1e6, 1)
    out["forward_cache_assisted"] = True
    for keep in (False, True):
        c.set_state(start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eps, grad = c.adjoint(T, M, keep_trace=keep)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tag = "keep_trace" if keep else "recompute"
        out[f"{tag}_s"] = round(dt, 4)
        out[f"{tag}_ratio"] = round(dt / fwd, 3)
        out["eps"] = eps
        out["grad_max_abs"] = float(grad.abs().max())
    keep = c.adjoint_path(T, M)
    out["default_path"] = "keep_trace" if keep else "recompute"
    out["ratio"] = out["keep_trace_ratio" if keep else "recompute_ratio"]
    c.close()
    return out


def c0_leg(max_steps=2_000_000):
    """C0 (200x100, one disc, FP64, A -> B): time to solution.  The lattice is
    far too small to fill the GPU (launch-bound), so only the wall time of the
    whole job is reported: 10,000 flow steps, then ADR until eps changes by
    less than 1e-8 of itself per 1000 steps."""
    import torch
    import paper_2109_04455_amd as L
    from workloads import make_workload
    w = make_workload("C0")
    p = L.params(w.nx, w.ny, real=w.real, nspecies=w.nspecies, tau_f=w.tau_f, u0=w.u0,
                 tau_g=w.tau_g, c_in=w.c_in, vel_scale=w.vel_scale)
    c = L.Context(p)
    c.set_geometry(w.node_type)
    c.set_rates(w.k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.flow_init()
    c.flow_run(10000)
    c.adr_init()
    n, conv = c.adr_run(max_steps, check_every=1000, tol=1e-8)
    eps, N, inflow = c.efficiency()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    c.close()
    return {"workload": f"C0: {w.nx}x{w.ny}, one disc, FP64, {w.nspecies} species",
            "flow_steps": 10000, "adr_steps": int(n), "converged": bool(conv), "eps": eps,
            "mass_balance": float(abs(N.sum() - inflow) / inflow),
            "seconds_to_solution": round(dt, 3)}


def precision_leg(steps=20000, flow_steps=5000):
    """FP32 path against the FP64 path of the same library on the C1 geometry
    at a quarter of its linear size, identical step counts: relative error of
    eps and of the concentration fields (max |dC| / max |C| per species)."""
    import paper_2109_04455_amd as L
    from workloads import make_workload
    w = make_workload("C1q")
    res = {}
    for real in ("f32", "f64"):
        p = L.params(w.nx, w.ny, real=real, nspecies=3, tau_f=w.tau_f, u0=w.u0, tau_g=w.tau_g,
                     c_in=w.c_in, vel_scale=w.vel_scale)
        c = L.Context(p)
        c.set_geometry(w.node_type)
        c.set_rates(w.k)
        c.flow_init()
        c.flow_run(flow_steps)
        c.adr_init()
        c.adr_run(steps, tol=0)
        eps, N, inflow = c.efficiency()
        res[real] = (eps, [c.concentration(s).double().cpu() for s in range(3)])
        c.close()
    e32, c32 = res["f32"]
    e64, c64 = res["f64"]
    field = max(float((a - b).abs().max() / b.abs().max()) for a, b in zip(c32, c64))
    return {"workload": "C1 quarter scale (512x128), %d flow + %d ADR steps" % (flow_steps, steps),
            "eps_f32": e32, "eps_f64": e64, "eps_rel_err": abs(e32 / e64 - 1),
            "field_rel_err": field}


_ORACLE_INSTANCE = """
import json, sys, time
sys.path.insert(0, sys.argv[1])
from oracle import lbref as R
from workloads import batch_instances
i, steps, flow_steps = int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4])
w = batch_instances()[i]
ux, uy, _, _ = R.flow_steady(w.node_type, w.tau_f, w.u0, flow_steps, tol=0)
g = R.adr_init(w.node_type, ux, uy, w.nspecies, w.c_in, w.vel_scale)
t0 = time.perf_counter()
R.adr_run(w.node_type, w.k, ux, uy, g, w.tau_g, steps, w.c_in, w.vel_scale)
print(json.dumps([w.node_type.size * steps, time.perf_counter() - t0]))
"""


def cpu_sweep_baseline(nproc=8, steps=20, flow_steps=5, timeout=300):
    """The oracle on the first nproc sweep instances at once, one
    single-threaded process per instance and core (child interpreters that
    never touch the GPU): aggregate MLUPS = all node-steps over the longest
    process's ADR time.  None if a child fails."""
    import subprocess
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    nproc = max(1, min(nproc, ncpu, 16))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, "-c", _ORACLE_INSTANCE, ROOT, str(i), str(steps),
                               str(flow_steps)], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL,
                              env=env) for i in range(nproc)]
    res = []
    try:
        for p in procs:
            out, _ = p.communicate(timeout=timeout)
            if p.returncode != 0:
                return None
            res.append(json.loads(out.decode().strip().splitlines()[-1]))
    except (subprocess.TimeoutExpired, ValueError, IndexError):
        return None
    finally:
        for p in procs:
            if p.poll() is None:
                p.kill()
                p.wait()
    work = sum(r[0] for r in res)
    longest = max(r[1] for r in res)
    return {"value": round(work / longest / 1e6, 2), "unit": "MLUPS", "processes": nproc,
            "kind": "oracle",
            "sample": f"first {nproc} sweep instances, {steps} ADR steps each after {flow_steps} "
                      f"flow steps, one single-threaded FP64 oracle process per instance, run at "
                      f"once ({longest:.1f} s)"}


def batch_leg(steps=2000, flow_steps=2000, cpu=True, tts_steps=0, tts_tol=1e-6):
    """The 64-instance Pe x Da sweep for a fixed number of steps: one batched
    launch per step (tile shape and launch mode chosen by the autotuner) vs
    the same instances run one after another through the single-lattice path
    (each with its own captured graphs)."""
    from paper_2109_04455_amd.autotune import autotune_batch
    from paper_2109_04455_amd.sweep import sweep_batched, sweep_serial
    from workloads import batch_instances
    ws = batch_instances()
    nodes = sum(w.nx * w.ny for w in ws)
    best, timings = autotune_batch(ws)
    tile, flags = (best[0], best[1]), best[2]
    b = sweep_batched(ws, flow_steps, steps, check_every=1000, tile=tile, flags=flags)
    s = sweep_serial(ws, flow_steps, steps, check_every=1000)
    same = bool((b["product_flux"] == s["product_flux"]).all())
    tts = None
    if tts_steps > 0:
        # time to solution: every instance runs until eps changes by less than
        # tts_tol of itself over 1000 steps, or tts_steps (converged instances
        # leave the batched launch; the serial path stops each on its own)
        bt = sweep_batched(ws, flow_steps, tts_steps, check_every=1000, tol=tts_tol, tile=tile,
                           flags=flags)
        st = sweep_serial(ws, flow_steps, tts_steps, check_every=1000, tol=tts_tol)
        tts = {"max_steps": tts_steps, "tol": tts_tol,
               "batched_s": round(bt["seconds"], 2), "serial_s": round(st["seconds"], 2),
               "speedup": round(st["seconds"] / bt["seconds"], 3),
               "converged": int((bt["steps"] < tts_steps).sum()),
               "same_steps": bool((bt["steps"] == st["steps"]).all())}
    return {"instances": len(ws), "nodes": nodes, "steps": steps,
            "autotuned": {"tile": list(tile), "mode": ("one block per tile" if flags & 8 else
                                                    "persistent tile walk") +
                          ("" if flags & 256 else ", two ADR steps per launch"),
                          "us_per_step": {str(k): round(v, 2) for k, v in timings.items()}},
            "batched_adr_s": round(b["adr_seconds"], 4), "serial_adr_s": round(s["adr_seconds"], 4),
            "batched_mlups": round(nodes * steps / b["adr_seconds"] / 1e6, 1),
            "serial_mlups": round(nodes * steps / s["adr_seconds"] / 1e6, 1),
            "speedup": round(s["adr_seconds"] / b["adr_seconds"], 3),
            "batched_total_s": round(b["seconds"], 3), "serial_total_s": round(s["seconds"], 3),
            "batched_flow_s": round(b["flow_seconds"], 3), "serial_flow_s": round(s["flow_seconds"], 3),
            "batched_setup_s": round(b["setup_seconds"], 3),
            "serial_setup_s": round(s["setup_seconds"], 3),
            "identical_results": same,
            "cpu_oracle": cpu_sweep_baseline() if cpu else None,
            "time_to_solution": tts}

def membrane3d_leg(steps=2000):
    """3D randomly oriented fibre membranes (D3Q19 forced flow, D3Q7 ADR, FP32
    storage).  Throughput and HBM roofline of both step kernels on the paper's
    cascade membrane doubled in every direction (400x120x120, 1.05 GB of ADR
    lattices); time to the steady efficiency on the paper's own 200x60x60 box."""
    import torch
    import paper_2109_04455_amd as L
    from workloads.configs3d import make_workload3d
    out = {}
    w = make_workload3d("M3c2")
    n = w.nx * w.ny * w.nz
    fluid = int((w.node_type == 0).sum())
    p = L.params3d(w.nx, w.ny, w.nz, real="f32", nspecies=3, tau_f=w.tau_f, force_x=w.force,
                   tau_g=w.tau_g)
    c = L.Context3D(p)
    c.set_geometry(w.node_type)
    c.set_rates(w.k)
    c.flow_init()
    c.flow_run(200)
    flow_ms = c.time_flow_steps(steps) / steps
    c.adr_init()
    c.adr_run(200, check_every=200, tol=0)
    adr_ms = c.time_adr_steps(steps) / steps
    adr_b = fluid * (2 * 21 * 4 + 3 * 4 + 2) + (n - fluid) * 2
    flow_b = fluid * (2 * 19 * 4 + 4) + (n - fluid) * 4
    out["M3c2"] = {
        "lattice": [w.nx, w.ny, w.nz], "fibres": 96, "steps": steps,
        "adr_us": round(adr_ms * 1e3, 2), "adr_mlups": round(n / adr_ms / 1e3, 1),
        "adr_gbs": round(adr_b / adr_ms / 1e6, 1), "adr_frac": round(adr_b / adr_ms / 1e6 / PEAK_HBM_GBS, 4),
        "adr_bytes_per_fluid_node": 182,
        "flow_us": round(flow_ms * 1e3, 2), "flow_mlups": round(n / flow_ms / 1e3, 1),
        "flow_gbs": round(flow_b / flow_ms / 1e6, 1),
        "flow_frac": round(flow_b / flow_ms / 1e6 / PEAK_HBM_GBS, 4), "flow_bytes_per_fluid_node": 156}
    c.close()
    w = make_workload3d("M3c")
    p = L.params3d(w.nx, w.ny, w.nz, real="f32", nspecies=3, tau_f=w.tau_f, force_x=w.force,
                   tau_g=w.tau_g)
    c = L.Context3D(p)
    c.set_geometry(w.node_type)
    c.set_rates(w.k)
    c.flow_init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fsteps, fres, fconv = c.flow_steady(200000, 1000, 1e-5)
    u = c.get_velocity()
    vs = w.vel_scale(u[0].double().cpu().numpy())
    c.close()
    # the ADR runs on the same flow, scaled to the entrance velocity of Pe
    p.vel_scale = vs
    c = L.Context3D(p)
    c.set_geometry(w.node_type)
    c.set_rates(w.k)
    c.set_velocity(u)
    c.adr_init()
    asteps, aconv = c.adr_run(400000, check_every=1000, tol=1e-6)
    eps, N, inflow = c.efficiency()
    torch.cuda.synchronize()
    out["M3c"] = {"lattice": [w.nx, w.ny, w.nz], "pe": w.params.pe, "da": w.params.da,
                  "flow_steps": fsteps, "flow_converged": fconv, "vel_scale": round(vs, 3),
                  "adr_steps": asteps, "adr_converged": aconv, "eps": eps,
                  "mass_balance": float(abs(N.sum() - inflow) / inflow),
                  "seconds_to_solution": round(time.perf_counter() - t0, 2)}
    c.close()
    return out


def rwpt_leg(w, ux, uy, steps=200, density=10.0):
    """The GPU random-walk tracker on the same geometry and flow as the
    headline ADR run: particle-steps per second and the bytes a step moves
    per particle (move: 25 B read + 17 B written; compaction, at the start of
    each 200-step graph block and every min(64, nx / 8) steps inside it: 8 B
    read to count, 25 B read + 25 B written to scatter)."""
    import torch
    import paper_2109_04455_amd as L
    p = L.rw_params(w.nx, w.ny, nspecies=w.nspecies, D=w.params.d, vel_scale=w.vel_scale,
                    density=density, seed=5)
    r = L.RandomWalk(p)
    r.set_fields(w.node_type, ux.double(), uy.double(), w.k)
    r.fill()
    r.run(50)
    ms = r.time_steps(steps, measure=True)
    n, held, _ = r.counts()
    r.close()
    per_step = ms * 1e-3 / steps
    every = min(64, max(1, w.nx // 8))
    bytes_pp = 42 + (8 + 50) * math.ceil(200 / every) / 200
    return {"workload": f"{w.name} geometry and flow, density {density} per unit area",
            "particles": held, "steps": steps, "us_per_step": round(per_step * 1e6, 1),
            "particle_steps_per_s": round(held / per_step, 1),
            "gbs": round(held * bytes_pp / per_step / 1e9, 1), "bytes_per_particle_step": bytes_pp,
            "N": [float(v) for v in n]}


def no_flow_leg(steps=(10000, 50000, 100000)):
    """The paper's pure-diffusion cascade (300x300 periodic box, Da 150, no
    flow): total C over time for two fibres 100 apart vs one side-by-side
    fibre of the same catalytic surface, and the production of C per step
    (B -> C conversion) at the same times."""
    import torch
    import paper_2109_04455_amd as L
    from workloads import box_workload
    res = {}
    for morph in ("pair", "side"):
        w = box_workload(morph, real="f32")
        p = L.params(w.nx, w.ny, real="f32", nspecies=3, tau_g=w.tau_g, c_in=w.c_in,
                     vel_scale=0.0, boundary=L.PERIODIC)
        c = L.Context(p)
        c.set_geometry(w.node_type)
        c.set_rates(w.k)
        z = torch.zeros((w.ny, w.nx), dtype=torch.float32)
        c.set_velocity(z, z)
        c.adr_init()
        done, series, prod = 0, [], []
        t0 = time.perf_counter()
        for s in steps:
            c.adr_run(s - done, check_every=s - done, tol=0)
            done = s
            tot = c.totals()
            series.append([s, float(tot[2] / tot.sum())])
            prod.append([s, float(c.production()[1] / tot.sum())])
        res[morph] = {"C_fraction": series, "C_production_per_step": prod,
                      "seconds": round(time.perf_counter() - t0, 3)}
        c.close()
    res["side_by_side_faster"] = all(b[1] > a[1] for a, b in zip(res["pair"]["C_fraction"],
                                                                  res["side"]["C_fraction"]))
    return res


def targets_leg(w, steps=2000):
    """Throughput against 70 % of the 8 TB/s HBM peak (5.6 TB/s of algorithmic
    bytes) for two more configurations of the same C2 lattice: the D2Q9 flow
    with FP32 arithmetic (flags bit 5; 74 B per fluid node-step) and the ADR
    with FP64 populations and two species (A -> B; 177 B per fluid node-step,
    two steps per launch).  The C2 geometry, 200 flow steps from the initial
    state, then timed steps."""
    import paper_2109_04455_amd as L
    out = {}
    nodes = w.nx * w.ny
    target = 0.7 * PEAK_HBM_GBS
    p = L.params(w.nx, w.ny, real="f32", nspecies=w.nspecies, tau_f=w.tau_f, u0=w.u0,
                 tau_g=w.tau_g, c_in=w.c_in, vel_scale=w.vel_scale, flags=32)
    c = L.Context(p)
    c.set_geometry(w.node_type)
    c.set_rates(w.k)
    c.flow_init()
    c.flow_run(200)
    ms = min(c.time_flow_steps(1000) for _ in range(3)) / 1000
    c.close()
    fb = flow_bytes_per_step(w.node_type, 4)
    out["flow_fp32_arithmetic"] = {
        "mlups": round(nodes / (ms * 1e-3) / 1e6, 1), "us_per_step": round(ms * 1e3, 2),
        "gbs": round(fb / (ms * 1e-3) / 1e9, 1), "frac": round(fb / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "target_mlups": round(target * 1e9 / (fb / nodes) / 1e6)}
    p = L.params(w.nx, w.ny, real="f64", nspecies=2, tau_f=w.tau_f, u0=w.u0, tau_g=w.tau_g,
                 c_in=w.c_in, vel_scale=w.vel_scale)
    c = L.Context(p)
    c.set_geometry(w.node_type)
    c.set_rates(w.k)
    c.flow_init()
    c.flow_run(200)
    c.adr_init()
    c.adr_run(1001, tol=0)
    ms = min(c.time_adr_steps(steps) for _ in range(2)) / steps
    c.close()
    ab, per_fluid = adr_bytes_per_step(w.node_type, 2, 8)
    out["adr_fp64_two_species"] = {
        "mlups": round(nodes / (ms * 1e-3) / 1e6, 1), "us_per_step": round(ms * 1e3, 2),
        "bytes_per_fluid_node_step": per_fluid,
        "gbs": round(ab / (ms * 1e-3) / 1e9, 1), "frac": round(ab / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
        "target_mlups": round(target * 1e9 / (ab / nodes) / 1e6)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--pe", type=float, default=None)
    ap.add_argument("--flow-max-steps", type=int, default=400000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe-copy-mib", type=int, default=1024)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=20000)
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--batch-tts-steps", type=int, default=0,
                    help="also time the sweep to convergence, capped at this many ADR steps")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-noflow", action="store_true")
    ap.add_argument("--no-rwpt", action="store_true")
    ap.add_argument("--no-c0", action="store_true")
    ap.add_argument("--no-targets", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the sweep would shard by instance and a large lattice by x-slabs).",
              file=sys.stderr)
        sys.exit(2)
    if args.steps % 1000:
        args.steps = (args.steps // 1000 + 1) * 1000

    import torch
    import paper_2109_04455_amd as L
    from workloads import make_workload

    w = make_workload(args.workload, pe=args.pe)
    real_bytes = {"f32": 4, "f64": 8}[w.real]
    p = L.params(w.nx, w.ny, real=w.real, nspecies=w.nspecies, tau_f=w.tau_f, u0=w.u0,
                 tau_g=w.tau_g, c_in=w.c_in, vel_scale=w.vel_scale)
    ctx = L.Context(p)
    ctx.set_geometry(w.node_type)
    ctx.set_rates(w.k)

    # ---- set-up: flow (a3), handoff + ADR initial state
    ctx.flow_init()
    t0 = time.perf_counter()
    flow_steps, flow_res, flow_conv = ctx.flow_steady(args.flow_max_steps, 1000, w.flow_tolerance)
    flow_s = time.perf_counter() - t0
    flow_ms = ctx.time_flow_steps(1000)
    flow_mlups = w.nx * w.ny * 1000 / (flow_ms * 1e-3) / 1e6
    ctx.adr_init()
    ctx.adr_run(args.warmup, check_every=1000, tol=0)
    # a block of 1000 steps is 499 two-step launches and 2 single steps (the
    # last step of a block is always a single one); the single-step launch is
    # timed on its own here, on the same stream
    single_ms = min(ctx.time_adr_steps(2) for _ in range(5)) / 2

    # ---- timed region: K ADR steps in blocks of 1000 + efficiency per block
    torch.cuda.synchronize()
    kernel_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps // 1000):
        kernel_ms += ctx.time_adr_steps(1000)
        eps, N, inflow = ctx.efficiency()
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0

    nodes = w.nx * w.ny
    mlups = nodes * args.steps / wall_s / 1e6
    step_bytes, per_fluid = adr_bytes_per_step(w.node_type, w.nspecies, real_bytes)
    blocks = args.steps // 1000
    pairs = (1000 - 1) // 2
    pair_ms = (kernel_ms / blocks - (1000 - 2 * pairs) * single_ms) / pairs
    # algorithmic bytes of a launch: 129 B per fluid node-step (the ADR
    # step's figure) times the two node-steps per node a launch performs;
    # the lattice itself crosses HBM once per launch (`traffic`, measured)
    launch_s = pair_ms * 1e-3
    launch_bytes = 2 * step_bytes
    achieved = launch_bytes / launch_s / 1e9
    traffic = traffic_from_profiles(args.workload)

    # practical ceiling: a plain device copy of the same library
    copy_ms = min(L.probe_copy(args.probe_copy_mib << 20) for _ in range(3))
    copy_gbs = 2 * (args.probe_copy_mib << 20) / (copy_ms * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "species_mlups": round(mlups * w.nspecies, 1),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_s * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if real_bytes == 4 else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: {w.nx}x{w.ny} side-by-side membrane" if w.name == "C2" else
                        f"{w.name}: {w.nx}x{w.ny}",
            "nx": w.nx, "ny": w.ny, "nspecies": w.nspecies, "pe": w.params.pe,
            "da": w.params.da, "tau_g": w.tau_g, "catalytic_nodes": w.n_catalytic(),
            "check_every": 1000, "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            "kernel": "k_adr_step2<float,double,3,true,false,false>", "steps_per_launch": 2,
            "bytes_per_launch": launch_bytes, "bytes_per_fluid_node_step": per_fluid,
            "avg_launch_us": round(launch_s * 1e6, 3),
            "us_per_step": round(kernel_ms * 1e3 / args.steps, 3),
            "measured_hbm_gbs": round(traffic / launch_s / 1e9, 1) if traffic else None,
            "measured_hbm_frac": round(traffic / launch_s / 1e9 / PEAK_HBM_GBS, 4) if traffic else None,
            "single_step_kernel": {
                "kernel": "k_adr_step<float,double,3,false,true,false>",
                "avg_launch_us": round(single_ms * 1e3, 3),
                "achieved": round(step_bytes / (single_ms * 1e-3) / 1e9, 1),
                "frac": round(step_bytes / (single_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            },
        },
        "eps": eps, "N": [float(v) for v in N], "inflow": inflow,
        "flow": {"steps": flow_steps, "residual": flow_res, "converged": flow_conv,
                 "seconds": round(flow_s, 2), "mlups": round(flow_mlups, 1),
                 "gbs": round(flow_bytes_per_step(w.node_type, real_bytes) / (flow_ms * 1e-3 / 1000) / 1e9, 1)},
        "copy_probe_gbs": round(copy_gbs, 1),
    }
    if not args.no_rwpt:
        ux, uy = ctx.get_velocity()
        out["rwpt"] = rwpt_leg(w, ux, uy)
    ctx.close()
    if not args.no_targets:
        out["throughput_targets"] = targets_leg(w)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(args.adjoint_steps)
    if not args.no_batch:
        out["batched_sweep"] = batch_leg(args.batch_steps, cpu=not args.no_cpu_baseline,
                                         tts_steps=args.batch_tts_steps)
    if not args.no_precision:
        out["fp32_vs_fp64"] = precision_leg()
    if not args.no_3d:
        out["membrane_3d"] = membrane3d_leg()
    if not args.no_noflow:
        out["no_flow_box"] = no_flow_leg()
    if not args.no_c0:
        out["c0_time_to_solution"] = c0_leg()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
