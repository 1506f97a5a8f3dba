"""Small autotuner for the stencil launch: times candidate kernel variants,
thread-block shapes and cache policies of the ADR step on a representative
lattice and keeps the fastest, with a JSON cache keyed by (architecture,
species, precision, nx bucket, ny)."""
from __future__ import annotations

import json
import os

import torch

DEFAULT_CANDIDATES = (
    # (variant, tile_x, tile_y, flags).  flags 0: two steps per launch with
    # the intermediate state in LDS (its tile is fixed; variant and tile
    # shape then apply to the single steps that end each block); flags bit 8
    # (256): one step per launch; bit 1 (2): cached instead of streaming.
    (1, 256, 1, 0), (1, 256, 1, 2),
    (1, 256, 1, 256), (1, 512, 1, 256), (1, 1024, 1, 256),
    (1, 64, 1, 256), (1, 64, 2, 256), (1, 64, 4, 256), (1, 64, 8, 256),
    (1, 128, 1, 256), (1, 128, 2, 256), (1, 128, 4, 256), (1, 128, 8, 256),
    (1, 256, 2, 256), (1, 256, 4, 256),
    (2, 64, 4, 256), (2, 64, 1, 256), (2, 128, 2, 256),
    (1, 256, 1, 256 | 2),
)


def _key(arch, nspecies, real, nx, ny):
    bucket = 1 << max(6, (int(nx) - 1).bit_length())
    return f"{arch}|S{nspecies}|{real}|nx{bucket}|ny{ny}"


def _arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def autotune(node_type, k, *, real="f32", nspecies=3, tau_g=0.8, vel_scale=1.0, steps=300,
             candidates=DEFAULT_CANDIDATES, cache_path=None, verbose=False):
    """Return (variant, tile_x, tile_y, flags) of the fastest ADR step for this
    lattice shape.  ``cache_path`` (JSON) is read and updated when given."""
    import paper_2109_04455_amd as L

    ny, nx = node_type.shape
    key = _key(_arch(), nspecies, real, nx, ny)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return tuple(cache[key]["best"])
    results = []
    for cand in candidates:
        variant, tx, ty, flags = cand
        p = L.params(nx, ny, real=real, nspecies=nspecies, tau_g=tau_g, vel_scale=vel_scale,
                     variant=variant, tile_x=tx, tile_y=ty, flags=flags)
        try:
            c = L.Context(p)
        except L.LbfError:
            continue
        c.set_geometry(node_type)
        c.set_rates(k)
        c.flow_init()
        c.flow_run(20)
        c.adr_init()
        c.adr_run(20, tol=0)
        ms = min(c.time_adr_steps(steps) for _ in range(2))
        c.close()
        results.append((ms, cand))
        if verbose:
            print(f"autotune {key} {cand}: {ms / steps * 1e3:.2f} us/step", flush=True)
    best = min(results)[1]
    if cache_path:
        cache[key] = {"best": list(best),
                      "timings_us": {str(c): ms / steps * 1e3 for ms, c in results}}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best


BATCH_CANDIDATES = (
    # (tile_x, tile_y, flags): flags bit 8 = one ADR step per launch instead
    # of two; bit 3 = one block per tile instead of the persistent tile walk.
    # Two steps per launch use the LDS tile fixed at compile time, which tile
    # shape and bit 3 do not change (the tile shape reaches only the flow and
    # the single steps, bit 3 only the single steps): one candidate.  One step
    # per launch: tile shapes, walk or not.
    (256, 1, 0),
    (256, 1, 256), (256, 1, 256 | 8), (128, 2, 256), (128, 2, 256 | 8), (64, 4, 256),
    (64, 4, 256 | 8), (128, 1, 256 | 8), (64, 1, 256 | 8),
)


def autotune_batch(instances, *, steps=200, flow_steps=20, candidates=BATCH_CANDIDATES,
                   verbose=False):
    """Time the batched ADR step over the actual instance set for each
    candidate (tile shape, persistent tile walk or one block per tile) and
    return (best_candidate, {candidate: us_per_step})."""
    import paper_2109_04455_amd as L

    timings = {}
    for cand in candidates:
        tx, ty, flags = cand
        plist = [L.params(w.nx, w.ny, real=w.real, nspecies=w.nspecies, tau_f=w.tau_f, u0=w.u0,
                          tau_g=w.tau_g, c_in=w.c_in, vel_scale=w.vel_scale, tile_x=tx,
                          tile_y=ty, flags=flags) for w in instances]
        try:
            b = L.Batch(plist)
        except L.LbfError:
            continue
        b.set_geometry([w.node_type for w in instances], [w.k for w in instances])
        b.flow(flow_steps, check_every=flow_steps, tol=0)
        b.run(1, check_every=1, tol=0)
        ms = min(b.time_steps(steps) for _ in range(2))
        b.close()
        timings[cand] = ms / steps * 1e3
        if verbose:
            print(f"autotune batch {cand}: {timings[cand]:.2f} us/step", flush=True)
    best = min(timings, key=timings.get)
    return best, timings
