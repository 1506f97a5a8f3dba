"""ctypes wrapper of the random-walk particle tracker ``rwpt.c`` (test
infrastructure only; paper Sec. "Random walk")."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rwpt.c")
_LIB = os.path.join(_HERE, "librwpt.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", _SRC, "-o", tmp,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
        d, i, l, p = ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_void_p
        _lib.rwpt_run.restype = i
        _lib.rwpt_run.argtypes = [i, i, i, p, p, p, d, d, p, d, d, d, d, i, l, l,
                                  ctypes.c_uint64, l, i, p]
        _lib.rwpt_walk.restype = i
        _lib.rwpt_walk.argtypes = [i, i, i, p, p, p, d, d, p, d, d, d, i, ctypes.c_uint64, l,
                                   p, p, p, p, l, l]
    return _lib


def run(node_type, ux, uy, k, nspecies, D, *, vel_scale=1.0, rate_w=1.0 / 6.0,
        density=10.0, dt=0.5, zone=1.0, xf=None, burn_steps=10000, meas_steps=20000,
        seed=1, max_particles=5_000_000, wall_mode=1):
    """Net crossing rates N_s of the plane xf + 1/2 (particles per unit time).

    With ``zone = 1`` and ``rate_w = 1/6`` a particle in the cell of a fluid node
    reacts with probability k(sigma)/6 * dt per catalytic neighbour sigma per
    step -- the lattice link reaction k w_i C read as a first-order sink in the
    cell adjacent to the catalytic face.  ``wall_mode = 1`` makes the
    interpolated velocity vanish on the half-way walls of the lattice;
    ``wall_mode = 0`` interpolates with zero velocity at solid nodes."""
    t = np.ascontiguousarray(node_type, dtype=np.uint8)
    ny, nx = t.shape
    xf = nx - 3 if xf is None else xf
    ux = np.ascontiguousarray(ux, dtype=np.float64)
    uy = np.ascontiguousarray(uy, dtype=np.float64)
    k = np.ascontiguousarray(k, dtype=np.float64)
    out = np.zeros(nspecies + 1)
    rc = lib().rwpt_run(nx, ny, nspecies, t.ctypes.data, ux.ctypes.data, uy.ctypes.data,
                        vel_scale, D, k.ctypes.data, rate_w, density, dt, zone, xf,
                        int(burn_steps), int(meas_steps), int(seed), int(max_particles),
                        int(wall_mode), out.ctypes.data)
    if rc != 0:
        raise RuntimeError("rwpt_run failed")
    return out[:nspecies]


def efficiency_batches(node_type, ux, uy, k, nspecies, D, batches=8, seed=1, **kw):
    """eps from independent runs (different seeds); returns (mean, standard
    error of the mean, per-run values)."""
    eps = []
    for b in range(batches):
        n = run(node_type, ux, uy, k, nspecies, D, seed=seed + 7919 * b, **kw)
        eps.append(n[-1] / n.sum())
    eps = np.array(eps)
    return eps.mean(), eps.std(ddof=1) / np.sqrt(len(eps)), eps


def walk(node_type, ux, uy, k, nspecies, D, ids, x, y, species, t0, steps, *, vel_scale=1.0,
         rate_w=1.0 / 6.0, dt=0.5, zone=1.0, wall_mode=1, seed=1):
    """Trajectory mode: advance the given particles (ids uint64, positions,
    species) by steps t0 .. t0+steps-1, no insertion or removal.  Returns new
    (x, y, species) arrays."""
    t = np.ascontiguousarray(node_type, dtype=np.uint8)
    ny, nx = t.shape
    ux = np.ascontiguousarray(ux, dtype=np.float64)
    uy = np.ascontiguousarray(uy, dtype=np.float64)
    k = np.ascontiguousarray(k, dtype=np.float64)
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    x = np.array(x, dtype=np.float64)
    y = np.array(y, dtype=np.float64)
    sp = np.array(species, dtype=np.uint8)
    lib().rwpt_walk(nx, ny, nspecies, t.ctypes.data, ux.ctypes.data, uy.ctypes.data, vel_scale,
                    D, k.ctypes.data, rate_w, dt, zone, int(wall_mode), int(seed), len(ids),
                    ids.ctypes.data, x.ctypes.data, y.ctypes.data, sp.ctypes.data, int(t0),
                    int(steps))
    return x, y, sp
