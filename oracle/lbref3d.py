"""ctypes wrapper of the FP64 3D C oracle ``lbref3d.c`` (test infrastructure only).

Arrays follow the C layout: fields ``[nz, ny, nx]``, flow populations
``[19, nz, ny, nx]``, species populations ``[ns, 7, nz, ny, nx]``; the state
between steps is the pre-collision population set.

Paper passages followed (Sitaru & Gekle, arXiv 2109.04455): flow LB with a
uniform body force in a box periodic in every direction (Sec.
"Lattice-Boltzmann for the Navier-Stokes equation", Eq. LBE); ADR LB (Eqs.
LBE_ADE, BGK, the equilibrium, Diffusion_LBM, source_lbm) on D3Q7; inlet and
outlet (Eq. BC) with the other boundaries periodic (Sec. "Boundary conditions
and flux computation in ADE"); efficiency Eq. A-B.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbref3d.c")
_LIB = os.environ.get("LBREF3D_LIB") or os.path.join(_HERE, "liblbref3d.so")

PERIODIC_X = 1
LINK = 0
NODE = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the 3D oracle with gcc (plain -O2, no OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
             "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if "LBREF3D_LIB" not in os.environ and (
                not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        _lib = ctypes.CDLL(_LIB)
        d, i, l, p = ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_void_p
        _lib.ref3_flow_init.argtypes = [i, i, i, p, p]
        _lib.ref3_flow_run.argtypes = [i, i, i, p, d, d, d, d, p, l]
        _lib.ref3_flow_velocity.argtypes = [i, i, i, p, p, d, d, d, p, p, p, p]
        _lib.ref3_adr_init.argtypes = [i, i, i, i, p, p, p, p, d, d, p]
        _lib.ref3_adr_run.argtypes = [i, i, i, i, p, p, p, p, p, p, d, d, d, i, i, p, l]
        _lib.ref3_adr_observe.argtypes = [i, i, i, i, p, p, d, i, p, p]
        _lib.ref3_adr_concentration.argtypes = [i, i, i, i, p, p, p]
        _lib.ref3_adr_totals.argtypes = [i, i, i, i, p, p, p]
    return _lib


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _dims(t):
    nz, ny, nx = t.shape
    return nx, ny, nz


# --------------------------------------------------------------------------- flow
def flow_init(node_type):
    t = _u8(node_type)
    nx, ny, nz = _dims(t)
    f = np.zeros((19, nz, ny, nx))
    lib().ref3_flow_init(nx, ny, nz, _ptr(t), _ptr(f))
    return f


def flow_run(node_type, f, tau, force, nsteps):
    t = _u8(node_type)
    nx, ny, nz = _dims(t)
    assert f.flags.c_contiguous and f.dtype == np.float64 and f.shape == (19, nz, ny, nx)
    lib().ref3_flow_run(nx, ny, nz, _ptr(t), tau, *map(float, force), _ptr(f), int(nsteps))
    return f


def flow_velocity(node_type, f, force):
    t = _u8(node_type)
    nx, ny, nz = _dims(t)
    u = np.zeros((3, nz, ny, nx))
    rho = np.zeros((nz, ny, nx))
    lib().ref3_flow_velocity(nx, ny, nz, _ptr(t), _ptr(f), *map(float, force), _ptr(u[0]),
                             _ptr(u[1]), _ptr(u[2]), _ptr(rho))
    return u, rho


def flow(node_type, tau, force, nsteps):
    """Rest-fluid start, nsteps forced steps; returns (u[3,nz,ny,nx], rho)."""
    f = flow_init(node_type)
    flow_run(node_type, f, tau, force, nsteps)
    return flow_velocity(node_type, f, force)


# ---------------------------------------------------------------------------- ADR
def adr_init(node_type, u, nspecies, c_in=1.0, vel_scale=1.0):
    t = _u8(node_type)
    nx, ny, nz = _dims(t)
    u = _f64(u)
    g = np.zeros((nspecies, 7, nz, ny, nx))
    lib().ref3_adr_init(nx, ny, nz, nspecies, _ptr(t), _ptr(u[0]), _ptr(u[1]), _ptr(u[2]),
                        vel_scale, c_in, _ptr(g))
    return g


def adr_run(node_type, k, u, g, tau, nsteps, c_in=1.0, vel_scale=1.0, mode=LINK, bc=0, k2=None):
    t = _u8(node_type)
    nx, ny, nz = _dims(t)
    ns = g.shape[0]
    assert g.flags.c_contiguous and g.dtype == np.float64 and g.shape == (ns, 7, nz, ny, nx)
    k = _f64(k)
    u = _f64(u)
    k2 = None if k2 is None else _f64(k2)
    lib().ref3_adr_run(nx, ny, nz, ns, _ptr(t), _ptr(k), _ptr(k2), _ptr(u[0]), _ptr(u[1]),
                       _ptr(u[2]), vel_scale, tau, c_in, mode, bc, _ptr(g), int(nsteps))
    return g


def adr_observe(node_type, g, c_in=1.0, xf=None):
    """(N[ns], inflow_A) of the last streaming; xf defaults to nx-3."""
    t = _u8(node_type)
    nx, ny, nz = _dims(t)
    ns = g.shape[0]
    xf = nx - 3 if xf is None else xf
    flux = np.zeros(ns)
    inflow = np.zeros(1)
    lib().ref3_adr_observe(nx, ny, nz, ns, _ptr(t), _ptr(g), c_in, xf, _ptr(flux), _ptr(inflow))
    return flux, float(inflow[0])


def adr_concentration(node_type, g):
    t = _u8(node_type)
    nx, ny, nz = _dims(t)
    ns = g.shape[0]
    c = np.zeros((ns, nz, ny, nx))
    lib().ref3_adr_concentration(nx, ny, nz, ns, _ptr(t), _ptr(g), _ptr(c))
    return c


def adr_totals(node_type, g):
    t = _u8(node_type)
    nx, ny, nz = _dims(t)
    ns = g.shape[0]
    tot = np.zeros(ns)
    lib().ref3_adr_totals(nx, ny, nz, ns, _ptr(t), _ptr(g), _ptr(tot))
    return tot


def efficiency(flux):
    flux = np.asarray(flux, dtype=np.float64)
    den = flux.sum()
    return float(flux[-1] / den) if den != 0 else float("nan")
