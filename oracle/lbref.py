"""ctypes wrapper of the FP64 C oracle ``lbref.c`` (test infrastructure only).

Arrays follow the C layout: fields ``[ny, nx]``, flow populations
``[9, ny, nx]``, species populations ``[ns, 5, ny, nx]``; state between steps is
the pre-collision population set.

Paper passages followed (Sitaru & Gekle, arXiv 2109.04455):
* efficiency, Eq. A-B (Sec. "System parameters and dimensionless numbers");
* flow LB, Eq. LBE (Sec. "Lattice-Boltzmann for the Navier-Stokes equation");
* ADR LB, Eqs. LBE_ADE, BGK, the equilibrium, Diffusion_LBM, source_lbm;
* boundaries and outflux, Eq. BC (Sec. "Boundary conditions and flux
  computation in ADE").
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbref.c")
_LIB = os.path.join(_HERE, "liblbref.so")

PERIODIC_X = 1
PERIODIC_Y = 2
LINK = 0
NODE = 1
NODE_AT_CATALYST = 2

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no OpenMP, no fast-math)."""
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
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
        d, i, l = ctypes.c_double, ctypes.c_int, ctypes.c_long
        p = ctypes.c_void_p
        _lib.ref_inlet_velocity.restype = d
        _lib.ref_inlet_velocity.argtypes = [i, d, i]
        _lib.ref_flow_init.argtypes = [i, i, p, d, p]
        _lib.ref_flow_run.argtypes = [i, i, p, d, d, p, l]
        _lib.ref_flow_velocity.argtypes = [i, i, p, p, p, p, p]
        _lib.ref_adr_init.argtypes = [i, i, i, p, p, p, d, d, p]
        _lib.ref_adr_run.argtypes = [i, i, i, p, p, p, p, p, d, d, d, i, i, p, l, p]
        _lib.ref_adr_observe.argtypes = [i, i, i, p, p, d, i, p, p]
        _lib.ref_adr_concentration.argtypes = [i, i, i, p, p, p]
        _lib.ref_adr_totals.argtypes = [i, i, i, p, p, p]
        _lib.ref_adr_production.argtypes = [i, i, i, p, p, p, i, i, p, p]
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


# --------------------------------------------------------------------------- flow
def inlet_velocity(ny: int, u0: float, y: int) -> float:
    return lib().ref_inlet_velocity(ny, u0, y)


def flow_init(node_type, u0):
    t = _u8(node_type)
    ny, nx = t.shape
    f = np.zeros((9, ny, nx))
    lib().ref_flow_init(nx, ny, _ptr(t), u0, _ptr(f))
    return f


def flow_run(node_type, f, tau, u0, nsteps):
    """Advance the D2Q9 state ``f`` (in place) by ``nsteps`` steps."""
    t = _u8(node_type)
    ny, nx = t.shape
    assert f.flags.c_contiguous and f.dtype == np.float64 and f.shape == (9, ny, nx)
    lib().ref_flow_run(nx, ny, _ptr(t), tau, u0, _ptr(f), int(nsteps))
    return f


def flow_velocity(node_type, f, with_rho=False):
    t = _u8(node_type)
    ny, nx = t.shape
    ux = np.zeros((ny, nx)); uy = np.zeros((ny, nx)); rho = np.zeros((ny, nx))
    lib().ref_flow_velocity(nx, ny, _ptr(t), _ptr(f), _ptr(ux), _ptr(uy), _ptr(rho))
    return (ux, uy, rho) if with_rho else (ux, uy)


def flow_steady(node_type, tau, u0, max_steps, check_every=1000, tol=1e-6):
    """Run until max|u(t)-u(t-check_every)| <= tol*u0 (or max_steps).

    Returns (ux, uy, steps_done, residual)."""
    f = flow_init(node_type, u0)
    ux, uy = flow_velocity(node_type, f)
    steps, res = 0, np.inf
    while steps < max_steps:
        n = min(check_every, max_steps - steps)
        flow_run(node_type, f, tau, u0, n)
        steps += n
        nux, nuy = flow_velocity(node_type, f)
        res = max(np.abs(nux - ux).max(), np.abs(nuy - uy).max())
        ux, uy = nux, nuy
        if tol > 0 and n == check_every and res <= tol * u0:
            break
    return ux, uy, steps, res


# ---------------------------------------------------------------------------- ADR
def adr_init(node_type, ux, uy, nspecies, c_in=1.0, vel_scale=1.0):
    t = _u8(node_type)
    ny, nx = t.shape
    g = np.zeros((nspecies, 5, ny, nx))
    lib().ref_adr_init(nx, ny, nspecies, _ptr(t), _ptr(_f64(ux)), _ptr(_f64(uy)),
                       vel_scale, c_in, _ptr(g))
    return g


def adr_run(node_type, k, ux, uy, g, tau, nsteps, c_in=1.0, vel_scale=1.0,
            mode=LINK, bc=0, k2=None, trace=False):
    """Advance the species state ``g`` (in place).  With ``trace`` the
    pre-collision concentration of every step is returned [nsteps, ns, ny, nx]."""
    t = _u8(node_type)
    ny, nx = t.shape
    ns = g.shape[0]
    assert g.flags.c_contiguous and g.dtype == np.float64 and g.shape == (ns, 5, ny, nx)
    k = _f64(k); ux = _f64(ux); uy = _f64(uy)
    k2 = None if k2 is None else _f64(k2)
    tr = np.zeros((int(nsteps), ns, ny, nx)) if trace else None
    lib().ref_adr_run(nx, ny, ns, _ptr(t), _ptr(k), _ptr(k2), _ptr(ux), _ptr(uy),
                      vel_scale, tau, c_in, mode, bc, _ptr(g), int(nsteps), _ptr(tr))
    return tr if trace else g


def adr_observe(node_type, g, c_in=1.0, xf=None):
    """(N[ns], inflow_A) of the last streaming; xf defaults to nx-3."""
    t = _u8(node_type)
    ny, nx = t.shape
    ns = g.shape[0]
    xf = nx - 3 if xf is None else xf
    flux = np.zeros(ns); inflow = np.zeros(1)
    lib().ref_adr_observe(nx, ny, ns, _ptr(t), _ptr(g), c_in, xf, _ptr(flux), _ptr(inflow))
    return flux, float(inflow[0])


def efficiency(flux):
    """Eq. A-B: N_B/(N_A+N_B) for A->B, N_C/(N_A+N_B+N_C) for the cascade."""
    flux = np.asarray(flux, dtype=np.float64)
    den = flux.sum()
    return float(flux[-1] / den) if den != 0 else float("nan")


def adr_concentration(node_type, g):
    t = _u8(node_type)
    ny, nx = t.shape
    ns = g.shape[0]
    c = np.zeros((ns, ny, nx))
    lib().ref_adr_concentration(nx, ny, ns, _ptr(t), _ptr(g), _ptr(c))
    return c


# A steady state accumulates nothing, so every cross-section carries the
# inflow: a check counts as steady only when the fluxes through the outlet
# face balance the inflow of A to this fraction of it.
MASS_BALANCE_TOL = 1e-3


def is_steady(flux, inflow, eps, prev, tol):
    """Steady-state reading of one check: eps changed by at most tol of itself
    since the previous check, the final product already leaves (positive
    outflux: before its front reaches the flux plane eps is 0 at every
    check) and the outlet fluxes balance the inflow."""
    if not tol > 0 or prev is None or not np.isfinite(eps) or not flux[-1] > 0:
        return False
    if not abs(float(np.sum(flux)) - inflow) <= MASS_BALANCE_TOL * abs(inflow):
        return False
    return abs(eps - prev) <= tol * abs(eps)


def adr_steady(node_type, k, ux, uy, nspecies, tau, max_steps, check_every=1000,
               tol=1e-8, c_in=1.0, vel_scale=1.0, mode=LINK, g=None):
    """Run until a check is steady (``is_steady``), or max_steps.

    Returns (g, steps_done, flux, inflow, eps)."""
    if g is None:
        g = adr_init(node_type, ux, uy, nspecies, c_in, vel_scale)
    steps, prev = 0, None
    flux, inflow, eps = None, None, float("nan")
    while steps < max_steps:
        n = min(check_every, max_steps - steps)
        adr_run(node_type, k, ux, uy, g, tau, n, c_in, vel_scale, mode)
        steps += n
        flux, inflow = adr_observe(node_type, g, c_in)
        eps = efficiency(flux)
        if is_steady(flux, inflow, eps, prev, tol):
            break
        prev = eps
    return g, steps, flux, inflow, eps


def adr_totals(node_type, g):
    """Total amount of each species over the fluid nodes."""
    t = _u8(node_type)
    ny, nx = t.shape
    ns = g.shape[0]
    tot = np.zeros(ns)
    lib().ref_adr_totals(nx, ny, ns, _ptr(t), _ptr(g), _ptr(tot))
    return tot


def adr_production(node_type, k, g, mode=LINK, bc=0, k2=None):
    """Amount each reaction converts in the next step from the pre-collision
    state g (Eq. source_lbm summed over the lattice): [A->B] or, with three
    species, [A->B, B->C]."""
    t = _u8(node_type)
    ny, nx = t.shape
    ns = g.shape[0]
    assert g.flags.c_contiguous and g.dtype == np.float64 and g.shape == (ns, 5, ny, nx)
    k = _f64(k)
    k2 = None if k2 is None else _f64(k2)
    rate = np.zeros(2)
    lib().ref_adr_production(nx, ny, ns, _ptr(t), _ptr(k), _ptr(k2), mode, bc, _ptr(g), _ptr(rate))
    return rate[: ns - 1]
