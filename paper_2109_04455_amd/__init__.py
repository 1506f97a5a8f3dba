"""MI355X lattice-Boltzmann flow + advection-diffusion-reaction for catalytic
fibre cross-sections (Sitaru & Gekle, arXiv 2109.04455).

Thin Python binding of the C ABI in ``include/lbf.h``: the methods marshal
arguments and device pointers; every step of the computation runs in the HIP
kernels of ``liblbf.so``.  PyTorch provides the device memory (workspace,
inputs, outputs) and the stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import Lbf3Params, LbfParams, LbfRwParams

__all__ = ["LbfError", "LbfNotConverged", "Context", "Batch", "params", "lib", "probe_copy",
           "workspace_tensor"]


class LbfError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


class LbfNotConverged(LbfError):
    pass


def lib():
    return _lib.load()


def _check(status, ctx_handle=None, what=""):
    if status == _lib.OK:
        return
    L = lib()
    msg = L.lbf_status_str(status).decode()
    if ctx_handle is not None:
        detail = L.lbf_last_error(ctx_handle)
        if detail:
            msg = f"{msg}: {detail.decode()}"
    if what:
        msg = f"{what}: {msg}"
    cls = LbfNotConverged if status == _lib.ENOTCONV else LbfError
    raise cls(status, msg)


LINK, NODE_AT_CATALYST = 0, 1   # reaction_mode
CHANNEL, PERIODIC = 0, 1         # boundary


def params(nx, ny, *, real="f32", nspecies=3, tau_f=0.8, u0=0.05, tau_g=0.8, c_in=1.0,
           vel_scale=1.0, flux_col=-1, tile_x=0, tile_y=0, variant=0, flags=0,
           reaction_mode=LINK, boundary=CHANNEL) -> LbfParams:
    p = LbfParams()
    _check(lib().lbf_params_default(ctypes.byref(p), nx, ny))
    p.real_bytes = {"f32": 4, "f64": 8}[real]
    p.nspecies = nspecies
    p.tau_f, p.u0, p.tau_g, p.c_in, p.vel_scale = tau_f, u0, tau_g, c_in, vel_scale
    p.flux_col, p.tile_x, p.tile_y = flux_col, tile_x, tile_y
    p.variant, p.flags = variant, flags
    p.reaction_mode, p.boundary = reaction_mode, boundary
    return p


def workspace_tensor(nbytes, device):
    """A 256-byte aligned uint8 device tensor of at least nbytes."""
    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t, t.data_ptr() + off


def _stream_handle(stream):
    return ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)


class Context:
    """One lattice: geometry, flow, ADR species, observables, adjoint.

    All device work is enqueued on ``stream`` (default: the current torch
    stream when the context is created)."""

    def __init__(self, p: LbfParams, device="cuda", stream=None):
        self.p = p
        self.device = torch.device(device)
        self.real = {4: torch.float32, 8: torch.float64}[p.real_bytes]
        self.nx, self.ny, self.ns = p.nx, p.ny, p.nspecies
        h = ctypes.c_void_p()
        st = lib().lbf_create(ctypes.byref(p), ctypes.byref(h))
        self._h = h
        if st != _lib.OK:
            try:
                _check(st, h, "lbf_create")
            finally:
                lib().lbf_destroy(h)
                self._h = None
        nbytes = ctypes.c_size_t()
        _check(lib().lbf_workspace_bytes(h, ctypes.byref(nbytes)), h)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ws, ptr = workspace_tensor(nbytes.value, self.device)
        _check(lib().lbf_bind(h, ctypes.c_void_p(ptr), nbytes.value, _stream_handle(self.stream)), h,
               "lbf_bind")
        self._keep = []

    # ---------------------------------------------------------------- helpers
    def _call(self, name, *args):
        _check(getattr(lib(), name)(self._h, *args), self._h, name)

    def _dev(self, a, dtype):
        t = torch.as_tensor(a)
        return t.to(device=self.device, dtype=dtype).contiguous()

    def close(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.device)
            lib().lbf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --------------------------------------------------------------- set-up
    def set_geometry(self, node_type):
        t = self._dev(node_type, torch.uint8)
        assert t.shape == (self.ny, self.nx)
        with torch.cuda.stream(self.stream):
            self._call("lbf_set_geometry", ctypes.c_void_p(t.data_ptr()))

    def set_rates(self, k):
        t = self._dev(k, torch.float64)
        assert t.shape == (self.ny, self.nx)
        with torch.cuda.stream(self.stream):
            self._call("lbf_set_rates", ctypes.c_void_p(t.data_ptr()))

    # ------------------------------------------------------------------ flow
    def flow_init(self):
        self._call("lbf_flow_init")

    def flow_run(self, nsteps):
        self._call("lbf_flow_run", int(nsteps))

    def flow_steady(self, max_steps, check_every=1000, tol=1e-6, raise_not_converged=False):
        steps = ctypes.c_long()
        res = ctypes.c_double()
        st = lib().lbf_flow_steady(self._h, int(max_steps), int(check_every), float(tol),
                                   ctypes.byref(steps), ctypes.byref(res))
        if st != _lib.ENOTCONV or raise_not_converged:
            _check(st, self._h, "lbf_flow_steady")
        return steps.value, res.value, st == _lib.OK

    def get_velocity(self):
        ux = torch.empty((self.ny, self.nx), dtype=self.real, device=self.device)
        uy = torch.empty_like(ux)
        self._call("lbf_get_velocity", ctypes.c_void_p(ux.data_ptr()), ctypes.c_void_p(uy.data_ptr()))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return ux, uy

    def set_velocity(self, ux, uy):
        a = self._dev(ux, self.real)
        b = self._dev(uy, self.real)
        with torch.cuda.stream(self.stream):
            self._call("lbf_set_velocity", ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()))
        self._keep = [a, b]

    # ------------------------------------------------------------------- ADR
    def adr_init(self):
        self._call("lbf_adr_init")

    def adr_run(self, max_steps, check_every=1000, tol=0.0, raise_not_converged=False):
        steps = ctypes.c_long()
        st = lib().lbf_adr_run(self._h, int(max_steps), int(check_every), float(tol),
                               ctypes.byref(steps))
        if st != _lib.ENOTCONV or raise_not_converged:
            _check(st, self._h, "lbf_adr_run")
        return steps.value, st == _lib.OK

    def efficiency(self):
        eps = ctypes.c_double()
        n = (ctypes.c_double * 3)()
        inflow = ctypes.c_double()
        self._call("lbf_efficiency", ctypes.byref(eps), n, ctypes.byref(inflow))
        return eps.value, np.array(n[: self.ns]), inflow.value

    def concentration(self, species):
        out = torch.empty((self.ny, self.nx), dtype=self.real, device=self.device)
        self._call("lbf_get_concentration", int(species), ctypes.c_void_p(out.data_ptr()))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return out

    def totals(self):
        """Total amount of every species over the fluid nodes (FP64 sums)."""
        t = (ctypes.c_double * 3)()
        self._call("lbf_adr_totals", t)
        return np.array(t[: self.ns])

    def production(self):
        """Amount each reaction converts in the next step: [A->B] or
        [A->B, B->C] (FP64 sums over the lattice)."""
        r = (ctypes.c_double * 2)()
        self._call("lbf_adr_production", r)
        return np.array(r[: self.ns - 1])

    def adr_steps(self):
        s = ctypes.c_long()
        self._call("lbf_adr_steps", ctypes.byref(s))
        return s.value

    # --------------------------------------------------------------- adjoint
    def adjoint_path(self, T, ckpt_every=200, budget_fraction=0.25):
        """True (keep the whole trace: ~2x the forward) when its workspace fits
        in budget_fraction of the free device memory, else False
        (checkpoints + recompute: ~3x the forward, memory ~ T/ckpt_every
        lattices)."""
        nbytes = ctypes.c_size_t()
        self._call("lbf_adjoint_workspace_bytes", int(T), int(ckpt_every), 1, ctypes.byref(nbytes))
        free, _ = torch.cuda.mem_get_info(self.device)
        return nbytes.value <= budget_fraction * free

    def adjoint(self, T, ckpt_every=200, keep_trace=None):
        """(eps, grad_k [ny, nx] float64 tensor) after T further steps.
        keep_trace None: chosen by adjoint_path."""
        if keep_trace is None:
            keep_trace = self.adjoint_path(T, ckpt_every)
        nbytes = ctypes.c_size_t()
        self._call("lbf_adjoint_workspace_bytes", int(T), int(ckpt_every), int(bool(keep_trace)),
                   ctypes.byref(nbytes))
        ws, ptr = workspace_tensor(nbytes.value, self.device)
        grad = torch.zeros((self.ny, self.nx), dtype=torch.float64, device=self.device)
        eps = ctypes.c_double()
        torch.cuda.synchronize(self.device)
        self._call("lbf_adr_adjoint", int(T), int(ckpt_every), int(bool(keep_trace)),
                   ctypes.c_void_p(ptr), nbytes.value, ctypes.byref(eps),
                   ctypes.c_void_p(grad.data_ptr()))
        del ws
        return eps.value, grad

    def adjoint_steady(self, max_iters=1_000_000, check_every=1000, tol=1e-12,
                       raise_not_converged=True):
        """(eps, grad_k, iterations) of the steady efficiency at the current
        (converged) state."""
        nbytes = ctypes.c_size_t()
        self._call("lbf_adjoint_workspace_bytes", 1, 1, 1, ctypes.byref(nbytes))
        ws, ptr = workspace_tensor(nbytes.value, self.device)
        grad = torch.zeros((self.ny, self.nx), dtype=torch.float64, device=self.device)
        eps = ctypes.c_double()
        iters = ctypes.c_long()
        torch.cuda.synchronize(self.device)
        st = lib().lbf_adr_adjoint_steady(self._h, int(max_iters), int(check_every), float(tol),
                                          ctypes.c_void_p(ptr), nbytes.value, ctypes.byref(eps),
                                          ctypes.c_void_p(grad.data_ptr()), ctypes.byref(iters))
        if st != _lib.ENOTCONV or raise_not_converged:
            _check(st, self._h, "lbf_adr_adjoint_steady")
        del ws
        return eps.value, grad, iters.value

    # ----------------------------------------------------- checkpoint/resume
    def get_state(self):
        n = ctypes.c_size_t()
        self._call("lbf_state_bytes", ctypes.byref(n))
        buf = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        self._call("lbf_get_state", ctypes.c_void_p(buf.data_ptr()))
        return buf

    def set_state(self, buf):
        torch.cuda.synchronize(self.device)
        self._call("lbf_set_state", ctypes.c_void_p(buf.data_ptr()))

    # ---------------------------------------------------------------- timing
    def prepare_adr_steps(self, nsteps):
        """Instantiate the step-block graphs of nsteps ADR steps ahead of use."""
        self._call("lbf_prepare_adr_steps", int(nsteps))

    def time_adr_steps(self, nsteps):
        ms = ctypes.c_double()
        self._call("lbf_time_adr_steps", int(nsteps), ctypes.byref(ms))
        return ms.value

    def time_flow_steps(self, nsteps):
        ms = ctypes.c_double()
        self._call("lbf_time_flow_steps", int(nsteps), ctypes.byref(ms))
        return ms.value


def params3d(nx, ny, nz, *, real="f32", nspecies=3, tau_f=0.8, force_x=1e-6, tau_g=0.8,
             c_in=1.0, vel_scale=1.0, flux_col=-1, tile_x=0, tile_y=0, flags=0) -> Lbf3Params:
    p = Lbf3Params()
    _check(lib().lbf3_params_default(ctypes.byref(p), nx, ny, nz))
    p.real_bytes = {"f32": 4, "f64": 8}[real]
    p.nspecies = nspecies
    p.tau_f, p.force_x, p.tau_g, p.c_in, p.vel_scale = tau_f, force_x, tau_g, c_in, vel_scale
    p.flux_col, p.tile_x, p.tile_y, p.flags = flux_col, tile_x, tile_y, flags
    return p


class Context3D:
    """One 3D lattice (fields ``[nz, ny, nx]``): forced periodic D3Q19 flow,
    D3Q7 ADR with inlet/outlet in x, observables."""

    def __init__(self, p: Lbf3Params, device="cuda", stream=None):
        self.p = p
        self.device = torch.device(device)
        self.real = {4: torch.float32, 8: torch.float64}[p.real_bytes]
        self.shape = (p.nz, p.ny, p.nx)
        self.ns = p.nspecies
        h = ctypes.c_void_p()
        st = lib().lbf3_create(ctypes.byref(p), ctypes.byref(h))
        self._h = h
        if st != _lib.OK:
            msg = lib().lbf3_last_error(h).decode()
            lib().lbf3_destroy(h)
            self._h = None
            raise LbfError(st, f"lbf3_create: {lib().lbf_status_str(st).decode()}: {msg}")
        nbytes = ctypes.c_size_t()
        self._call("lbf3_workspace_bytes", ctypes.byref(nbytes))
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ws, ptr = workspace_tensor(nbytes.value, self.device)
        self._call("lbf3_bind", ctypes.c_void_p(ptr), nbytes.value, _stream_handle(self.stream))
        self._keep = []

    def _call(self, name, *args):
        st = getattr(lib(), name)(self._h, *args)
        if st != _lib.OK:
            detail = lib().lbf3_last_error(self._h).decode()
            cls = LbfNotConverged if st == _lib.ENOTCONV else LbfError
            raise cls(st, f"{name}: {lib().lbf_status_str(st).decode()}: {detail}")

    def _dev(self, a, dtype):
        return torch.as_tensor(a).to(device=self.device, dtype=dtype).contiguous()

    def close(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.device)
            lib().lbf3_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_geometry(self, node_type):
        t = self._dev(node_type, torch.uint8)
        assert tuple(t.shape) == self.shape
        with torch.cuda.stream(self.stream):
            self._call("lbf3_set_geometry", ctypes.c_void_p(t.data_ptr()))

    def set_rates(self, k):
        t = self._dev(k, torch.float64)
        assert tuple(t.shape) == self.shape
        with torch.cuda.stream(self.stream):
            self._call("lbf3_set_rates", ctypes.c_void_p(t.data_ptr()))

    def flow_init(self):
        self._call("lbf3_flow_init")

    def flow_run(self, nsteps):
        self._call("lbf3_flow_run", int(nsteps))

    def flow_steady(self, max_steps, check_every=1000, tol=1e-5):
        """Returns (steps, residual, converged)."""
        steps, res = ctypes.c_long(), ctypes.c_double()
        st = lib().lbf3_flow_steady(self._h, int(max_steps), int(check_every), float(tol),
                                    ctypes.byref(steps), ctypes.byref(res))
        if st not in (_lib.OK, _lib.ENOTCONV):
            raise LbfError(st, lib().lbf3_last_error(self._h).decode())
        return steps.value, res.value, st == _lib.OK

    def get_velocity(self):
        u = [torch.empty(self.shape, dtype=self.real, device=self.device) for _ in range(3)]
        self._call("lbf3_get_velocity", *[ctypes.c_void_p(t.data_ptr()) for t in u])
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return torch.stack(u)

    def set_velocity(self, u):
        ts = [self._dev(u[c], self.real) for c in range(3)]
        with torch.cuda.stream(self.stream):
            self._call("lbf3_set_velocity", *[ctypes.c_void_p(t.data_ptr()) for t in ts])
        self._keep = ts

    def adr_init(self):
        self._call("lbf3_adr_init")

    def adr_run(self, max_steps, check_every=1000, tol=0.0):
        steps = ctypes.c_long()
        st = lib().lbf3_adr_run(self._h, int(max_steps), int(check_every), float(tol),
                                ctypes.byref(steps))
        if st not in (_lib.OK, _lib.ENOTCONV):
            raise LbfError(st, lib().lbf3_last_error(self._h).decode())
        return steps.value, st == _lib.OK

    def efficiency(self):
        eps, inflow = ctypes.c_double(), ctypes.c_double()
        n = (ctypes.c_double * 3)()
        self._call("lbf3_efficiency", ctypes.byref(eps), n, ctypes.byref(inflow))
        return eps.value, np.array(n[: self.ns]), inflow.value

    def concentration(self, species):
        out = torch.empty(self.shape, dtype=self.real, device=self.device)
        self._call("lbf3_get_concentration", int(species), ctypes.c_void_p(out.data_ptr()))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return out

    def totals(self):
        t = (ctypes.c_double * 3)()
        self._call("lbf3_adr_totals", t)
        return np.array(t[: self.ns])

    def time_adr_steps(self, nsteps):
        ms = ctypes.c_double()
        self._call("lbf3_time_adr_steps", int(nsteps), ctypes.byref(ms))
        return ms.value

    def time_flow_steps(self, nsteps):
        ms = ctypes.c_double()
        self._call("lbf3_time_flow_steps", int(nsteps), ctypes.byref(ms))
        return ms.value


def rw_params(nx, ny, *, nspecies=2, D=0.05, dt=0.5, zone=1.0, rate_w=1.0 / 6.0, density=10.0,
              vel_scale=1.0, xf=-1, wall_mode=1, seed=1, capacity=None) -> LbfRwParams:
    p = LbfRwParams()
    _check(lib().lbf_rw_params_default(ctypes.byref(p), nx, ny))
    p.nspecies, p.D, p.dt, p.zone, p.rate_w = nspecies, D, dt, zone, rate_w
    p.density, p.vel_scale, p.xf, p.wall_mode, p.seed = density, vel_scale, xf, wall_mode, seed
    p.capacity = int(capacity) if capacity else int(density * 1.5 * nx * ny) + 4096
    return p


class RandomWalk:
    """GPU random-walk particle tracker on a 2D lattice geometry and flow."""

    def __init__(self, p: LbfRwParams, device="cuda", stream=None):
        self.p = p
        self.device = torch.device(device)
        h = ctypes.c_void_p()
        st = lib().lbf_rw_create(ctypes.byref(p), ctypes.byref(h))
        self._h = h
        if st != _lib.OK:
            msg = lib().lbf_rw_last_error(h).decode()
            lib().lbf_rw_destroy(h)
            self._h = None
            raise LbfError(st, f"lbf_rw_create: {msg}")
        nbytes = ctypes.c_size_t()
        self._call("lbf_rw_workspace_bytes", ctypes.byref(nbytes))
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ws, ptr = workspace_tensor(nbytes.value, self.device)
        self._call("lbf_rw_bind", ctypes.c_void_p(ptr), nbytes.value, _stream_handle(self.stream))

    def _call(self, name, *args):
        st = getattr(lib(), name)(self._h, *args)
        if st != _lib.OK:
            raise LbfError(st, f"{name}: {lib().lbf_status_str(st).decode()}: "
                               f"{lib().lbf_rw_last_error(self._h).decode()}")

    def close(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.device)
            lib().lbf_rw_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fields(self, node_type, ux, uy, k):
        ts = [torch.as_tensor(node_type).to(self.device, torch.uint8).contiguous()]
        ts += [torch.as_tensor(a).to(self.device, torch.float64).contiguous() for a in (ux, uy, k)]
        with torch.cuda.stream(self.stream):
            self._call("lbf_rw_set_fields", *[ctypes.c_void_p(t.data_ptr()) for t in ts])
        torch.cuda.synchronize(self.device)

    def fill(self):
        self._call("lbf_rw_fill")

    def run(self, nsteps, measure=False):
        self._call("lbf_rw_run", int(nsteps), int(bool(measure)))

    def counts(self):
        """(N[ns] net crossings per unit time, particles held, measured steps)."""
        n = (ctypes.c_double * 3)()
        np_, steps = ctypes.c_long(), ctypes.c_long()
        self._call("lbf_rw_counts", n, ctypes.byref(np_), ctypes.byref(steps))
        return np.array(n[: self.p.nspecies]), np_.value, steps.value

    def walk(self, ids, x, y, species, t0, steps):
        """Trajectory mode on device copies; returns (x, y, species) tensors."""
        ids = torch.as_tensor(np.asarray(ids, dtype=np.uint64).view(np.int64)).to(self.device)
        x = torch.as_tensor(x, dtype=torch.float64).to(self.device).clone()
        y = torch.as_tensor(y, dtype=torch.float64).to(self.device).clone()
        sp = torch.as_tensor(species, dtype=torch.uint8).to(self.device).clone()
        with torch.cuda.stream(self.stream):
            self._call("lbf_rw_walk", int(x.numel()), ctypes.c_void_p(ids.data_ptr()),
                       ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                       ctypes.c_void_p(sp.data_ptr()), int(t0), int(steps))
        torch.cuda.synchronize(self.device)
        return x, y, sp

    def time_steps(self, nsteps, measure=False):
        ms = ctypes.c_double()
        self._call("lbf_rw_time_steps", int(nsteps), int(bool(measure)), ctypes.byref(ms))
        return ms.value


def probe_copy(nbytes, device="cuda", stream=None):
    """Time one device-to-device copy of nbytes with the library's copy kernel;
    returns milliseconds."""
    src = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
    dst = torch.empty_like(src)
    src.fill_(1)
    s = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
    torch.cuda.synchronize(device)
    ms = ctypes.c_double()
    _check(lib().lbf_probe_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                int(nbytes), _stream_handle(s), ctypes.byref(ms)))
    return ms.value


class Batch:
    """Many independent lattices stepped together (the Pe x Da sweep).

    ``plist`` holds one LbfParams per instance (shared precision, species
    count, tau_f, u0, c_in); geometry and rates are given per instance."""

    def __init__(self, plist, device="cuda", stream=None):
        self.n = len(plist)
        self.device = torch.device(device)
        self.plist = list(plist)
        arr = (LbfParams * self.n)(*self.plist)
        h = ctypes.c_void_p()
        st = lib().lbf_batch_create(self.n, arr, ctypes.byref(h))
        self._h = h
        if st != _lib.OK:
            msg = lib().lbf_batch_last_error(h).decode() if h else ""
            lib().lbf_batch_destroy(h)
            self._h = None
            raise LbfError(st, f"lbf_batch_create: {msg}")
        nbytes = ctypes.c_size_t()
        self._call("lbf_batch_workspace_bytes", ctypes.byref(nbytes))
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ws, ptr = workspace_tensor(nbytes.value, self.device)
        self._call("lbf_batch_bind", ctypes.c_void_p(ptr), nbytes.value, _stream_handle(self.stream))
        self.real = {4: torch.float32, 8: torch.float64}[self.plist[0].real_bytes]

    def _call(self, name, *args):
        st = getattr(lib(), name)(self._h, *args)
        if st != _lib.OK:
            msg = lib().lbf_batch_last_error(self._h).decode()
            cls = LbfNotConverged if st == _lib.ENOTCONV else LbfError
            raise cls(st, f"{name}: {msg}")

    def close(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.device)
            lib().lbf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_geometry(self, node_types, rates):
        t = torch.cat([torch.as_tensor(np.ascontiguousarray(a, dtype=np.uint8)).reshape(-1)
                       for a in node_types]).to(self.device)
        k = torch.cat([torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).reshape(-1)
                       for a in rates]).to(self.device)
        torch.cuda.synchronize(self.device)
        self._call("lbf_batch_set_geometry", ctypes.c_void_p(t.data_ptr()),
                   ctypes.c_void_p(k.data_ptr()))

    def flow(self, max_steps, check_every=1000, tol=0.0):
        self._call("lbf_batch_flow", int(max_steps), int(check_every), float(tol))

    def run(self, max_steps, check_every=1000, tol=0.0, raise_not_converged=False):
        """(eps[n], product_flux[n], steps[n]) as numpy arrays.  Afterwards
        ``all_converged`` says whether every instance passed its test."""
        return self._advance("lbf_batch_run", max_steps, check_every, tol, raise_not_converged)

    def resume(self, more_steps, check_every=1000, tol=0.0, raise_not_converged=False):
        """Continue the current run by more_steps steps (same outputs)."""
        return self._advance("lbf_batch_resume", more_steps, check_every, tol,
                             raise_not_converged)

    def _advance(self, name, nsteps, check_every, tol, raise_not_converged):
        eps = (ctypes.c_double * self.n)()
        prod = (ctypes.c_double * self.n)()
        steps = (ctypes.c_long * self.n)()
        st = getattr(lib(), name)(self._h, int(nsteps), int(check_every), float(tol), eps, prod,
                                  steps)
        if st != _lib.OK and (st != _lib.ENOTCONV or raise_not_converged):
            msg = lib().lbf_batch_last_error(self._h).decode()
            cls = LbfNotConverged if st == _lib.ENOTCONV else LbfError
            raise cls(st, f"{name}: {msg}")
        self.all_converged = st == _lib.OK and tol > 0
        return np.array(eps[:]), np.array(prod[:]), np.array(steps[:])

    def concentration(self, i, species):
        p = self.plist[i]
        out = torch.empty((p.ny, p.nx), dtype=self.real, device=self.device)
        self._call("lbf_batch_get_concentration", int(i), int(species),
                   ctypes.c_void_p(out.data_ptr()))
        torch.cuda.synchronize(self.device)
        return out

    def time_steps(self, nsteps):
        ms = ctypes.c_double()
        self._call("lbf_batch_time_steps", int(nsteps), ctypes.byref(ms))
        return ms.value
