"""lbf_efficiency_noalloc -- the outlet fluxes, inflow and eps of a state blob
with the scratch in the library's file-scope device array, for callers that
cannot allocate -- against lbf_efficiency of the context the blob came from:
two calls in a row, the second on a smaller lattice (and the other
precision), then the first again."""
import ctypes

import numpy as np
import pytest
import torch

from workloads import make_workload

pytestmark = pytest.mark.gpu


def _noalloc():
    from paper_2109_04455_amd import _lib
    return _lib.load().lbf_efficiency_noalloc


def _case(name, real, flow_steps, adr_steps):
    import paper_2109_04455_amd as L
    w = make_workload(name)
    p = L.params(w.nx, w.ny, real=real, nspecies=w.nspecies, tau_f=w.tau_f, u0=w.u0,
                 tau_g=w.tau_g, c_in=w.c_in, vel_scale=w.vel_scale)
    c = L.Context(p)
    c.set_geometry(w.node_type)
    c.set_rates(w.k)
    c.flow_init()
    c.flow_run(flow_steps)
    c.adr_init()
    c.adr_run(adr_steps, tol=0)
    ref = c.efficiency()
    blob = c.get_state()
    nt = torch.as_tensor(w.node_type, dtype=torch.uint8).to("cuda").contiguous()
    return p, c, ref, blob, nt


def _call(f, p, blob, nt, stream):
    eps = ctypes.c_double()
    n = (ctypes.c_double * 3)()
    inflow = ctypes.c_double()
    st = f(ctypes.byref(p), ctypes.c_void_p(blob.data_ptr()), ctypes.c_void_p(nt.data_ptr()),
           ctypes.c_void_p(stream.cuda_stream), ctypes.byref(eps), n, ctypes.byref(inflow))
    return st, eps.value, np.array(n[: p.nspecies]), inflow.value


def _check(got, ref, ns):
    st, eps, N, inflow = got
    eps_r, N_r, inflow_r = ref
    assert st == 0
    assert abs(inflow - inflow_r) <= 1e-12 * abs(inflow_r)
    assert np.abs(N - N_r).max() <= 1e-12 * abs(inflow_r)
    assert abs(eps - eps_r) <= 1e-10 * abs(eps_r)


def test_noalloc_efficiency_matches_the_context():
    f = _noalloc()
    stream = torch.cuda.current_stream()
    big = _case("C1q", "f32", 2000, 20000)
    small = _case("tiny", "f64", 1500, 2500)
    for p, c, ref, blob, nt in (big, small, big):
        got = _call(f, p, blob, nt, stream)
        print(p.nx, p.ny, p.real_bytes, got[1], ref[0], flush=True)
        assert got[1] > 0
        _check(got, ref, p.nspecies)
    # a blob of one lattice passed with the parameters of the other is refused
    st = _call(f, small[0], big[3], big[4], stream)[0]
    assert st == -1
    for case in (big, small):
        case[1].close()
