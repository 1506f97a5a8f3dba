"""The C-ABI library without a GPU: it loads, exports every entry point that
include/*.h declare, and its host-side validation rejects bad arguments
before any HIP call."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("lbf.h", "lbf3d.h", "lbf_rw.h")]


def _declared():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(lbf(?:3|_rw)?_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_every_header_is_scanned():
    assert sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))) == sorted(HEADERS)


@pytest.fixture(scope="module")
def L():
    from paper_2109_04455_amd import _lib
    return _lib.load()


def test_header_declares_the_expected_calls():
    names = _declared()
    for core in ("lbf_create", "lbf_bind", "lbf_set_geometry", "lbf_set_rates",
                 "lbf_flow_steady", "lbf_adr_run", "lbf_efficiency", "lbf_adr_adjoint",
                 "lbf_batch_run"):
        assert core in names


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_2109_04455_amd import _lib
    assert sorted(_lib.SIGNATURES) == _declared()


def _params(L, **kw):
    from paper_2109_04455_amd._lib import LbfParams
    p = LbfParams()
    assert L.lbf_params_default(ctypes.byref(p), kw.pop("nx", 64), kw.pop("ny", 32)) == 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _create(L, p):
    h = ctypes.c_void_p()
    st = L.lbf_create(ctypes.byref(p), ctypes.byref(h))
    msg = L.lbf_last_error(h).decode()
    L.lbf_destroy(h)
    return st, msg


@pytest.mark.parametrize("field,value,needle", [
    ("nx", 4, "nx >= 8"), ("ny", 2, "ny >= 3"), ("real_bytes", 2, "real_bytes"),
    ("nspecies", 4, "nspecies"), ("reaction_mode", 2, "reaction_mode"),
    ("boundary", 2, "boundary"),
    ("tau_f", 0.5, "tau_f"), ("tau_g", 0.4, "tau_g"), ("u0", 0.4, "u0"),
    ("vel_scale", -1.0, "vel_scale"), ("flux_col", 63, "flux_col"), ("tile_x", 1000, "tile_x"), ("tile_y", 20, "tile_x"),
])
def test_invalid_parameters_rejected(L, field, value, needle):
    st, msg = _create(L, _params(L, **{field: value}))
    assert st == -1 and needle in msg


def test_lattice_size_limits(L):
    # 2^32 nodes is the largest 2D lattice; 3D stops at 2e9 nodes
    st, msg = _create(L, _params(L, nx=70000, ny=70000))
    assert st == -1 and "too large" in msg
    st, _ = _create(L, _params(L, nx=65536, ny=65536))
    assert st == 0
    h = ctypes.c_void_p()
    st = L.lbf3_create(ctypes.byref(_params3(L, nx=2000, ny=1000, nz=1001)), ctypes.byref(h))
    msg = L.lbf3_last_error(h).decode()
    L.lbf3_destroy(h)
    assert st == -1 and "too large" in msg


def test_valid_parameters_and_workspace_arithmetic(L):
    p = _params(L, nx=100, ny=30)
    h = ctypes.c_void_p()
    assert L.lbf_create(ctypes.byref(p), ctypes.byref(h)) == 0
    n = ctypes.c_size_t()
    assert L.lbf_workspace_bytes(h, ctypes.byref(n)) == 0
    nxp, plane = 128, 128 * 30
    # masks, trace maps, rates, two D2Q9 and two 3-species D2Q5 lattices, velocities
    expect_min = plane * (1 + 1 + 2 + 4 + 4 + 4 + 2 * 9 * 4 + 3 * 2 * 4 + 2 * 15 * 4)
    assert expect_min <= n.value <= expect_min + 64 * 1024
    s = ctypes.c_size_t()
    assert L.lbf_state_bytes(h, ctypes.byref(s)) == 0
    assert s.value == 2 * 15 * plane * 4 + 256
    # calls that need a bound workspace report the order error, not a crash
    assert L.lbf_flow_init(h) == -6
    assert L.lbf_bind(h, None, 0, None) == -1
    L.lbf_destroy(h)


@pytest.mark.parametrize("kw", [dict(reaction_mode=1, variant=2), dict(boundary=1, variant=2)])
def test_vector_kernel_rejects_reaction_variant_and_periodic_box(L, kw):
    st, msg = _create(L, _params(L, **kw))
    assert st == -1 and "vector" in msg


def test_reaction_variant_and_periodic_box_accepted(L):
    for kw in (dict(reaction_mode=1), dict(boundary=1), dict(reaction_mode=1, boundary=1, real_bytes=8)):
        st, msg = _create(L, _params(L, **kw))
        assert st == 0, msg


def _params3(L, **kw):
    from paper_2109_04455_amd._lib import Lbf3Params
    p = Lbf3Params()
    assert L.lbf3_params_default(ctypes.byref(p), 40, 24, 20) == 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("field,value,needle", [
    ("nx", 4, "nx >= 8"), ("nz", 1, "nz >= 2"), ("real_bytes", 2, "real_bytes"),
    ("nspecies", 1, "nspecies"), ("tau_f", 0.5, "tau_f"), ("tau_g", 0.2, "tau_g"),
    ("force_x", 0.1, "force_x"), ("vel_scale", -1.0, "vel_scale"), ("flux_col", 39, "flux_col"),
    ("tile_x", 100, "tile_x"), ("tile_y", 20, "tile_x"),
])
def test_3d_invalid_parameters_rejected(L, field, value, needle):
    h = ctypes.c_void_p()
    st = L.lbf3_create(ctypes.byref(_params3(L, **{field: value})), ctypes.byref(h))
    msg = L.lbf3_last_error(h).decode()
    L.lbf3_destroy(h)
    assert st == -1 and needle in msg


def test_3d_workspace_arithmetic(L):
    h = ctypes.c_void_p()
    assert L.lbf3_create(ctypes.byref(_params3(L)), ctypes.byref(h)) == 0
    n = ctypes.c_size_t()
    assert L.lbf3_workspace_bytes(h, ctypes.byref(n)) == 0
    plane = 64 * 24 * 20
    # type, D3Q7 and D3Q19 masks, rates, two D3Q19 and two 3-species D3Q7
    # lattices, three velocity blocks
    expect = plane * (1 + 2 + 4 + 4 + 2 * 19 * 4 + 2 * 21 * 4 + 3 * 3 * 4)
    assert expect <= n.value <= expect + 64 * 1024
    assert L.lbf3_flow_init(h) == -6          # no workspace bound yet
    L.lbf3_destroy(h)


def test_status_strings(L):
    for s in range(0, -7, -1):
        assert L.lbf_status_str(s)
    assert L.lbf_version() >= 1


def test_unshifted_a_with_fp32_arithmetic_rejected(L):
    # flags bit 2 (A stored unshifted) with bit 4 (FP32 arithmetic) misses
    # the 1e-4 accuracy bar on the A field; each alone, and FP64 storage, pass
    st, msg = _create(L, _params(L, flags=4 | 16))
    assert st == -1 and "bits 2 and 4" in msg
    for f in (4, 16, 4 | 32):
        st, msg = _create(L, _params(L, flags=f))
        assert st == 0, msg
    st, msg = _create(L, _params(L, flags=4 | 16, real_bytes=8))
    assert st == 0, msg


def test_noalloc_efficiency_rejects_before_any_device_work(L):
    # host-side checks of the allocation-free entry point: bad parameters,
    # NULL inputs and lattices taller than its scratch (262144 rows)
    p = _params(L, nx=8, ny=300000)
    d = ctypes.c_double()
    assert L.lbf_efficiency_noalloc(ctypes.byref(p), ctypes.c_void_p(16), ctypes.c_void_p(16),
                                    None, ctypes.byref(d), None, None) == -2
    p = _params(L)
    assert L.lbf_efficiency_noalloc(ctypes.byref(p), None, ctypes.c_void_p(16), None,
                                    ctypes.byref(d), None, None) == -1
    p = _params(L, boundary=1)
    assert L.lbf_efficiency_noalloc(ctypes.byref(p), ctypes.c_void_p(16), ctypes.c_void_p(16),
                                    None, ctypes.byref(d), None, None) == -1
    p = _params(L, tau_g=0.4)
    assert L.lbf_efficiency_noalloc(ctypes.byref(p), ctypes.c_void_p(16), ctypes.c_void_p(16),
                                    None, ctypes.byref(d), None, None) == -1
