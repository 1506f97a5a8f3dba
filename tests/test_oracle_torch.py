"""The PyTorch-CPU twin of the ADR step (used for reference gradients) against
the C oracle, and its autograd gradient against central finite differences of
the C oracle."""
import numpy as np
import pytest
import torch

from oracle import lbref as R
from oracle import torch_ref as TR
from workloads import make_workload


@pytest.fixture(scope="module")
def tiny():
    w = make_workload("tiny")
    ux, uy, _, _ = R.flow_steady(w.node_type, w.tau_f, w.u0, 3000, tol=0)
    return w, ux, uy


def test_twin_equals_c_oracle(tiny):
    w, ux, uy = tiny
    g0 = R.adr_init(w.node_type, ux, uy, 3)
    g = g0.copy()
    R.adr_run(w.node_type, w.k, ux, uy, g, w.tau_g, 300)
    sch = TR.Scheme(w.node_type, ux, uy, 3, w.tau_g)
    gt = torch.as_tensor(g0.copy())
    kt = torch.as_tensor(w.k)
    for _ in range(300):
        gt = sch.step(gt, kt)
    assert np.abs(gt.numpy() - g).max() < 1e-13
    n_c, _ = R.adr_observe(w.node_type, g)
    assert np.abs(sch.fluxes(gt).numpy() - n_c).max() < 1e-13


def test_twin_equals_c_oracle_two_species_cdisc():
    w = make_workload("C0")
    # coarse check on the C0 geometry for 50 steps (A->B only)
    ux, uy, _, _ = R.flow_steady(w.node_type, w.tau_f, w.u0, 200, tol=0)
    g0 = R.adr_init(w.node_type, ux, uy, 2)
    g = g0.copy()
    k = w.k * 200  # make the reaction visible within 50 steps
    R.adr_run(w.node_type, k, ux, uy, g, w.tau_g, 50)
    sch = TR.Scheme(w.node_type, ux, uy, 2, w.tau_g)
    gt = torch.as_tensor(g0.copy())
    for _ in range(50):
        gt = sch.step(gt, torch.as_tensor(k))
    assert np.abs(gt.numpy() - g).max() < 1e-13


def test_autograd_gradient_matches_oracle_finite_differences(tiny):
    w, ux, uy = tiny
    g0 = R.adr_init(w.node_type, ux, uy, 3)
    R.adr_run(w.node_type, w.k, ux, uy, g0, w.tau_g, 500)
    T = 600
    eps, grad, _ = TR.eps_and_grad(w.node_type, w.k, ux, uy, g0, 3, w.tau_g, T)
    ys, xs = np.nonzero(w.node_type >= 2)
    assert (grad[w.node_type < 2] == 0).all()
    for j in (3, 25):
        y, x = ys[j], xs[j]
        h = 1e-3 * w.k[y, x]
        e = []
        for sgn in (1, -1):
            kk = w.k.copy(); kk[y, x] += sgn * h
            g = g0.copy()
            R.adr_run(w.node_type, kk, ux, uy, g, w.tau_g, T)
            e.append(R.efficiency(R.adr_observe(w.node_type, g)[0]))
        fd = (e[0] - e[1]) / (2 * h)
        assert abs(grad[y, x] - fd) < 1e-6 * np.abs(grad).max()
