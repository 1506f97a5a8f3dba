"""``torch.autograd.Function`` around the adjoint entry point: the efficiency
after T steps as a differentiable function of the catalytic rates, for
catalyst-placement studies.

    f = EfficiencyOfRates(ctx, node_type, T=20000, ckpt_every=200)
    k = torch.tensor(..., requires_grad=True)   # one rate per catalytic node
    eps = f(k)
    eps.backward()                              # k.grad = d eps / d k

Every call restarts from the state the context had when ``f`` was built (that
pre-collision state is held fixed), sets the rates and runs the forward +
reverse sweep of ``lbf_adr_adjoint`` on the GPU.
"""
from __future__ import annotations

import numpy as np
import torch


class _Eps(torch.autograd.Function):
    @staticmethod
    def forward(fctx, k_cat, runner):
        eps, grad_cat = runner._run(k_cat)
        fctx.save_for_backward(grad_cat)
        return torch.tensor(eps, dtype=torch.float64)

    @staticmethod
    def backward(fctx, grad_out):
        (grad_cat,) = fctx.saved_tensors
        return grad_out * grad_cat, None


class EfficiencyOfRates:
    """eps(k) over a fixed window of T ADR steps of an existing context."""

    def __init__(self, ctx, node_type, T, ckpt_every=200, keep_trace=None):
        self.ctx = ctx
        t = np.asarray(node_type)
        self.cat = np.nonzero(t >= 2)
        self.shape = t.shape
        self.T, self.M = int(T), int(ckpt_every)
        self.keep = None if keep_trace is None else bool(keep_trace)  # None: by memory
        self.start = ctx.get_state()

    def _run(self, k_cat):
        k = np.zeros(self.shape)
        k[self.cat] = k_cat.detach().cpu().double().numpy()
        self.ctx.set_rates(k)
        self.ctx.set_state(self.start)
        eps, grad = self.ctx.adjoint(self.T, self.M, self.keep)
        g = grad.cpu()[torch.as_tensor(self.cat[0]), torch.as_tensor(self.cat[1])]
        return eps, g.to(dtype=k_cat.dtype)

    def __call__(self, k_cat):
        return _Eps.apply(k_cat, self)
