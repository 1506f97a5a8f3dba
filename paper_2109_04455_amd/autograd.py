"""``torch.autograd.Function`` around the adjoint entry point: the efficiency
after T steps as a differentiable function of the catalytic rates, for
catalyst-placement studies.

    f = EfficiencyOfRates(ctx, node_type, T=20000, ckpt_every=200)
    k = torch.tensor(..., requires_grad=True)   # one rate per catalytic node
    eps = f(k)
    eps.backward()                              # k.grad = d eps / d k

The rates are those of the catalytic nodes (node type 2 or 3) in row-major
order of the [ny, nx] lattice.  Every call restarts from the state the context
had when ``f`` was built (that pre-collision state is held fixed), scatters
the rates into the rate map and runs the forward + reverse sweep of
``lbf_adr_adjoint`` on the GPU.  eps is returned as a float64 scalar on the
device of ``k``; the gradient lands on that device with the dtype of ``k``.
After a call the context holds that call's rates and the state T steps after
the start, as ``lbf_adr_adjoint`` leaves it.
"""
from __future__ import annotations

import numpy as np
import torch


class _Eps(torch.autograd.Function):
    @staticmethod
    def forward(fctx, k_cat, runner):
        eps, grad_cat = runner._run(k_cat)
        fctx.save_for_backward(grad_cat)
        return torch.tensor(eps, dtype=torch.float64, device=k_cat.device)

    @staticmethod
    def backward(fctx, grad_out):
        (grad_cat,) = fctx.saved_tensors
        return grad_out.to(grad_cat.dtype) * grad_cat, None


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
        dev = ctx.device
        self._rows = torch.as_tensor(self.cat[0], device=dev)
        self._cols = torch.as_tensor(self.cat[1], device=dev)

    @property
    def ncat(self):
        return int(self.cat[0].size)

    def _run(self, k_cat):
        if k_cat.shape != (self.ncat,):
            raise ValueError(f"expected {self.ncat} rates (one per catalytic node), "
                             f"got shape {tuple(k_cat.shape)}")
        dev = self.ctx.device
        k = torch.zeros(self.shape, dtype=torch.float64, device=dev)
        k[self._rows, self._cols] = k_cat.detach().to(device=dev, dtype=torch.float64)
        self.ctx.set_rates(k)
        self.ctx.set_state(self.start)
        eps, grad = self.ctx.adjoint(self.T, self.M, self.keep)
        g = grad[self._rows, self._cols]
        return eps, g.to(device=k_cat.device, dtype=k_cat.dtype)

    def __call__(self, k_cat):
        return _Eps.apply(k_cat, self)
