"""Iterative reconstruction on top of the projector (TomoSphero Sec. 4.5).

- power_iteration: largest eigenvalue of F^T F (for a safe gradient step);
- CountingOperator: forwards F / F^T and counts calls per object;
- gd: plain gradient descent on ||y - F rho||^2 (Eq. 6) with step
  eta = 1 / (2 lambda_max), rho <- rho - eta * 2 F^T (F rho - y), stopping
  per object when its residual reaches a target;
- adam_tv: ||y - F rho||^2 + lambda TV(rho) minimised with Adam (Listing 7),
  gradients from DataTerm / TV (hand-written kernels, no autograd tracing
  of the ray tracer).
The vector arithmetic (residuals, dot products, updates) runs in the
library's kernels too (nn.residual / dot / axpy / scale).
Batched: every function works on a batch of objects at once (the projector
kernels take batches natively).
"""
import math

import torch

from . import nn as NN
from .nn import TV, Adam


class CountingOperator:
    """F and F^T of a Projector with a per-object call counter."""

    def __init__(self, P, method=None):
        self.P = P
        self.method = method
        self.calls = None

    def reset(self, batch):
        self.calls = torch.zeros(batch, dtype=torch.int64)

    def F(self, rho, active=None):
        self._count(rho.shape[0], active)
        return self.P.forward(rho)

    def FT(self, y, active=None):
        self._count(y.shape[0], active)
        return self.P.backproject(y, self.method)

    def _count(self, B, active):
        if self.calls is None or len(self.calls) != B:
            self.reset(B)
        if active is None:
            self.calls += 1
        else:
            self.calls += active.cpu().long()


def power_iteration(P, iters=20, seed=0):
    """lambda_max(F^T F) by power iteration from a seeded random start."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    v = torch.rand(P.shape, generator=g).to(P.device)[None]
    lam = 0.0
    for _ in range(iters):
        w = P.backproject(P.forward(v))
        lam = float(NN.dot(w, v)[0]) / float(NN.dot(v, v)[0])
        v = NN.scale(w, 1.0 / math.sqrt(float(NN.dot(w, w)[0])))
    return lam


def residual(y, Fr):
    """||y - F rho||^2 per object."""
    return NN.residual(y, Fr)


def gd(op, y, rho0, lam_max, iters=None, target=None, max_iters=10000, Fr0=None):
    """Plain gradient descent from rho0 (B objects).

    Runs `iters` iterations, or until each object's residual <= target[b]
    (then it stops updating; its calls stop counting).  Returns
    (rho, residual history list of (B,) tensors, iterations done per object).
    Each iteration costs one F^T and one F call per active object; the first
    residual costs one F call unless Fr0 (F rho0) is given.
    """
    rho = rho0.clone()
    B = rho.shape[0]
    Fr = op.F(rho) if Fr0 is None else Fr0
    diff = torch.empty_like(Fr)  # F rho - y, the adjoint's input
    res = NN.residual(y, Fr, diff=diff)
    hist = [res.clone()]
    done = torch.zeros(B, dtype=torch.bool, device=rho.device)
    if target is not None:
        done |= res <= target
    n_it = torch.zeros(B, dtype=torch.int64)
    k = 0
    while True:
        if iters is not None and k >= iters:
            break
        if iters is None and (bool(done.all()) or k >= max_iters):
            break
        active = ~done
        g = op.FT(diff, active)
        NN.axpy(rho, g, -1.0 / lam_max, active=active)
        Fr = op.F(rho, active)
        NN.residual(y, Fr, diff=diff, out=res, active=active)
        hist.append(res.clone())
        n_it += active.cpu().long()
        if target is not None:
            done |= res <= target
        k += 1
    return rho, hist, n_it, Fr


class DataTerm(torch.autograd.Function):
    """||F rho - y||^2 summed over objects; the gradient 2 F^T (F rho - y).
    Both run in the library's kernels (projector, residual, scaling)."""

    @staticmethod
    def forward(ctx, rho, proj, y):
        Fr = proj.forward(rho)
        res = NN.residual(y.reshape(1, -1), Fr.reshape(1, -1), diff=Fr.reshape(1, -1))
        ctx.proj = proj
        ctx.save_for_backward(Fr)  # now F rho - y
        return res[0]

    @staticmethod
    def backward(ctx, g):
        (d,) = ctx.saved_tensors
        x = ctx.proj.backproject(d)
        return NN.scale(x, 2.0 * float(g), out=x), None, None


def adam_tv(P, y, rho0, lam_tv=1e-3, lr=1e-2, steps=200, eps_tv=1e-6):
    """min ||y - F rho||^2 + lam_tv TV(rho) by Adam; returns (rho, losses)."""
    rho = rho0.clone()
    opt = Adam([rho], lr=lr)
    losses = []
    for _ in range(steps):
        r = rho.detach().requires_grad_(True)
        loss = DataTerm.apply(r, P, y) + lam_tv * TV.apply(r, eps_tv)
        loss.backward()
        opt.step([r.grad])
        losses.append(float(loss))
    return rho, losses
