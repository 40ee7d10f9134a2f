"""Iterative reconstruction on top of the projector (TomoSphero Sec. 4.5).

- power_iteration: largest eigenvalue of F^T F (for a safe gradient step);
- CountingOperator: forwards F / F^T and counts calls per object;
- gd: plain gradient descent on ||y - F rho||^2 (Eq. 6) with step
  eta = 1 / (2 lambda_max), rho <- rho - eta * 2 F^T (F rho - y), stopping
  per object when its residual reaches a target;
- adam_tv: ||y - F rho||^2 + lambda TV(rho) minimised with Adam (Listing 7),
  gradients from ProjectorFn / TV (hand-written kernels, no autograd tracing
  of the ray tracer).
Batched: every function works on a batch of objects at once (the projector
kernels take batches natively).
"""
import torch

from .nn import TV, Adam
from .projector import ProjectorFn


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
        lam = float((w * v).sum() / (v * v).sum())
        v = w / w.norm()
    return lam


def residual(y, Fr):
    """||y - F rho||^2 per object."""
    return ((y - Fr) ** 2).flatten(1).sum(1)


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
    res = residual(y, Fr)
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
        g = op.FT(Fr - y, active)
        step = (g / lam_max) * active.float().reshape(B, *([1] * (rho.dim() - 1)))
        rho = rho - step
        Fr = op.F(rho, active)
        res = torch.where(active, residual(y, Fr), res)
        hist.append(res.clone())
        n_it += active.cpu().long()
        if target is not None:
            done |= res <= target
        k += 1
    return rho, hist, n_it, Fr


def adam_tv(P, y, rho0, lam_tv=1e-3, lr=1e-2, steps=200, eps_tv=1e-6):
    """min ||y - F rho||^2 + lam_tv TV(rho) by Adam; returns (rho, losses)."""
    rho = rho0.clone()
    opt = Adam([rho], lr=lr)
    losses = []
    for _ in range(steps):
        r = rho.detach().requires_grad_(True)
        loss = ((ProjectorFn.apply(r, P) - y) ** 2).sum() + lam_tv * TV.apply(r, eps_tv)
        loss.backward()
        opt.step([r.grad])
        losses.append(float(loss))
    return rho, losses
