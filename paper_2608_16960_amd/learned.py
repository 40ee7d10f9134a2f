"""Learned warm start for iterative reconstruction.

A small 3-D CNN on the (r, e, a) grid (nn.CNN) maps a few-iteration plain
gradient-descent reconstruction x_in to a starting point for the same plain
gradient descent.  The plain solve stays the arbiter: the CNN output is used
only if its data residual ||y - F rho||^2 is below that of x_in (fallback),
and the solve then runs until it reaches the residual R* that plain GD
reaches after K iterations from zero.  Every projector call is counted,
including the calls that build x_in.

Training data: phantoms (exponential background with a random scale plus
1-8 Gaussian plumes), projections made by this projector, x_in from k0 plain
GD iterations; loss ||CNN(s x_in) - rho_true||^2 (mean over voxels), Adam on
FP32 master weights, BF16 MFMA kernels for the hidden layers.
"""
import numpy as np
import torch

from . import nn as NN
from . import solvers
from .nn import CNN, Adam


class WarmStart:
    def __init__(self, P, k0=2, K=60, power_iters=20, seed=8):
        self.P = P
        self.k0 = k0
        self.K = K
        self.op = solvers.CountingOperator(P)
        self.lam = solvers.power_iteration(P, power_iters)  # shared setup, not counted
        self.net = CNN(device=P.device, seed=seed)
        self.scale = 1.0

    # ------------------------------------------------------------ data
    def measure(self, rho):
        return self.P.forward(rho)

    def inputs(self, y):
        """x_in = k0 plain GD iterations from zero: 2 k0 calls per object
        (F of zero is zero).  Returns (x_in, its residual, F x_in)."""
        B = y.shape[0]
        z = torch.zeros((B, *self.P.shape), device=y.device)
        x, hist, _, Fx = solvers.gd(self.op, y, z, self.lam, iters=self.k0,
                                    Fr0=torch.zeros_like(y))
        return x, hist[-1], Fx

    # ------------------------------------------------------------ training
    def fit(self, x_in, truth, epochs=20, batch=8, lr=2e-3, seed=0, log=None):
        """Train on (x_in, truth) stacks already on the GPU; returns the loss per epoch."""
        n = x_in.shape[0]
        self.scale = float(truth.abs().mean() / x_in.abs().mean().clamp_min(1e-12))
        opt = Adam(self.net.parameters(), lr=lr)
        g = torch.Generator().manual_seed(seed)
        hist = []
        nvox = float(np.prod(x_in.shape[1:]))
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g)
            tot = 0.0
            for b0 in range(0, n - batch + 1, batch):
                idx = perm[b0:b0 + batch].to(x_in.device)
                xb = x_in[idx]
                NN.scale(xb, self.scale, out=xb)
                tb = truth[idx]
                out = self.net.forward(xb)
                res = NN.residual(tb, out, diff=out)  # out now holds out - tb
                grads = self.net.backward(NN.scale(out, 2.0 / (batch * nvox), out=out))
                opt.step(grads, bf16_copies=self.net.bf16_targets())
                tot += float(res.cpu().double().sum()) / nvox
            hist.append(tot / (n - n % batch))
            if log:
                log(f"epoch {ep}: mse {hist[-1]:.4e}")
        return hist

    def predict(self, x_in):
        return self.net.forward(NN.scale(x_in, self.scale), keep=False)

    # ------------------------------------------------------------ evaluation
    def evaluate(self, truth, batch=8, curves=False, curve_iters=20):
        """Per object: plain calls to R* (= 2K by definition), warm-start calls
        to R*, whether the fallback was taken, and the residuals of the CNN
        output and of x_in.  With curves=True also the residual-vs-calls
        curves, as medians over the objects of residual / R*: plain GD from
        zero after 2k calls (k = 0 .. K), and the warm start after 5 + 2k
        calls (k = 0 .. curve_iters; the GD run for the curve is separate
        from the counted solve and not counted)."""
        out = {"plain_calls": [], "warm_calls": [], "fallback": [], "R_star": [],
               "warm_res0": [], "xin_res": []}
        plain_rel, warm_rel = [], []
        for b0 in range(0, truth.shape[0], batch):
            t = truth[b0:b0 + batch]
            B = t.shape[0]
            y = self.measure(t)
            z = torch.zeros_like(t)
            # plain GD: K iterations from zero define R*
            self.op.reset(B)
            _, hist, _, _ = solvers.gd(self.op, y, z, self.lam, iters=self.K,
                                       Fr0=torch.zeros_like(y))
            plain_calls = self.op.calls.clone()
            r_star = hist[-1]
            # warm start: x_in (2 k0 calls), CNN, its residual (1 call), fallback, GD to R*
            self.op.reset(B)
            x_in, res_in, F_in = self.inputs(y)
            x0 = self.predict(x_in)
            F0 = self.op.F(x0)
            res0 = solvers.residual(y, F0)
            use_net = res0 <= res_in
            start = torch.where(use_net.reshape(B, 1, 1, 1), x0, x_in)
            Fstart = torch.where(use_net.reshape(B, *([1] * (F0.dim() - 1))), F0, F_in)
            solvers.gd(self.op, y, start, self.lam, target=r_star, max_iters=4 * self.K,
                       Fr0=Fstart)
            if curves:
                rs = r_star.clamp_min(1e-30)
                plain_rel.append(torch.stack([h / rs for h in hist]).cpu())
                free = solvers.CountingOperator(self.P)
                _, wh, _, _ = solvers.gd(free, y, start, self.lam, iters=curve_iters, Fr0=Fstart)
                warm_rel.append(torch.stack([h / rs for h in wh]).cpu())
            out["plain_calls"] += plain_calls.tolist()
            out["warm_calls"] += self.op.calls.tolist()
            out["fallback"] += (~use_net).cpu().tolist()
            out["R_star"] += r_star.cpu().tolist()
            out["warm_res0"] += res0.cpu().tolist()
            out["xin_res"] += res_in.cpu().tolist()
        if curves:
            pm = torch.cat(plain_rel, 1).double().median(1).values
            wm = torch.cat(warm_rel, 1).double().median(1).values
            out["curves"] = {
                "plain": [[2 * k, float(pm[k])] for k in range(len(pm))],
                "warm": [[2 * self.k0 + 1 + 2 * k, float(wm[k])] for k in range(len(wm))],
                "y": "median residual / R*"}
        return out
