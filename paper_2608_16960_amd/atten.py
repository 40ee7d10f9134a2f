"""Attenuated emission model (TomoSphero Sec. 9.3, Eqs. 14-18) on the GPU.

    A = Attenuated(P, sigma, sun_dir)      # P: line-of-sight Projector (csr mode)
    y = A.forward(rho)                     # y = sum_k (exp(-tau1) rho)[v_k] exp(-T_k) len_k
    y = AttenuatedFn.apply(rho, A)         # differentiable in rho

tau1 = F_sun(sigma rho) along one sunward ray per voxel centroid; T is the
inclusive running sum of sigma rho len along each line of sight from the
detector.  Every step runs in libtsp (tsp_atten_forward / tsp_atten_backward);
this module only marshals tensors.
"""
import numpy as np
import torch

from . import native as N
from .projector import Projector


class Attenuated:
    """P: line-of-sight Projector traced in csr mode (static object);
    sigma: (Nr, Ne, Na) cross sections; sun_dir: 3 floats towards the Sun."""

    def __init__(self, P, sigma, sun_dir, sun_csc=True):
        if P.mode != "csr":
            raise ValueError("the attenuated model needs the line-of-sight projector in csr mode")
        self.P = P
        self.device = P.device
        self.sun = Projector(P._keep, sun_dir=sun_dir, csc=sun_csc, device=P.device)
        self.sigma = self._f32(torch.as_tensor(sigma, dtype=torch.float32).to(P.device),
                               "sigma")
        if tuple(self.sigma.shape) != P.shape:
            raise ValueError(f"sigma must have shape {P.shape}")

    def _f32(self, t, name):
        return self.P._dev_f32(t, name)

    def _lead(self, rho):
        rho = self._f32(rho, "rho")
        if tuple(rho.shape[-3:]) != self.P.shape:
            raise ValueError(f"rho must end in {self.P.shape}, got {tuple(rho.shape)}")
        lead = rho.shape[:-3]
        return rho, lead, int(np.prod(lead)) if lead else 1

    def forward(self, rho, keep_tau=False):
        """y (..., *out_shape); with keep_tau also tau1 (..., Nr, Ne, Na)."""
        rho, lead, B = self._lead(rho)
        y = torch.empty((*lead, *self.P.out_shape), dtype=torch.float32, device=self.device)
        tau = torch.empty_like(rho) if keep_tau else None
        N.check(N.lib.tsp_atten_forward(self.P._h, self.sun._h, N.ptr(rho), N.ptr(self.sigma), B,
                                        N.ptr(y), N.ptr(tau) if keep_tau else None,
                                        N.stream_handle()))
        return (y, tau) if keep_tau else y

    def backward(self, rho, tau, gy, method=None):
        """d<gy, y>/d rho for the rho whose forward produced tau.  method:
        "deterministic" (exact fixed-point sums, bitwise reproducible; needs
        the sunward geometry's voxel-major store), "atomic", or None: the
        deterministic one when the sunward geometry has its store."""
        rho, lead, B = self._lead(rho)
        tau = self._f32(tau, "tau")
        gy = self._f32(gy, "gy")
        if method is None:
            method = "deterministic" if self.sun.csc else "atomic"
        m = {"deterministic": N.TSP_ADJ_DETERMINISTIC, "atomic": N.TSP_ADJ_ATOMIC}[method]
        grad = torch.empty_like(rho)
        N.check(N.lib.tsp_atten_backward(self.P._h, self.sun._h, N.ptr(rho), N.ptr(self.sigma),
                                         N.ptr(tau), N.ptr(gy), B, N.ptr(grad), m,
                                         N.stream_handle()))
        return grad

    __call__ = forward


class AttenuatedFn(torch.autograd.Function):
    """Differentiable attenuated forward; the backward is the hand-written
    tsp_atten_backward (autograd never sees the tracer)."""

    @staticmethod
    def forward(ctx, rho, model):
        y, tau = model.forward(rho.detach(), keep_tau=True)
        ctx.model = model
        ctx.save_for_backward(rho.detach(), tau)
        return y

    @staticmethod
    def backward(ctx, gy):
        rho, tau = ctx.saved_tensors
        return ctx.model.backward(rho, tau, gy.contiguous()), None
