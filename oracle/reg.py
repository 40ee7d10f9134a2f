"""FP64 references for the regulariser and optimiser of differentiable
reconstruction (test infrastructure only).

tv_value_grad: anisotropic smoothed total variation on a (D0, D1, D2) grid,
    TV = sum_v sum_d sqrt((D_d rho)_v^2 + eps^2) with forward differences,
    none past the last index along the first two axes, circular along the
    third (azimuth), and its exact gradient (chain rule on every term).
adam_step: one Adam update (Kingma & Ba, with L2 weight decay added to the
    gradient as PyTorch's Adam does; the paper's reconstruction example uses
    that optimiser, TomoSphero Listing 7).
"""
import numpy as np


def _diffs(rho):
    dr = rho[..., 1:, :, :] - rho[..., :-1, :, :]
    de = rho[..., :, 1:, :] - rho[..., :, :-1, :]
    da = np.roll(rho, -1, axis=-1) - rho
    return dr, de, da


def tv_value_grad(rho, eps):
    rho = np.asarray(rho, np.float64)
    dr, de, da = _diffs(rho)
    tr, te, ta = (np.sqrt(d * d + eps * eps) for d in (dr, de, da))
    axes = tuple(range(rho.ndim - 3, rho.ndim))
    val = tr.sum(axis=axes) + te.sum(axis=axes) + ta.sum(axis=axes)
    g = np.zeros_like(rho)
    qr, qe, qa = dr / tr, de / te, da / ta
    # d/d rho of sqrt((rho[i+1] - rho[i])^2 + eps^2): -q at i, +q at i+1
    g[..., :-1, :, :] -= qr
    g[..., 1:, :, :] += qr
    g[..., :, :-1, :] -= qe
    g[..., :, 1:, :] += qe
    g -= qa
    g += np.roll(qa, 1, axis=-1)
    return val, g


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    g = g + weight_decay * p
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
