"""Pins of the FP64 references for TV, Adam and the grid convolution."""
import numpy as np
import torch

from oracle import conv as OC
from oracle import reg as OR


def test_tv_of_linear_ramp_closed_form():
    """rho = s * i along r: every r-difference is s, e-differences 0, azimuth
    differences 0: TV = (D0-1) D1 D2 sqrt(s^2+eps^2) + (D0 (D1-1) D2 + D0 D1 D2) eps."""
    D0, D1, D2, s, eps = 5, 4, 6, 0.7, 1e-3
    rho = s * np.arange(D0)[:, None, None] * np.ones((D0, D1, D2))
    val, _ = OR.tv_value_grad(rho, eps)
    ref = (D0 - 1) * D1 * D2 * np.sqrt(s * s + eps * eps) + (D0 * (D1 - 1) * D2 + D0 * D1 * D2) * eps
    assert abs(val - ref) < 1e-12


def test_tv_azimuth_is_circular():
    """A ramp along azimuth wraps: the last difference is -(D2-1) s."""
    D0, D1, D2, s, eps = 2, 3, 5, 0.3, 1e-4
    rho = s * np.arange(D2)[None, None, :] * np.ones((D0, D1, D2))
    val, _ = OR.tv_value_grad(rho, eps)
    per_row = (D2 - 1) * np.sqrt(s * s + eps * eps) + np.sqrt(((D2 - 1) * s) ** 2 + eps * eps)
    ref = D0 * D1 * per_row + ((D0 - 1) * D1 * D2 + D0 * (D1 - 1) * D2) * eps
    assert abs(val - ref) < 1e-12


def test_tv_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    rho = rng.normal(size=(4, 3, 5))
    eps = 0.05
    _, g = OR.tv_value_grad(rho, eps)
    h = 1e-6
    for idx in [(0, 0, 0), (3, 2, 4), (1, 1, 2), (2, 0, 4)]:
        e = np.zeros_like(rho)
        e[idx] = h
        fd = (OR.tv_value_grad(rho + e, eps)[0] - OR.tv_value_grad(rho - e, eps)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-7


def test_adam_matches_torch_optimizer():
    rng = np.random.default_rng(1)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(5)]
    pt = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=0.01, betas=(0.9, 0.99), eps=1e-7, weight_decay=0.3)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, start=1):
        pt.grad = torch.tensor(g)
        opt.step()
        p, m, v = OR.adam_step(p, g, m, v, t, 0.01, 0.9, 0.99, 1e-7, 0.3)
    assert np.allclose(p, pt.detach().numpy(), rtol=0, atol=1e-12)


def test_conv_library_step_equals_direct_loops():
    """PyTorch conv3d + circular pad equals the layer's definition by loops."""
    g = torch.Generator().manual_seed(3)
    x = torch.randn((2, 3, 2, 5, 4), generator=g, dtype=torch.float64)
    w = torch.randn((27, 6, 4), generator=g, dtype=torch.float64)
    b = torch.randn(6, generator=g, dtype=torch.float64)
    assert torch.allclose(OC.conv(x, w, b), OC.conv_direct(x, w, b), atol=1e-12)


def test_conv_tap_orientation():
    """A single tap (dr, de, da) = (1, 0, -1) picks x[i+1, j, k-1 mod D2]."""
    x = torch.zeros((1, 3, 2, 4, 1), dtype=torch.float64)
    x[0, 2, 1, 3, 0] = 1.0
    w = torch.zeros((27, 1, 1), dtype=torch.float64)
    w[(1 + 1) * 9 + (0 + 1) * 3 + (-1 + 1), 0, 0] = 1.0
    y = OC.conv(x, w)
    # output at (i, j, k) = x[i+1, j, k-1]: nonzero at i=1, j=1, k=0 (k-1 = -1 -> 3)
    nz = torch.nonzero(y[..., 0])
    assert nz.tolist() == [[0, 1, 1, 0]]
