"""GPU parity of rays that start inside the grid and of the attenuated
emission model (Sec. 9.3, Eqs. 14-18) against the CPU FP64 oracle
(oracle/projector.py with interior starts, oracle/atten.py).

Bars:
  - interior and sunward rays: the static parity bars (bit-exact index
    lists on non-tie rays, FP32 lengths, forward / adjoint within 1e-5 of the
    absolute integrand);
  - attenuated model (both backward methods; the deterministic one is
    also bitwise repeatable): the projection bar (1e-5 of the absolute integrand)
    carried through the model's arithmetic to first order.  A segment's
    term w[v] exp(-T) len has its optical depths tau_1[v] and T from FP32
    projections, each within 1e-5 of the same depth of |sigma rho|
    (tau_abs, T_abs); exp turns an absolute error d of a depth into a
    relative error d of the term.  So
      |y - y_ora| <= 1e-5 sum_k |w| exp(-T_k) len_k (1 + tau_abs[v_k] + T_abs,k) + 1e-7,
    and the gradient, a sum of products of the same factors with the
    upstream g, is within 1e-5 kappa of its terms' magnitudes,
    kappa = 1 + max tau_abs + max T_abs:
      |g - g_ora| <= 1e-5 kappa (exp(-tau_1) Gw + sigma (Gs + F_1^T(|w| Gw))) + 1e-9 max,
    Gw = sum |g_i| exp(-T_k) len_k, Gs = sum |g_i| len_k sum_{m >= k} |w| exp(-T_m) len_m
    (the oracle's gradient formula with every term taken in magnitude).
"""
import numpy as np
import pytest
import torch

from oracle import atten as A
from paper_2608_16960_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda", 0)


def _P():
    from paper_2608_16960_amd.projector import Projector
    return Projector


def test_interior_starts(ora, dev):
    """Explicit rays from random points inside the grid (in the hole, at the
    origin, on the polar axis too): full element-wise parity."""
    from test_gpu_parity import _check_all
    for g in (W.uniform_grid((8, 7, 9), r=(1.0, 6.0)),
              W.Grid(np.array([2.0, 2.7, 3.1, 4.4, 6.0]), np.array([0.3, 0.8, 1.5708, 2.9]),
                     np.array([-0.4, 0.3, 1.9, 3.0, 4.1]))):
        rng = np.random.default_rng(60)
        Ro = g.r_b[-1]
        u = rng.normal(size=(3000, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        p = u * Ro * rng.uniform(0, 1, (3000, 1)) ** (1 / 3)
        d = rng.normal(size=(3000, 3))
        p = np.concatenate([p, [[0, 0, 0], [0, 0, 0.5 * Ro], [0, 0, -0.3 * Ro]]])
        d = np.concatenate([d, [[0.3, 0.4, 0.5], [1.0, 0.2, -0.1], [-0.5, 0.1, 0.3]]])
        P = _P()(g, rays=(p, d))
        rho = rng.uniform(-0.5, 1.5, (1, *g.shape)).astype(np.float32)
        _check_all(ora, g, P, p, d, rho)


def test_sunward_geometry(ora, dev):
    """One ray per voxel centroid along the sun direction: rays and lists."""
    from test_gpu_parity import _check_all
    w = W.tiny()
    sun = np.array([0.3, -0.8, 0.5])
    P = _P()(w.grid, sun_dir=sun)
    assert P.out_shape == w.grid.shape
    c = A.centroids(w.grid.arrays())
    d = np.tile(sun / np.linalg.norm(sun), (len(c), 1))
    rho = np.random.default_rng(61).uniform(0, 1, (2, *w.grid.shape)).astype(np.float32)
    _check_all(ora, w.grid, P, c, d, rho)


def _bounds(ora, tr, trs, rho, sigma, g):
    """(per-ray forward bound, per-voxel gradient bound, kappa); see the
    module docstring."""
    V = rho.size
    rp = np.asarray(tr["row_ptr"])
    seg_ray = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    vox, ln = tr["vox"], tr["len"]
    s = sigma * rho
    tau1 = ora.forward(trs, s)
    tau_abs = ora.forward(trs, np.abs(s))
    e1 = np.exp(-tau1)
    wabs = np.abs(e1 * rho)
    E = np.exp(-A._row_cumsum(s[vox] * ln, rp))
    T_abs = A._row_cumsum(np.abs(s)[vox] * ln, rp)
    cabs = wabs[vox] * E * ln
    ybound = np.bincount(seg_ray, weights=cabs * (1.0 + tau_abs[vox] + T_abs),
                         minlength=len(rp) - 1)
    kappa = 1.0 + float(tau_abs.max()) + float(T_abs.max() if T_abs.size else 0.0)
    ga = np.abs(g)[seg_ray]
    cnt_rev = np.concatenate([[0], np.cumsum(np.diff(rp)[::-1])])
    suffix = A._row_cumsum(cabs[::-1], cnt_rev)[::-1]
    Gw = np.bincount(vox, weights=ga * E * ln, minlength=V)
    Gs = np.bincount(vox, weights=ga * ln * suffix, minlength=V)
    gbound = e1 * Gw + sigma * (Gs + ora.adjoint(trs, wabs * Gw, V))
    return ybound, gbound, kappa


def _model(P, grid, sun, seed):
    from paper_2608_16960_amd.atten import Attenuated
    sig = np.random.default_rng(seed).uniform(0.02, 0.3, grid.shape).astype(np.float32)
    return Attenuated(P, torch.from_numpy(sig), sun), sig


def _check_atten(ora, grid, P, starts, dirs, rho, sun, seed, sample=None):
    M, sig = _model(P, grid, sun, seed)
    dev = P.device
    rho_t = torch.from_numpy(rho).to(dev)
    y, tau = M.forward(rho_t, keep_tau=True)
    y = y.reshape(rho.shape[0], -1).cpu().numpy().astype(np.float64)
    if sample is not None:
        y = y[:, sample]
    tr = ora.trace(grid.arrays(), starts, dirs)
    trs = A.sun_trace(grid.arrays(), sun)
    gy = np.random.default_rng(seed + 1).normal(size=y.shape).astype(np.float32)
    for b in range(rho.shape[0]):
        r64, s64 = rho[b].reshape(-1).astype(np.float64), sig.reshape(-1).astype(np.float64)
        yo = A.forward(tr, trs, r64, s64)
        ybound, _, _ = _bounds(ora, tr, trs, r64, s64, np.zeros(len(yo)))
        err = np.abs(y[b] - yo)
        assert np.all(err <= 1e-5 * ybound + 1e-7), (b, float(np.max(err / (ybound + 1e-7))))
    if sample is not None:
        return
    gyt = torch.from_numpy(gy).to(dev).reshape(rho.shape[0], *P.out_shape)
    for method in ("deterministic", "atomic"):
        grad = M.backward(rho_t, tau, gyt, method).reshape(rho.shape[0], -1).cpu().numpy()
        for b in range(rho.shape[0]):
            r64, s64 = rho[b].reshape(-1).astype(np.float64), sig.reshape(-1).astype(np.float64)
            go = A.gradient(tr, trs, r64, s64, gy[b].astype(np.float64))
            _, gbound, kappa = _bounds(ora, tr, trs, r64, s64, gy[b].astype(np.float64))
            err = np.abs(grad[b] - go)
            tol = 1e-5 * kappa * gbound + 1e-9 * gbound.max()
            assert np.all(err <= tol), (method, b, float(np.max(err / (kappa * gbound + 1e-30))))
    # the deterministic backward repeats bit for bit, and the autograd
    # wrapper runs it
    g1 = M.backward(rho_t, tau, gyt, "deterministic")
    assert torch.equal(g1, M.backward(rho_t, tau, gyt, "deterministic"))
    from paper_2608_16960_amd.atten import AttenuatedFn
    r = rho_t.clone().requires_grad_(True)
    (AttenuatedFn.apply(r, M) * gyt).sum().backward()
    assert torch.equal(r.grad, g1)


def test_attenuated_tiny(ora, dev):
    w = W.tiny()
    v = w.views
    P = _P()(w.grid, views=v)
    s, d = ora.cone_rays(v.pos, v.look, v.up, v.fov_deg, v.H, v.W)
    rho = np.concatenate([np.abs(w.rho), np.random.default_rng(62).uniform(
        0, 2, (1, *w.grid.shape))]).astype(np.float32)
    _check_atten(ora, w.grid, P, s, d, rho, np.array([0.6, -0.3, 0.74]), 63)


def test_attenuated_ragged_wedge(ora, dev):
    g = W.Grid(np.array([2.0, 2.7, 3.1, 4.4, 6.0, 9.5]), np.array([0.3, 0.8, 1.2, 1.5708, 2.0, 2.9]),
               np.array([-0.4, 0.3, 1.0, 1.9, 2.2, 3.0, 4.1]))
    pos = np.array([[20.0, 3.0, 5.0], [-4.0, 18.0, -7.0]])
    v = W.views_at(pos, (45.0, 38.0), 37, 29, look=[0.5, -0.2, 0.1])
    s, d = ora.cone_rays(v.pos, v.look, v.up, v.fov_deg, v.H, v.W)
    P = _P()(g, views=v)
    rho = np.random.default_rng(64).uniform(0, 1.5, (1, *g.shape)).astype(np.float32)
    _check_atten(ora, g, P, s, d, rho, np.array([-0.2, 0.9, 0.1]), 65)


def test_attenuated_medium_grid_three_views(ora, dev):
    """Medium grid and detector (50^3, 256x256), three of its views: every
    ray's attenuated measurement and the whole gradient against the oracle."""
    w = W.medium()
    v = w.views
    sel = [0, 10, 20]
    vv = W.views_at(v.pos[sel], v.fov_deg[0], v.H, v.W)
    P = _P()(w.grid, views=vv)
    s, d = ora.cone_rays(vv.pos, vv.look, vv.up, vv.fov_deg, vv.H, vv.W)
    rho = w.rho.astype(np.float32)
    _check_atten(ora, w.grid, P, s, d, rho, np.array([0.0, 1.0, 0.0]), 66)
