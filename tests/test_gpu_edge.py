"""Edge cases of the projector: geometries whose rays all miss the grid (no
segments at all: empty stores, empty transposed lists, empty chunks) and a
geometry of one ray.

Bars: with no segments every projection and every adjoint voxel is exactly 0
in every mode and method, and the exported lists are empty; the one-ray
geometry meets the static parity bars against the oracle (projection and
adjoint within 1e-5 of the absolute integrand, + 1e-7), and its chunked
deterministic adjoint equals the stored one bit for bit.
"""
import numpy as np
import pytest
import torch

from paper_2608_16960_amd import workloads as W

pytestmark = pytest.mark.gpu


def _P():
    from paper_2608_16960_amd.projector import Projector
    return Projector


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda", 0)


def _missing_geometries(mode):
    w = W.tiny()
    # cone views outside the grid looking away from it (narrow field)
    pos = np.array([[50.0, 0.0, 0.0], [0.0, -40.0, 10.0]])
    cv = W.views_at(pos, (10.0, 10.0), 19, 23, look=pos * 2.0)
    yield w.grid, _P()(w.grid, views=cv, mode=mode)
    # explicit rays passing beside the grid (r_max = 25)
    rng = np.random.default_rng(50)
    s = rng.uniform(-5, 5, (300, 3)) + np.array([0.0, 0.0, 60.0])
    d = np.tile([1.0, 0.0, 0.0], (300, 1)) + rng.normal(0, 0.01, (300, 3))
    yield w.grid, _P()(w.grid, rays=(s, d), mode=mode)


@pytest.mark.parametrize("mode", ["csr", "onthefly"])
def test_all_rays_miss(dev, mode):
    for grid, P in _missing_geometries(mode):
        inf = P.info()
        assert inf["n_segments"] == 0
        rho = torch.rand((3, *grid.shape), device=dev)
        y = P.forward(rho)
        assert y.shape == (3, *P.out_shape) and torch.count_nonzero(y) == 0
        yy = torch.randn((3, *P.out_shape), device=dev)
        for m in ("deterministic", "atomic"):
            x = P.backproject(yy, m)
            assert x.shape == (3, *grid.shape) and torch.count_nonzero(x) == 0, m
        if mode == "csr":
            rp, vox, ln = P.segments()
            assert torch.count_nonzero(rp) == 0 and vox.numel() == 0 and ln.numel() == 0


def test_one_ray(ora, dev):
    """One explicit ray through the Tiny grid, off the origin: forward and
    adjoint against the oracle in both modes; every adjoint method agrees."""
    w = W.tiny()
    s = np.array([[40.0, 3.0, -2.0]])
    d = np.array([[-1.0, -0.05, 0.07]])
    tr = ora.trace(w.grid.arrays(), s, d)
    assert tr["counts"][0] > 10
    rho = np.random.default_rng(51).uniform(0, 1, (2, w.grid.size)).astype(np.float32)
    yo = ora.forward(tr, rho.astype(np.float64))
    yy = np.array([[1.5], [-0.75]], np.float32)
    xo = ora.adjoint(tr, yy.astype(np.float64), w.grid.size)
    seg = np.repeat(np.arange(1), tr["counts"])
    xs = {}
    for mode in ("csr", "onthefly"):
        P = _P()(w.grid, rays=(s, d), mode=mode)
        y = P.forward(torch.from_numpy(rho).reshape(2, *w.grid.shape).to(dev))
        y = y.reshape(2).cpu().numpy().astype(np.float64)
        for b in range(2):
            tol = 1e-5 * np.sum(np.abs(rho[b][tr["vox"]]) * tr["len"]) + 1e-7
            assert abs(y[b] - yo[b, 0]) <= tol, (mode, b)
        y_t = torch.from_numpy(yy).to(dev)
        for m in ("deterministic", "atomic"):
            x = P.backproject(y_t, m)
            xs[mode, m] = x
            xg = x.reshape(2, -1).cpu().numpy().astype(np.float64)
            for b in range(2):
                tol = np.zeros(w.grid.size)
                np.add.at(tol, tr["vox"], np.abs(yy[b][seg]) * tr["len"])
                assert np.all(np.abs(xg[b] - xo[b]) <= 1e-5 * tol + 1e-7), (mode, m, b)
    assert torch.equal(xs["onthefly", "deterministic"], xs["csr", "deterministic"])
