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


def _half_quantum(yb, R, r_out):
    M = max(float(np.abs(np.float32(yb)).max()), 1e-30) * 4.0 * R * r_out
    return 2.0 ** (int(np.frexp(M)[1]) - 1 + 1 - 62 - 1)


def test_finest_boundary_tables(ora, dev):
    """A grid at the boundary-table limit (nr + ne + 3 na = 5620 of 5627,
    45 KB of FP64 tables): the on-the-fly adjoints' workgroups then need
    more than 64 KiB of LDS, which their launches request.  600 explicit
    rays, on the fly: forward, atomic and fixed-point adjoints at batch 1
    and 4 against the oracle, at the static bars (1e-5 of the absolute
    integrand + 1e-7; fixed point 2e-7 of it plus one float rounding plus
    half a quantum per term, 2^(q-1) with q = ilogb(max|y| 4 R r_out) + 1 - 62)."""
    g = W.uniform_grid((20, 20, 1860), r=(1.0, 5.0))
    s, d = W.random_rays(600, np.random.default_rng(52), r_start=(8.0, 12.0), aim=3.0)
    tr = ora.trace(g.arrays(), s, d)
    R, V = len(s), g.size
    assert tr["counts"].sum() > 50_000
    seg = np.repeat(np.arange(R), tr["counts"])
    nterms = np.bincount(tr["vox"], minlength=V)
    P = _P()(g, rays=(s, d), mode="onthefly")
    rng = np.random.default_rng(53)
    for B in (1, 4):
        rho = rng.uniform(0, 1, (B, V)).astype(np.float32)
        yo = ora.forward(tr, rho.astype(np.float64))
        y = P.forward(torch.from_numpy(rho).reshape(B, *g.shape).to(dev))
        y = y.reshape(B, R).cpu().numpy().astype(np.float64)
        for b in range(B):
            tol = np.zeros(R)
            np.add.at(tol, seg, np.abs(rho[b][tr["vox"]]) * tr["len"])
            assert np.all(np.abs(y[b] - yo[b]) <= 1e-5 * tol + 1e-7), (B, b)
        yy = rng.normal(size=(B, R)).astype(np.float32)
        xo = ora.adjoint(tr, yy.astype(np.float64), V)
        y_t = torch.from_numpy(yy).to(dev)
        for m in ("atomic", "fixedpoint"):
            xg = P.backproject(y_t, m).reshape(B, V).cpu().numpy().astype(np.float64)
            for b in range(B):
                absx = np.zeros(V)
                np.add.at(absx, tr["vox"], np.abs(yy[b][seg]) * tr["len"])
                tol = (1e-5 * absx + 1e-7 if m == "atomic"
                       else 2e-7 * absx + 2.0 ** -24 * np.abs(xo[b]) + 1e-30
                       + nterms * _half_quantum(yy[b], R, float(g.r_b[-1])))
                assert np.all(np.abs(xg[b] - xo[b]) <= tol), (B, m, b)
    P.close()


def test_four_objects_past_2p32_elements(ora, dev):
    """1500 x 1500 x 500 voxels (1.125e9): four objects voxel-major hold
    4.5e9 floats and the fixed-point sums 4.5e9 words, more than one dispatch
    has work-items, so the staging, clearing and conversion kernels stride
    over capped grids.  300 explicit rays on the fly, batch 4: forward,
    atomic and fixed-point adjoints against the oracle at the static bars,
    on the traced voxels (the oracle runs on the voxels the rays reach,
    renumbered), and every other voxel exactly 0.  With 1500 shells and 1500
    cones many segments are very short, so the fixed-point bar also carries
    each length's FP64 root error, at the walker's length bars (1e-10 r_max,
    1e-7 r_max on rays the oracle marks length-sensitive) times |y|."""
    g = W.uniform_grid((1500, 1500, 500), r=(1.0, 5.0))
    V, B = g.size, 4
    assert 4 * V > 2 ** 32
    s, d = W.random_rays(300, np.random.default_rng(54), r_start=(8.0, 12.0), aim=3.0)
    tr = ora.trace(g.arrays(), s, d)
    R = len(s)
    uv, inv = np.unique(tr["vox"], return_inverse=True)
    trc = dict(tr, vox=inv.astype(np.int32))  # the same lists on the reached voxels only
    seg = np.repeat(np.arange(R), tr["counts"])
    P = _P()(g, rays=(s, d), mode="onthefly")
    gen = torch.Generator(device=dev).manual_seed(55)
    rho = torch.rand((B, *g.shape), device=dev, generator=gen)
    idx = torch.from_numpy(uv.astype(np.int64)).to(dev)
    rho_c = rho.reshape(B, V)[:, idx].cpu().numpy().astype(np.float64)
    y = P.forward(rho).reshape(B, R).cpu().numpy().astype(np.float64)
    yo = ora.forward(trc, rho_c)
    for b in range(B):
        tol = np.zeros(R)
        np.add.at(tol, seg, np.abs(rho_c[b][inv]) * tr["len"])
        assert np.all(np.abs(y[b] - yo[b]) <= 1e-5 * tol + 1e-7), b
    del rho
    yy = np.random.default_rng(56).normal(size=(B, R)).astype(np.float32)
    xo = ora.adjoint(trc, yy.astype(np.float64), len(uv))
    nterms = np.bincount(inv, minlength=len(uv))
    dl = np.where(tr["sensitive"][seg], 1e-7, 1e-10) * float(g.r_b[-1])
    for m in ("atomic", "fixedpoint"):
        x = P.backproject(torch.from_numpy(yy).to(dev), m).reshape(B, V)
        assert int(torch.count_nonzero(x)) <= B * len(uv), m
        xg = x[:, idx].cpu().numpy().astype(np.float64)
        del x
        for b in range(B):
            absx, lerr = np.zeros(len(uv)), np.zeros(len(uv))
            np.add.at(absx, inv, np.abs(yy[b][seg]) * tr["len"])
            np.add.at(lerr, inv, np.abs(yy[b][seg]) * dl)
            tol = (1e-5 * absx + 1e-7 if m == "atomic"
                   else 2e-7 * absx + 2.0 ** -24 * np.abs(xo[b]) + lerr + 1e-30
                   + nterms * _half_quantum(yy[b], R, float(g.r_b[-1])))
            err = np.abs(xg[b] - xo[b])
            k = int(np.argmax(err - tol))
            assert np.all(err <= tol), (m, b, k, xg[b][k], xo[b][k], absx[k], lerr[k], nterms[k])
    P.close()
