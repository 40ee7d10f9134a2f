"""Deterministic adjoint of geometries without a stored voxel-major list (on
the fly, or stored lists traced without it): traced chunk by chunk within the
call, each chunk's lists transposed and packed, the chunks added in order.

Bars: as the static parity tests (tests/test_gpu_parity.py): each adjoint
voxel within 1e-5 of the oracle's sum of |y| len (+1e-7).  The result is
bitwise repeatable, every object of a batch equals its adjoint alone bit for
bit, and with one chunk it equals the stored deterministic adjoint bit for
bit.  TSP_CHUNK_SEGMENTS forces several chunks on these small geometries.
"""
import contextlib
import os

import numpy as np
import pytest
import torch

from oracle import dynamic as D
from oracle.views import parallel_rays
from paper_2608_16960_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-5


def _P():
    from paper_2608_16960_amd.projector import Projector
    return Projector


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda", 0)


@contextlib.contextmanager
def chunk_segments(n):
    old = os.environ.get("TSP_CHUNK_SEGMENTS")
    if n is not None:
        os.environ["TSP_CHUNK_SEGMENTS"] = str(int(n))
    try:
        yield
    finally:
        if old is None:
            os.environ.pop("TSP_CHUNK_SEGMENTS", None)
        else:
            os.environ["TSP_CHUNK_SEGMENTS"] = old


def _abs_adjoint(tr, y, V):
    out = np.zeros(V)
    seg_ray = np.repeat(np.arange(len(tr["counts"])), tr["counts"])
    np.add.at(out, tr["vox"], np.abs(y[seg_ray]) * tr["len"])
    return out


def _check(ora, grid, P, s, d, B, seed):
    """Chunked deterministic adjoint of a batch vs the oracle; repeatable;
    each object equal to its adjoint alone."""
    tr = ora.trace(grid.arrays(), s, d)
    R, V = len(tr["counts"]), grid.size
    yy = np.random.default_rng(seed).normal(size=(B, R)).astype(np.float32)
    y_t = torch.from_numpy(yy).cuda().reshape(B, *P.out_shape)
    x = P.backproject(y_t, "deterministic")
    assert torch.equal(x, P.backproject(y_t, "deterministic"))
    for b in range(B):
        assert torch.equal(x[b:b + 1], P.backproject(y_t[b:b + 1], "deterministic")), b
    xo = ora.adjoint(tr, yy.astype(np.float64), V)
    xg = x.reshape(B, V).cpu().numpy().astype(np.float64)
    for b in range(B):
        tol = RTOL * _abs_adjoint(tr, yy[b].astype(np.float64), V) + 1e-7
        err = np.abs(xg[b] - xo[b])
        assert np.all(err <= tol), f"b={b}: worst voxel {np.argmax(err - tol)}"


@pytest.mark.parametrize("mode", ["onthefly", "csr_without_csc"])
@pytest.mark.parametrize("chunks", [1, 4])
def test_tiny(ora, dev, mode, chunks):
    """Tiny (4 views 32x32), batch 3, in one chunk or one view per chunk."""
    w = W.tiny()
    v = w.views
    s, d = ora.cone_rays(v.pos, v.look, v.up, v.fov_deg, v.H, v.W)
    P = _P()(w.grid, views=v, mode="onthefly" if mode == "onthefly" else "csr", csc=False)
    S = P.info()["n_segments"]
    with chunk_segments(None if chunks == 1 else (S + chunks - 1) // chunks):
        _check(ora, w.grid, P, s, d, 3, 40 + chunks)


def test_one_chunk_equals_stored(dev):
    """One chunk traces exactly the stored geometry: same lists, same sums."""
    w = W.tiny()
    Ps = _P()(w.grid, views=w.views)
    Po = _P()(w.grid, views=w.views, mode="onthefly")
    Pn = _P()(w.grid, views=w.views, csc=False)
    y = torch.from_numpy(np.random.default_rng(44).normal(size=(2, *Ps.out_shape))
                         .astype(np.float32)).to(dev)
    xs = Ps.backproject(y, "deterministic")
    assert torch.equal(Po.backproject(y, "deterministic"), xs)
    assert torch.equal(Pn.backproject(y, "deterministic"), xs)
    # the defaults: stored deterministic with the voxel-major store, else atomic
    assert torch.equal(Ps.backproject(y), xs)
    xa = Po.backproject(y)
    assert torch.allclose(xa, xs, rtol=1e-5, atol=1e-5)


def test_explicit_rays_in_chunks(ora, dev):
    """1500 explicit rays (5.9 windows of 256) on a ragged wedge grid, cut
    into runs of whole windows."""
    g = W.Grid(np.array([2.0, 2.7, 3.1, 4.4, 6.0, 9.5]), np.array([0.3, 0.8, 1.2, 1.5708, 2.0, 2.9]),
               np.array([-0.4, 0.3, 1.0, 1.9, 2.2, 3.0, 4.1]))
    s, d = W.random_rays(1500, np.random.default_rng(46), r_start=(12.0, 20.0), aim=5.0)
    P = _P()(g, rays=(s, d), mode="onthefly")
    S = P.info()["n_segments"]
    with chunk_segments(S // 5):
        _check(ora, g, P, s, d, 2, 47)


def test_frames_and_mixed_views_in_chunks(ora, dev):
    """Two cone and two parallel views with object frames (0, 1, 1, 0), one
    view per chunk: each chunk reads its views' frames and object frames."""
    w = W.tiny()
    cv = W.views_at([[50.0, 0.0, 0.0], [0.0, 50.0, 10.0]], (30.0, 30.0), 32, 32)
    pv = W.parallel_views_at([[0.0, -40.0, 5.0], [30.0, 30.0, -20.0]], (50.0, 50.0), 32, 32)
    sc, dc = ora.cone_rays(cv.pos, cv.look, cv.up, cv.fov_deg, 32, 32)
    sp, dp = parallel_rays(pv.pos, pv.look, pv.up, pv.size, 32, 32)
    s, d = np.concatenate([sc, sp]), np.concatenate([dc, dp])
    frames = [0, 1, 1, 0]
    F, V = 2, w.grid.size
    P = _P()(w.grid, views=[cv, pv], frames=frames, mode="onthefly")
    tr = ora.trace(w.grid.arrays(), s, d)
    fr = np.repeat(frames, 32 * 32)
    yy = np.random.default_rng(48).normal(size=(2, len(fr))).astype(np.float32)
    y_t = torch.from_numpy(yy).to(dev).reshape(2, *P.out_shape)
    S = P.info()["n_segments"]
    with chunk_segments((S + 3) // 4):
        x = P.backproject(y_t, "deterministic")
        assert torch.equal(x, P.backproject(y_t, "deterministic"))
    x = x.reshape(2, F, V).cpu().numpy().astype(np.float64)
    xo = D.adjoint_frames(tr, yy.astype(np.float64), fr, F, V)
    for b in range(2):
        tol = RTOL * D.adjoint_frames(tr, np.abs(yy[b]).astype(np.float64), fr, F, V) + 1e-7
        assert np.all(np.abs(x[b] - xo[b]) <= tol), b


def test_medium_in_chunks(dev):
    """Medium (50^3, 30 views 256x256) on the fly, deterministic adjoint in
    four chunks: the adjoint identity against the stored forward (FP64 sums on
    the host), columns of F at sampled voxels, the stored deterministic
    adjoint within the reordering of its sums, bitwise repeatable, and each
    object of a batch equal to its adjoint alone."""
    w = W.medium()
    Ps = _P()(w.grid, views=w.views)
    Po = _P()(w.grid, views=w.views, mode="onthefly")
    S = Po.info()["n_segments"]
    assert S == Ps.info()["n_segments"]
    V = Ps.info()["n_voxels"]
    g = torch.Generator(device=dev).manual_seed(49)
    yr = torch.rand((2, *Ps.out_shape), device=dev, generator=g)
    xr = torch.rand((2, *Ps.shape), device=dev, generator=g)
    with chunk_segments((S + 3) // 4):
        x = Po.backproject(yr, "deterministic")
        assert torch.equal(x, Po.backproject(yr, "deterministic"))
        for b in range(2):
            assert torch.equal(x[b:b + 1], Po.backproject(yr[b:b + 1], "deterministic")), b
    Fx = Ps.forward(xr).double()
    for b in range(2):
        lhs = float((Fx[b] * yr[b].double()).sum())
        rhs = float((xr[b].double() * x[b].double()).sum())
        assert abs(lhs - rhs) <= 1e-5 * abs(lhs), b
    xs = Ps.backproject(yr, "deterministic")
    assert torch.allclose(x, xs, rtol=1e-5, atol=1e-6 * float(xs.abs().max()))
    rng = np.random.default_rng(50)
    for v in rng.choice(V, 6, replace=False):
        e = torch.zeros(V, device=dev)
        e[v] = 1.0
        col = Ps.forward(e.reshape(1, *w.grid.shape)).double()[0]
        ref = float((col * yr[0].double()).sum())
        scale = float((col.abs() * yr[0].double().abs()).sum())
        assert abs(float(x[0].reshape(-1)[v]) - ref) <= 1e-5 * scale + 1e-7, v
