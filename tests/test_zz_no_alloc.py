"""The no-allocation deterministic adjoint (tsp_backproject_noalloc) against
tsp_backproject with TSP_ADJ_DETERMINISTIC, called through the C ABI.

Both run the same kernels in the same order, so the bar is bitwise equality.
Two calls in a row share the fixed device workspace: the 30-view Medium
geometry at batch 4 first, then the 4-view Tiny geometry at batch 1 (a
smaller copy of y that leaves the first call's contents behind it).  The
Tiny result is also checked against the CPU FP64 oracle at the projection
bar (1e-5 of the absolute integrand per voxel).
"""

import numpy as np
import pytest
import torch

from paper_2608_16960_amd import workloads as W

pytestmark = pytest.mark.gpu


def _noalloc(P, y, B):
    from paper_2608_16960_amd import native as N
    x = torch.full((B, *P.obj_shape), float("nan"), dtype=torch.float32, device=P.device)
    N.check(N.lib.tsp_backproject_noalloc(P._h, N.ptr(y), B, N.ptr(x), N.stream_handle()))
    return x


def _reference(P, y, B):
    from paper_2608_16960_amd import native as N
    x = torch.full((B, *P.obj_shape), float("nan"), dtype=torch.float32, device=P.device)
    N.check(N.lib.tsp_backproject(P._h, N.ptr(y), B, N.ptr(x), N.TSP_ADJ_DETERMINISTIC,
                                  N.stream_handle()))
    return x


def test_noalloc_equals_backproject_two_calls(ora):
    from paper_2608_16960_amd.projector import Projector
    dev = torch.device("cuda", 0)
    print("noalloc: Medium batch 4, then Tiny batch 1", flush=True)
    wm = W.medium()
    Pm = Projector(wm.grid, views=wm.views)
    g = torch.Generator(device="cpu").manual_seed(11)
    ym = torch.randn((4, Pm.n_rays), generator=g).to(dev)
    xa = _noalloc(Pm, ym, 4)
    xb = _reference(Pm, ym, 4)
    torch.cuda.synchronize()
    assert torch.isfinite(xa).all()
    assert torch.equal(xa, xb)
    del Pm

    wt = W.tiny()
    Pt = Projector(wt.grid, views=wt.views)
    yt = torch.randn((1, Pt.n_rays), generator=g).to(dev)
    xa = _noalloc(Pt, yt, 1)
    xb = _reference(Pt, yt, 1)
    torch.cuda.synchronize()
    assert torch.isfinite(xa).all()
    assert torch.equal(xa, xb)

    v = wt.views
    s, d = ora.cone_rays(v.pos, v.look, v.up, v.fov_deg, v.H, v.W)
    tr = ora.trace(wt.grid.arrays(), s, d)
    yy = yt.cpu().numpy().astype(np.float64)
    xo = ora.adjoint(tr, yy[0], wt.grid.size)
    seg_ray = np.repeat(np.arange(len(s)), tr["counts"])
    absx = np.zeros(wt.grid.size)
    np.add.at(absx, tr["vox"], np.abs(yy[0][seg_ray]) * tr["len"])
    err = np.abs(xa.reshape(-1).cpu().numpy().astype(np.float64) - xo)
    assert np.all(err <= 1e-5 * absx + 1e-7)


def test_noalloc_batches_and_limits():
    """Batches above four go through the workspace in groups; a copy of y
    beyond the workspace is refused with TSP_E_NOMEM, and a geometry
    without the voxel-major store with TSP_E_STATE."""
    from paper_2608_16960_amd import native as N
    from paper_2608_16960_amd.projector import Projector
    dev = torch.device("cuda", 0)
    print("noalloc: Tiny batch 6, limits", flush=True)
    wt = W.tiny()
    Pt = Projector(wt.grid, views=wt.views)
    g = torch.Generator(device="cpu").manual_seed(12)
    y6 = torch.randn((6, Pt.n_rays), generator=g).to(dev)
    assert torch.equal(_noalloc(Pt, y6, 6), _reference(Pt, y6, 6))

    # 16 voxels, 3 views of 2048 x 2048 rays: 12.6M slots, 50 MB at batch 1,
    # 201 MB at batch 4 (beyond the 128 MiB workspace)
    grid = W.uniform_grid((2, 2, 4), r=(1.0, 2.0))
    pos = np.array([[10.0, 0, 0], [0, 10.0, 0], [0, 0, 10.0]])
    views = W.views_at(pos, (25.0, 25.0), 2048, 2048)
    P = Projector(grid, views=views)
    assert P.info()["n_stored"] >= 0
    y1 = torch.randn((1, P.n_rays), generator=g).to(dev)
    assert torch.equal(_noalloc(P, y1, 1), _reference(P, y1, 1))
    y4 = torch.randn((4, P.n_rays), generator=g).to(dev)
    x4 = torch.empty((4, *P.obj_shape), dtype=torch.float32, device=dev)
    st = N.lib.tsp_backproject_noalloc(P._h, N.ptr(y4), 4, N.ptr(x4), N.stream_handle())
    assert st == N.TSP_E_NOMEM
    assert b"workspace" in N.lib.tsp_last_error()
    del P

    Pn = Projector(wt.grid, views=wt.views, csc=False)
    y1 = torch.randn((1, Pn.n_rays), generator=g).to(dev)
    x1 = torch.empty((1, *Pn.obj_shape), dtype=torch.float32, device=dev)
    st = N.lib.tsp_backproject_noalloc(Pn._h, N.ptr(y1), 1, N.ptr(x1), N.stream_handle())
    assert st == N.TSP_E_STATE
    st = N.lib.tsp_backproject_noalloc(Pn._h, N.ptr(y1), 0, N.ptr(x1), N.stream_handle())
    assert st == N.TSP_E_INVALID
    torch.cuda.synchronize()
