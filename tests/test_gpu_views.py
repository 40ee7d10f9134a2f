"""GPU parity for parallel-beam views (ParallelGeom, Sec. 4.2, Listing 3)
and mixed collections of cone and parallel views (Sec. 4.3) against the CPU
oracle (oracle/views.py for the parallel rays).  The static parity bars
apply (tests/test_gpu_parity.py): rays within 1e-13, index lists
bit-exact on non-tie rays, projections and adjoints within 1e-5 of the
absolute integrand."""
import numpy as np
import pytest
import torch

from oracle.views import parallel_rays
from paper_2608_16960_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda", 0)


def _P():
    from paper_2608_16960_amd.projector import Projector
    return Projector


@pytest.mark.parametrize("mode", ["csr", "onthefly"])
def test_parallel_views(ora, dev, mode):
    from test_gpu_parity import _check_all
    w = W.tiny()
    pv = W.parallel_views_at([[40.0, 5.0, 3.0], [-2.0, 45.0, -10.0], [0.0, 0.0, -50.0]],
                             (44.0, 52.0), 24, 40, look=[1.0, -0.5, 0.5])
    s, d = parallel_rays(pv.pos, pv.look, pv.up, pv.size, pv.H, pv.W)
    P = _P()(w.grid, views=pv, mode=mode)
    rho = np.concatenate([w.rho, np.random.default_rng(70).uniform(-1, 2, (1, *w.grid.shape))])
    _check_all(ora, w.grid, P, s, d, rho.astype(np.float32))


def test_mixed_collection(ora, dev):
    """Two cone views and two parallel views of one detector shape, in that
    order; plus object frames over the collection."""
    from test_gpu_parity import _check_all
    w = W.tiny()
    cv = W.views_at([[50.0, 0.0, 0.0], [0.0, 50.0, 10.0]], (30.0, 30.0), 32, 32)
    pv = W.parallel_views_at([[0.0, -40.0, 5.0], [30.0, 30.0, -20.0]], (50.0, 50.0), 32, 32)
    sc, dc = ora.cone_rays(cv.pos, cv.look, cv.up, cv.fov_deg, 32, 32)
    sp, dp = parallel_rays(pv.pos, pv.look, pv.up, pv.size, 32, 32)
    s, d = np.concatenate([sc, sp]), np.concatenate([dc, dp])
    P = _P()(w.grid, views=[cv, pv])
    assert P.out_shape == (4, 32, 32)
    _check_all(ora, w.grid, P, s, d, w.rho.astype(np.float32))
    from oracle import dynamic as D
    Pd = _P()(w.grid, views=[cv, pv], frames=[0, 1, 1, 0])
    rho = np.random.default_rng(71).uniform(0, 1, (2, w.grid.size)).astype(np.float32)
    y = Pd.forward(torch.from_numpy(rho).reshape(1, 2, *w.grid.shape).to(dev))
    tr = ora.trace(w.grid.arrays(), s, d)
    yo = D.forward_frames(tr, rho.astype(np.float64), np.repeat([0, 1, 1, 0], 32 * 32))
    assert np.all(np.abs(y.reshape(-1).cpu().numpy() - yo) <= 1e-5 * np.abs(yo) + 1e-7)


def test_parallel_unit_sphere_fp32(dev):
    """Unit ball on (50, 50, 50), rho = 1, parallel views: y = 2 sqrt(1 - b^2)."""
    g = W.uniform_grid((50, 50, 50), r=(0.0, 1.0))
    pv = W.parallel_views_at([[3.0, 0.0, 0.0], [0.0, -2.0, 1.5]], (2.4, 2.4), 41, 41)
    P = _P()(g, views=pv)
    y = P.forward(torch.ones(g.shape, device=dev)).cpu().numpy().reshape(-1).astype(np.float64)
    s, d = (t.cpu().numpy() for t in P.rays())
    ref = 2 * np.sqrt(np.maximum(1 - np.sum(np.cross(s, d) ** 2, 1), 0))
    hit = ref > 1e-2
    assert np.max(np.abs(y - ref)[hit] / ref[hit]) < 1e-6
    assert np.all(np.abs(y[~hit] - ref[~hit]) < 1e-5)
