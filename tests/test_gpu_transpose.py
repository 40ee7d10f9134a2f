"""The voxel-major store built in passes over key ranges (so that its
temporaries fit the free device memory): every pass is a stable sort of a
contiguous range of (frame, voxel) keys, so the store, and with it the
deterministic adjoint, does not depend on the number of passes.  Forced here
with TSP_TRANSPOSE_MAX_ENTRIES and compared bit for bit with one pass."""
import numpy as np
import pytest
import torch

from paper_2608_16960_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda", 0)


def _P():
    from paper_2608_16960_amd.projector import Projector
    return Projector


def _same_adjoints(monkeypatch, dev, grid, views, frac, frames=None, B=3):
    """Passes of at most frac * S entries (at least three passes)."""
    P1 = _P()(grid, views=views, frames=frames)
    S = P1.info()["n_segments"]
    cap = int(S * frac) + 1
    monkeypatch.setenv("TSP_TRANSPOSE_MAX_ENTRIES", str(cap))
    P2 = _P()(grid, views=views, frames=frames)
    monkeypatch.delenv("TSP_TRANSPOSE_MAX_ENTRIES")
    assert P2.info()["n_segments"] == S > 2 * cap
    y = torch.randn((B, *P1.out_shape), device=dev)
    assert torch.equal(P1.backproject(y), P2.backproject(y))
    assert torch.equal(P1.backproject(y[:1]), P2.backproject(y[:1]))


def test_tiny_in_many_passes(monkeypatch, dev):
    w = W.tiny()
    _same_adjoints(monkeypatch, dev, w.grid, w.views, 0.01)


def test_dynamic_ragged_in_passes(monkeypatch, dev):
    g = W.Grid(np.array([2.0, 2.7, 3.1, 4.4, 6.0, 9.5]), np.array([0.3, 0.8, 1.2, 1.5708, 2.0, 2.9]),
               np.array([-0.4, 0.3, 1.0, 1.9, 2.2, 3.0, 4.1]))
    pos = np.array([[20.0, 3.0, 5.0], [-4.0, 18.0, -7.0], [2.0, -3.0, 22.0]])
    v = W.views_at(pos, (45.0, 38.0), 37, 29, look=[0.5, -0.2, 0.1])
    _same_adjoints(monkeypatch, dev, g, v, 0.2, frames=[1, 0, 1])


def test_medium_in_passes(monkeypatch, dev):
    w = W.medium()
    _same_adjoints(monkeypatch, dev, w.grid, w.views, 0.2, B=1)


def test_pass_smaller_than_a_key_is_out_of_memory(monkeypatch, dev):
    from paper_2608_16960_amd import native as N
    w = W.tiny()
    monkeypatch.setenv("TSP_TRANSPOSE_MAX_ENTRIES", "5")
    with pytest.raises(N.TspError) as e:
        _P()(w.grid, views=w.views)
    assert e.value.status == N.TSP_E_NOMEM
