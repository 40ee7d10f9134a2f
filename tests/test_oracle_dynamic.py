"""Pins of the dynamic-object oracle (one frame per view, Sec. 4.4 / 4.6)
against the static oracle, which is pinned on its own: a single frame is the
static operator; frames that are multiples of one object scale each view's
measurements by that view's factor; the frame adjoints sum to the static
adjoint; and the forward / adjoint pair satisfies <F rho, y> = <rho, F^T y>."""
import numpy as np
import pytest

from oracle import dynamic as D
from paper_2608_16960_amd import workloads as W


@pytest.fixture(scope="module")
def case(ora):
    w = W.tiny()
    v = w.views
    s, d = ora.cone_rays(v.pos, v.look, v.up, v.fov_deg, v.H, v.W)
    tr = ora.trace(w.grid.arrays(), s, d)
    per_view = v.H * v.W
    frame_of_view = np.array([2, 0, 1, 2])  # 4 views, 3 frames, view 3 shares frame 2
    frame_of_ray = np.repeat(frame_of_view, per_view)
    return w, tr, frame_of_ray


def test_single_frame_is_static(ora, case):
    w, tr, _ = case
    V = w.grid.size
    rho = np.random.default_rng(0).uniform(-1, 2, (2, 1, V))
    y = D.forward_frames(tr, rho, np.zeros(len(tr["counts"]), int))
    ys = ora.forward(tr, rho[:, 0])
    assert np.allclose(y, ys, rtol=1e-12, atol=1e-12)
    yy = np.random.default_rng(1).normal(size=(2, len(tr["counts"])))
    x = D.adjoint_frames(tr, yy, np.zeros(len(tr["counts"]), int), 1, V)
    assert np.allclose(x[:, 0], ora.adjoint(tr, yy, V), rtol=1e-12, atol=1e-12)


def test_scaled_frames_scale_views(ora, case):
    w, tr, fr = case
    V = w.grid.size
    rho0 = w.rho[0].reshape(-1).astype(np.float64)
    c = np.array([0.5, -2.0, 3.0])
    y = D.forward_frames(tr, c[:, None] * rho0[None], fr)
    ys = ora.forward(tr, rho0)
    assert np.allclose(y, c[fr] * ys, rtol=1e-12, atol=1e-12)


def test_frame_adjoints_sum_to_static(ora, case):
    w, tr, fr = case
    V = w.grid.size
    yy = np.random.default_rng(2).normal(size=len(tr["counts"]))
    x = D.adjoint_frames(tr, yy, fr, 3, V)
    assert np.allclose(x.sum(0), ora.adjoint(tr, yy, V), rtol=1e-12, atol=1e-12)
    # a frame no view uses receives nothing
    x4 = D.adjoint_frames(tr, yy, fr, 4, V)
    assert np.all(x4[3] == 0)


def test_adjoint_identity(case):
    w, tr, fr = case
    V = w.grid.size
    rng = np.random.default_rng(3)
    rho = rng.normal(size=(3, V))
    yy = rng.normal(size=len(tr["counts"]))
    lhs = np.dot(D.forward_frames(tr, rho, fr), yy)
    rhs = np.sum(rho * D.adjoint_frames(tr, yy, fr, 3, V))
    assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + 1)
