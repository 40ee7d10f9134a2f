"""Pins of the oracle's cone-beam rays (Sec. 4.2 ConeRectGeom; detector at
the cone vertex, Sec. 4.6) under the pinhole reading: w = unit(look - pos),
u = unit(w x up) (up = +Z when zero, +X when w is parallel to it),
v = u x w; pixel (i, j) of an H x W detector looks along
unit(w + sx u + sy v), sx = (2 (j + 1/2) / W - 1) tan(fov_w / 2),
sy = (2 (i + 1/2) / H - 1) tan(fov_h / 2); fov is the full angle; ray id
= (view H + i) W + j.

The checks are geometric facts of that reading, computed here from angles
and explicit world directions (not by re-running the formula), and chosen
so that each plausible misreading fails one of them: the FOV taken as a
half angle, H and W (or fov_h and fov_w) swapped, the sign of v or u
flipped, pixel edges instead of centres, a wrong fallback axis, or a wrong
ray-id order."""
import numpy as np
import pytest


def _angle(a, b):
    return np.arccos(np.clip(np.sum(a * b, -1) / (np.linalg.norm(a, axis=-1) *
                                                   np.linalg.norm(b, axis=-1)), -1, 1))


def _rays(ora, pos, look, up, fov, H, W):
    pos = np.atleast_2d(np.asarray(pos, float))
    n = pos.shape[0]
    look = np.broadcast_to(np.asarray(look, float), (n, 3)).copy()
    up = np.broadcast_to(np.asarray(up, float), (n, 3)).copy()
    fov = np.broadcast_to(np.asarray(fov, float), (n, 2)).copy()
    s, d = ora.cone_rays(pos, look, up, fov, H, W)
    return s.reshape(n, H, W, 3), d.reshape(n, H, W, 3)


def test_axis_along_x_world_orientation(ora):
    """View on +X looking at the origin, up = +Z: w = -X, u = w x Z = +Y,
    v = u x w = +Z.  Columns (j) therefore sweep towards +Y, rows (i)
    towards +Z; with an odd, non-square detector the centre pixel looks
    exactly at the origin."""
    H, W, fov = 5, 9, (20.0, 40.0)
    s, d = _rays(ora, [10.0, 0, 0], [0, 0, 0], [0, 0, 0], fov, H, W)
    s, d = s[0], d[0]
    assert np.all(s == np.array([10.0, 0, 0]))
    assert np.allclose(np.linalg.norm(d, axis=-1), 1.0, atol=1e-15)
    assert np.allclose(d[2, 4], [-1.0, 0, 0], atol=1e-15)
    # centre row: no z component, y grows with j; centre column: no y, z grows with i
    assert np.allclose(d[2, :, 2], 0.0, atol=1e-15)
    assert np.all(np.diff(d[2, :, 1]) > 0) and d[2, -1, 1] > 0
    assert np.allclose(d[:, 4, 1], 0.0, atol=1e-15)
    assert np.all(np.diff(d[:, 4, 2]) > 0) and d[-1, 4, 2] > 0
    # the corner pixel (0, W-1): +Y and -Z
    assert d[0, -1, 1] > 0 and d[0, -1, 2] < 0


@pytest.mark.parametrize("H,W,fov", [(5, 9, (20.0, 40.0)), (7, 3, (50.0, 15.0)),
                                     (1, 6, (10.0, 70.0))])
def test_angles_are_full_fov_at_pixel_centres(ora, H, W, fov):
    """The angle of pixel (i, j) from the optical axis is
    atan(sqrt(sx^2 + sy^2)); along the centre row / column it is
    atan(|2 (j + 1/2) / W - 1| tan(fov_w / 2)), so the outermost centres sit
    half a pixel inside the full field: the edge pixels' axis angle is
    atan((1 - 1/W) tan(fov_w / 2)) (not fov_w / 2, not fov_w / 4)."""
    pos = np.array([3.0, -40.0, 12.0])
    look = np.array([0.5, 0.2, -0.3])
    s, d = _rays(ora, pos, look, [0, 0, 0], fov, H, W)
    d = d[0]
    w = (look - pos) / np.linalg.norm(look - pos)
    th, tw = np.tan(np.radians(fov[0]) / 2), np.tan(np.radians(fov[1]) / 2)
    i, j = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    sx = (2 * (j + 0.5) / W - 1) * tw
    sy = (2 * (i + 0.5) / H - 1) * th
    ang = _angle(d, np.broadcast_to(w, d.shape))
    assert np.allclose(ang, np.arctan(np.hypot(sx, sy)), atol=1e-14)
    # the edge columns of any row straddle the axis by the FOV less half a pixel
    c = d[:, [0, -1]]
    if H % 2 == 1:
        mid = H // 2
        edge = np.arctan((1 - 1 / W) * tw)
        assert np.allclose(_angle(c[mid, 0], w), edge, atol=1e-14)
        assert np.allclose(_angle(c[mid, 0], c[mid, 1]), 2 * edge, atol=1e-13)


def test_full_angle_limit(ora):
    """With many pixels the two outermost columns of the centre row span
    almost exactly the full field of view fov_w (a half-angle reading would
    give fov_w / 2, a swap of H and W would give fov_h)."""
    H, W, fov = 3, 4001, (10.0, 60.0)
    s, d = _rays(ora, [0.0, 0.0, -30.0], [0, 0, 0], [0.0, 1.0, 0.0], fov, H, W)
    span = np.degrees(_angle(d[0, 1, 0], d[0, 1, -1]))
    assert abs(span - 60.0) < 0.02
    span_rows = np.degrees(_angle(d[0, 0, W // 2], d[0, -1, W // 2]))
    assert abs(span_rows - np.degrees(2 * np.arctan(np.tan(np.radians(5.0)) * 2 / 3))) < 1e-10


def test_frame_axes_and_user_up(ora):
    """sx and sy are the tangent offsets along u = unit(w x up) and
    v = u x w: (d.u)/(d.w) and (d.v)/(d.w) recover them, for a tilted up
    hint that is not perpendicular to w."""
    H, W, fov = 4, 6, (30.0, 45.0)
    pos = np.array([-20.0, 15.0, 8.0])
    up = np.array([0.3, 0.1, 1.0])
    s, d = _rays(ora, pos, [0, 0, 0], up, fov, H, W)
    d = d[0]
    w = -pos / np.linalg.norm(pos)
    u = np.cross(w, up)
    u /= np.linalg.norm(u)
    v = np.cross(u, w)
    # v lies in the plane of w and up, on up's side
    assert np.dot(v, up) > 0 and abs(np.dot(np.cross(w, up), v)) < 1e-12
    dw = d @ w
    th, tw = np.tan(np.radians(fov[0]) / 2), np.tan(np.radians(fov[1]) / 2)
    i, j = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    assert np.allclose((d @ u) / dw, (2 * (j + 0.5) / W - 1) * tw, atol=1e-14)
    assert np.allclose((d @ v) / dw, (2 * (i + 0.5) / H - 1) * th, atol=1e-14)


def test_fallback_up_when_looking_along_z(ora):
    """A view on +Z looking at the origin has w = -Z parallel to the
    default up: up becomes +X, so u = (-Z) x X = -Y and v = u x w = +X."""
    H, W = 3, 5
    s, d = _rays(ora, [0.0, 0.0, 10.0], [0, 0, 0], [0, 0, 0], (20.0, 30.0), H, W)
    d = d[0]
    assert np.allclose(d[1, 2], [0, 0, -1.0], atol=1e-15)
    assert np.allclose(d[1, :, 0], 0.0, atol=1e-15)
    assert np.all(np.diff(d[1, :, 1]) < 0)       # columns towards -Y
    assert np.allclose(d[:, 2, 1], 0.0, atol=1e-15)
    assert np.all(np.diff(d[:, 2, 0]) > 0)       # rows towards +X
    # an explicit up parallel to w falls back the same way
    s2, d2 = _rays(ora, [0.0, 0.0, 10.0], [0, 0, 0], [0, 0, -2.0], (20.0, 30.0), H, W)
    assert np.array_equal(d2[0], d)


def test_ray_id_order_over_views(ora):
    """Ray id = (view H + i) W + j: the flat arrays hold view 0's rows
    first, each row's columns consecutively; starts are the view position."""
    pos = np.array([[30.0, 0, 0], [0, 30.0, 0], [0, 0, -30.0]])
    H, W = 2, 3
    s, d = ora.cone_rays(pos, np.zeros((3, 3)), np.zeros((3, 3)), np.full((3, 2), 20.0), H, W)
    assert s.shape == (3 * H * W, 3)
    for v in range(3):
        blk = slice(v * H * W, (v + 1) * H * W)
        assert np.all(s[blk] == pos[v])
        w = -pos[v] / 30.0
        assert np.all(d[blk] @ w > np.cos(np.radians(15.0)))
        one = ora.cone_rays(pos[v:v + 1], np.zeros((1, 3)), np.zeros((1, 3)),
                            np.full((1, 2), 20.0), H, W)[1]
        assert np.array_equal(d[blk], one)
    # within a view, id + 1 moves one column (j), id + W one row (i)
    dv = d[:H * W].reshape(H, W, 3)
    assert np.array_equal(d[1], dv[0, 1]) and np.array_equal(d[W], dv[1, 0])
