"""Pins of the oracle for rays that start inside the grid (the sunward rays
from voxel centroids of Sec. 9.3; the integral runs over l >= 0 from the
start, Eq. 3).  Checked against things other than the oracle itself: the
exit distance of a ball in closed form, hand-derived lists, and the
already-pinned outside-start traces (an outside ray cut at an interior point
must leave exactly the interior ray's segments)."""
import numpy as np

from paper_2608_16960_amd import workloads as W


def test_ball_exit_distance(ora):
    """Grid filling the unit ball: total length = distance to the sphere."""
    g = W.uniform_grid((5, 6, 8), r=(0.0, 1.0))
    rng = np.random.default_rng(40)
    u = rng.normal(size=(400, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    p = u * rng.uniform(0.05, 0.95, (400, 1)) ** (1 / 3)
    n = rng.normal(size=(400, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    tr = ora.trace(g.arrays(), p, n)
    tot = np.zeros(400)
    np.add.at(tot, np.repeat(np.arange(400), tr["counts"]), tr["len"])
    pn = np.sum(p * n, 1)
    t_exit = -pn + np.sqrt(pn * pn - np.sum(p * p, 1) + 1.0)
    assert np.allclose(tot, t_exit, rtol=1e-12, atol=1e-12)


def test_start_at_origin_and_in_the_hole(ora):
    """Shell r in [1, 2], one voxel: from the origin (or anywhere in the
    hole) a ray crosses the shell once, length 1 from the origin."""
    g = W.Grid(np.array([1.0, 2.0]), np.array([0.0, np.pi]), np.array([0.0, 2 * np.pi]))
    n = np.array([[0.3, -0.5, 0.8], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0]])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    tr = ora.trace(g.arrays(), np.zeros((3, 3)), n)
    assert list(tr["counts"]) == [1, 1, 1]
    assert np.all(tr["vox"] == 0) and np.allclose(tr["len"], 1.0, atol=1e-14)
    # start in the hole off-centre: exit chord of r = 2 minus that of r = 1
    p = np.array([[0.4, 0.1, -0.2]])
    d = np.array([[0.0, 1.0, 0.0]])
    tr = ora.trace(g.arrays(), p, d)
    py = 0.1
    rho2 = 0.4 ** 2 + 0.2 ** 2
    expect = (np.sqrt(4 - rho2) - py) - (np.sqrt(1 - rho2) - py)
    assert tr["counts"][0] == 1 and abs(tr["len"][0] - expect) < 1e-14


def test_start_on_a_sphere_moving_inwards(ora):
    """Shells r_b = (1, 2, 3), full angular range; start on r = 2 moving
    towards the centre along -x: shell 0 for length 1, the hole for 2,
    shell 0 again for 1, shell 1 for 1 (re-entry after a gap is a new
    segment)."""
    g = W.Grid(np.array([1.0, 2.0, 3.0]), np.array([0.0, np.pi]), np.array([0.0, 2 * np.pi]))
    tr = ora.trace(g.arrays(), np.array([[2.0, 0.0, 0.0]]), np.array([[-1.0, 0.0, 0.0]]))
    assert list(tr["vox"]) == [0, 0, 1]
    assert np.allclose(tr["len"], [1.0, 1.0, 1.0], atol=1e-14)
    assert np.allclose(tr["t0"], [0.0, 3.0, 4.0], atol=1e-14)


def test_cut_outside_ray_equals_interior_ray(ora):
    """For rays from outside, start a second ray at a point p = x + n t_p
    inside the grid: its segment list is the outside ray's list after t_p
    (the segment containing t_p shortened to end - t_p)."""
    for grid in (W.uniform_grid((8, 7, 9), r=(1.0, 6.0)),
                 W.Grid(np.array([2.0, 2.7, 3.1, 4.4, 6.0]), np.array([0.3, 0.8, 1.5708, 2.9]),
                        np.array([-0.4, 0.3, 1.9, 3.0, 4.1]))):
        rng = np.random.default_rng(41)
        s, d = W.random_rays(600, rng, r_start=(8.0, 12.0), aim=3.0)
        d = d / np.linalg.norm(d, axis=1, keepdims=True)
        tro = ora.trace(grid.arrays(), s, d)
        Ro = grid.r_b[-1]
        sn = np.sum(s * d, 1)
        disc = sn * sn - (np.sum(s * s, 1) - Ro * Ro)
        hit = disc > 0
        tin = -sn - np.sqrt(np.where(hit, disc, 0))
        tout = -sn + np.sqrt(np.where(hit, disc, 0))
        tp = tin + rng.uniform(0.1, 0.9, 600) * (tout - tin)
        p = s + d * tp[:, None]
        tri = ora.trace(grid.arrays(), p, d)
        checked = 0
        for i in np.nonzero(hit & ~tro["tie"] & ~tri["tie"])[0]:
            a, b = tro["row_ptr"][i], tro["row_ptr"][i + 1]
            t0, ln, vx = tro["t0"][a:b], tro["len"][a:b], tro["vox"][a:b]
            keep = t0 + ln > tp[i]
            exp_v = vx[keep]
            exp_l = np.minimum(ln[keep], t0[keep] + ln[keep] - tp[i])
            c, e = tri["row_ptr"][i], tri["row_ptr"][i + 1]
            assert np.array_equal(tri["vox"][c:e], exp_v), i
            # p itself is rounded, and a crossing met at a grazing angle moves by
            # eps |p| / sin(angle): 1e-8 absolute, against lengths of 0.1 - 2
            assert np.allclose(tri["len"][c:e], exp_l, rtol=1e-9, atol=1e-8), i
            checked += 1
        assert checked > 200
