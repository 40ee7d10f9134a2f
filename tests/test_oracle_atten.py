"""Pins of the attenuated-emission oracle (Sec. 9.3, Eqs. 14-18): no
absorption is the plain projector; a one-voxel ball and a radial ray
through two shells against hand-written closed forms (they fix the
inclusive cumulative sum, the line-of-sight order from the detector and
the sunward optical depth); the analytic gradient against central
differences of the forward."""
import numpy as np

from oracle import atten as A


def _ball(R=2.0):
    return (np.array([0.0, R]), np.array([0.0, np.pi]), np.array([0.0, 2 * np.pi]))


def test_no_absorption_is_plain_projector(ora):
    g = (np.linspace(1.0, 5.0, 6), np.linspace(0, np.pi, 5), np.linspace(0, 2 * np.pi, 7))
    rng = np.random.default_rng(50)
    s = rng.normal(size=(300, 3))
    s = 9.0 * s / np.linalg.norm(s, axis=1, keepdims=True)
    d = rng.uniform(-2, 2, (300, 3)) - s
    tr = ora.trace(g, s, d)
    trs = A.sun_trace(g, [0.2, 0.9, -0.3])
    rho = rng.uniform(0, 2, 5 * 4 * 6)
    y = A.forward(tr, trs, rho, np.zeros_like(rho))
    assert np.allclose(y, ora.forward(tr, rho), rtol=1e-13, atol=1e-13)


def test_one_voxel_ball_closed_form(ora):
    """Ball of radius R, one voxel, rho = c, sigma = k.  Centroid at
    (r, theta, phi) = (R/2, pi/2, pi), i.e. (-R/2, 0, 0); sun along +x, so
    tau_1 = k c (R/2 + R).  A line of sight with impact parameter b has one
    segment of length L = 2 sqrt(R^2 - b^2): y = exp(-tau_1) c exp(-k c L) L."""
    R, c, k = 2.0, 0.7, 0.3
    g = _ball(R)
    bs = np.array([0.0, 0.5, 1.2, 1.9])
    s = np.stack([np.full(4, -10.0), bs, np.zeros(4)], 1)
    d = np.tile([1.0, 0.0, 0.0], (4, 1))
    tr = ora.trace(g, s, d)
    trs = A.sun_trace(g, [1.0, 0.0, 0.0])
    y = A.forward(tr, trs, np.array([c]), np.array([k]))
    L = 2 * np.sqrt(R * R - bs * bs)
    tau1 = k * c * 1.5 * R
    assert np.allclose(y, np.exp(-tau1) * c * np.exp(-k * c * L) * L, rtol=1e-13)


def test_radial_ray_two_shells(ora):
    """Shells r_b = (0, 1, 3) (one angular voxel each), radial ray from
    x = 5 along -x: outer (length 2), inner (length 2), outer (length 2).
    y = w1 e^{-2 s1} 2 + w0 e^{-2 s1 - 2 s0} 2 + w1 e^{-4 s1 - 2 s0} 2."""
    g = (np.array([0.0, 1.0, 3.0]), np.array([0.0, np.pi]), np.array([0.0, 2 * np.pi]))
    tr = ora.trace(g, np.array([[5.0, 0.0, 0.0]]), np.array([[-1.0, 0.0, 0.0]]))
    assert list(tr["vox"]) == [1, 0, 1]
    rho = np.array([0.8, 0.5])
    sig = np.array([0.4, 0.1])
    sun = [0.0, 0.0, 1.0]
    trs = A.sun_trace(g, sun)
    s = sig * rho
    # sunward optical depths from the centroids (r = 1/2 and 2 on the -x axis,
    # theta = pi/2, phi = pi), straight up +z: voxel 0 crosses the rest of
    # shell 0 then shell 1; voxel 1 stays in shell 1
    h0 = np.sqrt(1 - 0.25)
    tau0 = s[0] * h0 + s[1] * (np.sqrt(9 - 0.25) - h0)
    tau1 = s[1] * np.sqrt(9 - 4)
    w = np.exp(-np.array([tau0, tau1])) * rho
    T1 = 2 * s[1]
    T2 = T1 + 2 * s[0]
    T3 = T2 + 2 * s[1]
    expect = w[1] * np.exp(-T1) * 2 + w[0] * np.exp(-T2) * 2 + w[1] * np.exp(-T3) * 2
    y = A.forward(tr, trs, rho, sig)
    assert abs(y[0] - expect) <= 1e-13 * abs(expect)


def test_gradient_matches_central_differences(ora):
    g = (np.linspace(1.0, 4.0, 4), np.linspace(0.2, 2.9, 4), np.linspace(0, 2 * np.pi, 5))
    V = 3 * 3 * 4
    rng = np.random.default_rng(51)
    s = rng.normal(size=(60, 3))
    s = 7.0 * s / np.linalg.norm(s, axis=1, keepdims=True)
    d = rng.uniform(-1.5, 1.5, (60, 3)) - s
    tr = ora.trace(g, s, d)
    trs = A.sun_trace(g, [0.5, -0.5, 0.7])
    rho = rng.uniform(0.2, 1.5, V)
    sig = rng.uniform(0.1, 0.6, V)
    gy = rng.normal(size=60)
    grad = A.gradient(tr, trs, rho, sig, gy)
    h = 1e-6
    fd = np.empty(V)
    for v in range(V):
        e = np.zeros(V)
        e[v] = h
        fd[v] = (gy @ A.forward(tr, trs, rho + e, sig) - gy @ A.forward(tr, trs, rho - e, sig)) / (2 * h)
    assert np.allclose(grad, fd, rtol=1e-6, atol=1e-8 * np.abs(fd).max())
