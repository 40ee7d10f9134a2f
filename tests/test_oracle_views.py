"""Pins of the oracle's parallel-beam views (Sec. 4.2, Listing 3): every ray
runs along unit(look - pos); origins lie on the detector plane through pos,
centred on it, one pixel pitch apart along the frame axes; and through a
uniform ball each ray measures the chord 2 sqrt(R^2 - b^2)."""
import numpy as np

from oracle.views import parallel_rays


def test_geometry_of_the_rays():
    pos = np.array([[10.0, 2.0, -1.0], [0.0, -9.0, 4.0]])
    look = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 0.0]])
    H, W, size = 5, 7, (3.0, 4.2)
    s, d = parallel_rays(pos, look, [0, 0, 0], size, H, W)
    for k in range(2):
        w = (look[k] - pos[k]) / np.linalg.norm(look[k] - pos[k])
        sk = s[k * H * W:(k + 1) * H * W].reshape(H, W, 3)
        assert np.allclose(d[k * H * W:(k + 1) * H * W], w, atol=1e-15)
        assert np.allclose((sk - pos[k]) @ w, 0.0, atol=1e-13)        # on the detector plane
        assert np.allclose(sk.mean((0, 1)), pos[k], atol=1e-13)       # centred on pos
        assert np.allclose(np.linalg.norm(sk[:, 1:] - sk[:, :-1], axis=-1), 4.2 / W)
        assert np.allclose(np.linalg.norm(sk[1:] - sk[:-1], axis=-1), 3.0 / H)
        # columns grow along u = w x up (up = +Z), rows along v = u x w
        u = np.cross(w, [0.0, 0.0, 1.0])
        u /= np.linalg.norm(u)
        assert np.allclose((sk[:, 1] - sk[:, 0]) @ u, 4.2 / W)
        assert np.allclose((sk[1, :] - sk[0, :]) @ np.cross(u, w), 3.0 / H)


def test_ball_chords(ora):
    g = (np.linspace(0.0, 1.0, 6), np.linspace(0, np.pi, 7), np.linspace(0, 2 * np.pi, 9))
    s, d = parallel_rays([[3.0, 0.5, -2.0]], [[0.1, -0.2, 0.3]], [0, 0, 0], (2.6, 2.6), 17, 17)
    tr = ora.trace(g, s, d)
    y = ora.forward(tr, np.ones(5 * 6 * 8))
    b2 = np.sum(np.cross(s, d) ** 2, 1)
    ref = 2 * np.sqrt(np.maximum(1 - b2, 0))
    ok = ~tr["tie"]
    assert np.allclose(y[ok], ref[ok], atol=1e-12)
    assert np.sum(ref > 0) > 100
