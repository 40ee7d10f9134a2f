"""Parallel-beam views (ParallelGeom, TomoSphero Sec. 4.2, Listing 3) for
the oracle, plain numpy.  Test infrastructure only.

Frame of a view (the same convention as the cone views): w = unit(look - pos),
u = unit(w x up) with up = +Z when all zero and +X when w is parallel to up,
v = u x w.  Pixel (i, j) of an H x W detector of size (height, width) starts
at pos + sx (width / 2) u + sy (height / 2) v with sx = 2 (j + 1/2) / W - 1
and sy = 2 (i + 1/2) / H - 1, and runs along w.  Ray id (view * H + i) * W + j.
"""
import numpy as np


def _frame(pos, look, up):
    w = np.asarray(look, np.float64) - np.asarray(pos, np.float64)
    w = w / np.linalg.norm(w)
    upv = np.asarray(up, np.float64)
    if not np.any(upv):
        upv = np.array([0.0, 0.0, 1.0])
    u = np.cross(w, upv)
    if np.linalg.norm(u) < 1e-12:
        u = np.cross(w, np.array([1.0, 0.0, 0.0]))
    u = u / np.linalg.norm(u)
    return w, u, np.cross(u, w)


def parallel_rays(pos, look, up, size, H, W):
    """(starts, dirs) float64 (V*H*W, 3) for V parallel views."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    V = len(pos)
    look = np.broadcast_to(np.asarray(look, np.float64), (V, 3))
    up = np.broadcast_to(np.asarray(up, np.float64), (V, 3))
    size = np.broadcast_to(np.asarray(size, np.float64), (V, 2))
    j = np.arange(W)
    i = np.arange(H)
    sx = (2.0 * (j + 0.5) / W - 1.0)[None, :] * np.ones((H, 1))
    sy = (2.0 * (i + 0.5) / H - 1.0)[:, None] * np.ones((1, W))
    starts, dirs = [], []
    for k in range(V):
        w, u, v = _frame(pos[k], look[k], up[k])
        o = (pos[k][None, None, :] + (sx * size[k, 1] / 2)[..., None] * u
             + (sy * size[k, 0] / 2)[..., None] * v)
        starts.append(o.reshape(-1, 3))
        dirs.append(np.tile(w, (H * W, 1)))
    return np.concatenate(starts), np.concatenate(dirs)
