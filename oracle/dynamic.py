"""Dynamic (4-D) objects: one object frame per view (TomoSphero Sec. 4.4,
where the operator accepts a 3-D or 4-D object, and Sec. 4.6, where the grid
stays fixed across frames).

Ray r of view v measures frame f(v) of the object,
    y[b, r] = sum_k len_k rho[b, f(v), vox_k],
and the adjoint sends y[b, r] len_k to x[b, f(v), vox_k].  Plain numpy over the
oracle's own segment lists, FP64.  Test infrastructure only, like the rest of
this package.
"""
import numpy as np


def _seg_rays(tr):
    R = len(tr["row_ptr"]) - 1
    return np.repeat(np.arange(R), np.diff(tr["row_ptr"])), R


def forward_frames(tr, rho, frame_of_ray):
    """rho: (B, F, V) or (F, V); frame_of_ray: (R,) ints.  Returns (B, R) or (R,)."""
    rho = np.asarray(rho, np.float64)
    single = rho.ndim == 2
    rho3 = rho[None] if single else rho
    B = rho3.shape[0]
    seg_ray, R = _seg_rays(tr)
    f = np.asarray(frame_of_ray)[seg_ray]
    y = np.zeros((B, R))
    for b in range(B):
        np.add.at(y[b], seg_ray, rho3[b][f, tr["vox"]] * tr["len"])
    return y[0] if single else y


def adjoint_frames(tr, y, frame_of_ray, F, V):
    """y: (B, R) or (R,).  Returns x (B, F, V) or (F, V)."""
    y = np.asarray(y, np.float64)
    single = y.ndim == 1
    y2 = y[None] if single else y
    B = y2.shape[0]
    seg_ray, _ = _seg_rays(tr)
    f = np.asarray(frame_of_ray)[seg_ray]
    x = np.zeros((B, F, V))
    for b in range(B):
        np.add.at(x[b], (f, tr["vox"]), y2[b][seg_ray] * tr["len"])
    return x[0] if single else x
