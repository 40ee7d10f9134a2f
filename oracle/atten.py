"""Attenuated emission model (TomoSphero Sec. 9.3, Eqs. 14-18) on the
oracle's own segment lists, FP64.  Test infrastructure only.

With s = sigma * rho (absorption per unit length in each voxel):
  - tau_1[v] = sum over the sunward ray from voxel v's centroid of
    s[vox] * len: Eq. 14 discretised by the projector F_1 of Eq. 17, whose
    rays start at the centroids and run towards the Sun;
  - w = exp(-tau_1) * rho;
  - along a line of sight, segments k = 0, 1, ... in order of distance from
    the detector, T_k = sum over j <= k of s[v_j] len_j (Eq. 15 restricted to
    the line of sight, the inclusive cumulative sum of Eq. 18);
  - y = sum over k of w[v_k] * exp(-T_k) * len_k (Eqs. 16-17, with the
    constant g phi / 4 pi of Eq. 16 left to the caller).

gradient() is the derivative of forward() with respect to rho, written out
from these formulas (chain rule through w, tau_1 and T); the tests pin it
against central differences of forward().
"""
import numpy as np

from .projector import adjoint as _adjoint
from .projector import forward as _forward
from .projector import trace as _trace


def centroids(grid):
    """(V, 3) voxel centroids at the mid-boundaries (r_c, theta_c, phi_c),
    voxel order (ir, ie, ia)."""
    rb, eb, ab = (np.asarray(a, np.float64) for a in grid)
    rc, tc, pc = 0.5 * (rb[1:] + rb[:-1]), 0.5 * (eb[1:] + eb[:-1]), 0.5 * (ab[1:] + ab[:-1])
    R, Tt, P = np.meshgrid(rc, tc, pc, indexing="ij")
    X = np.stack([R * np.sin(Tt) * np.cos(P), R * np.sin(Tt) * np.sin(P), R * np.cos(Tt)], -1)
    return X.reshape(-1, 3)


def sun_trace(grid, sun_dir):
    """Segment lists of the sunward rays, one per voxel centroid (F_1)."""
    c = centroids(grid)
    d = np.tile(np.asarray(sun_dir, np.float64).reshape(1, 3), (len(c), 1))
    return _trace(grid, c, d)


def _rows(tr):
    rp = np.asarray(tr["row_ptr"])
    R = len(rp) - 1
    return np.repeat(np.arange(R), np.diff(rp)), rp, R


def _row_cumsum(vals, rp):
    """Inclusive cumulative sum of vals within each row (rows given by rp)."""
    cs = np.cumsum(vals)
    starts = rp[:-1]
    cnt = np.diff(rp)
    base = np.zeros(len(starts))
    nz = cnt > 0
    base[nz] = cs[starts[nz]] - vals[starts[nz]]
    return cs - np.repeat(base, cnt)


def forward(tr, tr_sun, rho, sigma):
    """y (R,) for one object rho (V,) with cross sections sigma (V,)."""
    rho = np.asarray(rho, np.float64).reshape(-1)
    sigma = np.asarray(sigma, np.float64).reshape(-1)
    s = sigma * rho
    tau1 = _forward(tr_sun, s)
    w = np.exp(-tau1) * rho
    seg_ray, rp, R = _rows(tr)
    vox, ln = tr["vox"], tr["len"]
    T = _row_cumsum(s[vox] * ln, rp)
    return np.bincount(seg_ray, weights=w[vox] * np.exp(-T) * ln, minlength=R)


def gradient(tr, tr_sun, rho, sigma, g):
    """d<g, y(rho)>/d rho (V,) for upstream g (R,)."""
    rho = np.asarray(rho, np.float64).reshape(-1)
    sigma = np.asarray(sigma, np.float64).reshape(-1)
    g = np.asarray(g, np.float64).reshape(-1)
    V = rho.size
    s = sigma * rho
    tau1 = _forward(tr_sun, s)
    e1 = np.exp(-tau1)
    w = e1 * rho
    seg_ray, rp, R = _rows(tr)
    vox, ln = tr["vox"], tr["len"]
    E = np.exp(-_row_cumsum(s[vox] * ln, rp))
    c = w[vox] * E * ln                       # contribution of each segment to y
    suffix = _row_cumsum(c[::-1], np.concatenate([[0], np.cumsum(np.diff(rp)[::-1])]))[::-1]
    gw = np.bincount(vox, weights=g[seg_ray] * E * ln, minlength=V)         # dy/dw
    gs = np.bincount(vox, weights=-g[seg_ray] * ln * suffix, minlength=V)   # dy/ds via T
    gs = gs + _adjoint(tr_sun, -w * gw, V)                                   # via tau_1
    return e1 * gw + sigma * gs
