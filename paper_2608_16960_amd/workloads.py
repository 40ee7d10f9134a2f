"""Seeded synthetic inputs: grids, cone-beam orbits and phantoms.

This module produces input arrays only.  It holds none of the projector's
arithmetic (no ray generation, no intersections), so that the HIP path and the
CPU oracle can both be fed from it without sharing code.

Workloads (the paper's own exosphere data is not available; these stand in):

  tiny      20 log-spaced shells r in [3, 25] x 10 colatitude bins over
            [0, pi] x 12 azimuth bins; 4 views 32x32, FOV 30 deg, circular
            equatorial orbit of radius 50; rho = exp(-(r - 3)/4) + N(0, 0.01^2)
  medium    50 x 50 x 50 (linear r in [3, 25]); 30 views 256x256, FOV 20 deg,
            circular orbit of radius 40 inclined 30 deg about +X; rho = exp
            background + 5 Gaussian blobs
  diff      100 x 60 x 120; 100 views 512x512, FOV 50 deg, radius-60 circular
            orbit with a seeded random inclination
  learned   64 x 32 x 64; 64 views 256x256, FOV 50 deg, radius-60 orbit with a
            seeded random inclination; phantoms exp(-(r-3)/s), s ~ U[2, 6],
            plus 1..8 Gaussian plumes
  large     200 x 90 x 180; 180 views 512x512, FOV 50 deg, elliptical orbit
            (apoapsis 80, periapsis 30) uniform in mean anomaly; batch of 4

Voxel centroids (used to sample phantoms) are the arithmetic mid-boundaries
(r_c, theta_c, phi_c) mapped to Cartesian.  All views look at the origin with
+Z as the up hint.
"""
from dataclasses import dataclass, field
from typing import Tuple

import numpy as np

TWO_PI = 2.0 * np.pi


@dataclass
class Grid:
    """Boundary arrays of a spherical grid (r_b: Nr+1, e_b: Ne+1, a_b: Na+1)."""
    r_b: np.ndarray
    e_b: np.ndarray
    a_b: np.ndarray

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (len(self.r_b) - 1, len(self.e_b) - 1, len(self.a_b) - 1)

    @property
    def size(self) -> int:
        nr, ne, na = self.shape
        return nr * ne * na

    def arrays(self):
        return (self.r_b, self.e_b, self.a_b)


@dataclass
class ConeViews:
    """A stack of equal-shape cone-beam views (detector at the vertex)."""
    pos: np.ndarray          # (V, 3)
    look: np.ndarray         # (V, 3) point the optical axis passes through
    up: np.ndarray           # (V, 3) up hint
    fov_deg: np.ndarray      # (V, 2) full angles (along rows H, along columns W)
    H: int
    W: int

    @property
    def n_views(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_rays(self) -> int:
        return self.n_views * self.H * self.W


@dataclass
class ParallelViews:
    """A stack of equal-shape parallel-beam views (ParallelGeom, Sec. 4.2):
    rays start on the detector rectangle (centre pos, `size` = (height,
    width) in grid units) and all run along unit(look - pos)."""
    pos: np.ndarray          # (V, 3)
    look: np.ndarray         # (V, 3)
    up: np.ndarray           # (V, 3)
    size: np.ndarray         # (V, 2)
    H: int
    W: int

    @property
    def n_views(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_rays(self) -> int:
        return self.n_views * self.H * self.W


def parallel_views_at(pos, size, H, W, look=None, up=None) -> ParallelViews:
    c = views_at(pos, (1.0, 1.0), H, W, look, up)
    sz = np.broadcast_to(np.asarray(size, np.float64), (c.n_views, 2)).copy()
    return ParallelViews(c.pos, c.look, c.up, sz, int(H), int(W))


@dataclass
class Workload:
    name: str
    grid: Grid
    views: ConeViews
    rho: np.ndarray                      # (B, Nr, Ne, Na) float32
    mode: str = "csr"
    extra: dict = field(default_factory=dict)


def uniform_grid(shape, r=(3.0, 25.0), e=(0.0, np.pi), a=(0.0, TWO_PI), log_r=False) -> Grid:
    nr, ne, na = shape
    rb = np.geomspace(r[0], r[1], nr + 1) if log_r else np.linspace(r[0], r[1], nr + 1)
    return Grid(rb.astype(np.float64), np.linspace(e[0], e[1], ne + 1),
                np.linspace(a[0], a[1], na + 1))


def views_at(pos, fov_deg, H, W, look=None, up=None) -> ConeViews:
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    V = pos.shape[0]
    look = np.zeros((V, 3)) if look is None else np.broadcast_to(np.asarray(look, np.float64),
                                                                 (V, 3)).copy()
    up = np.tile([0.0, 0.0, 1.0], (V, 1)) if up is None else np.broadcast_to(
        np.asarray(up, np.float64), (V, 3)).copy()
    fov = np.broadcast_to(np.asarray(fov_deg, np.float64), (V, 2)).copy()
    return ConeViews(pos, look, up, fov, int(H), int(W))


def _rot_x(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])


def _rot_z(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def circular_orbit(n, radius, incl=0.0, node=0.0):
    """n positions at phases 2 pi v / n (endpoint excluded) on a circle of the
    given radius, orbit plane rotated by `incl` about +X then by `node` about +Z."""
    ph = TWO_PI * np.arange(n) / n
    p = np.stack([radius * np.cos(ph), radius * np.sin(ph), np.zeros(n)], 1)
    Rm = _rot_z(node) @ _rot_x(incl)
    return p @ Rm.T


def elliptical_orbit(n, apo, peri, rng):
    """n positions uniform in mean anomaly on an ellipse with a focus at the
    origin; orientation (i, Omega, omega) drawn from rng."""
    a = 0.5 * (apo + peri)
    e = (apo - peri) / (apo + peri)
    M = TWO_PI * np.arange(n) / n
    E = M.copy()
    for _ in range(50):  # Kepler's equation by Newton's method
        E = E - (E - e * np.sin(E) - M) / (1 - e * np.cos(E))
    xo = a * (np.cos(E) - e)
    yo = a * np.sqrt(1 - e * e) * np.sin(E)
    p = np.stack([xo, yo, np.zeros(n)], 1)
    inc, node, argp = rng.uniform(0, np.pi), rng.uniform(0, TWO_PI), rng.uniform(0, TWO_PI)
    Rm = _rot_z(node) @ _rot_x(inc) @ _rot_z(argp)
    return p @ Rm.T


def centroids(grid: Grid):
    """Cartesian voxel centroids (arithmetic mid-boundaries), shape (Nr,Ne,Na,3)."""
    rc = 0.5 * (grid.r_b[1:] + grid.r_b[:-1])
    tc = 0.5 * (grid.e_b[1:] + grid.e_b[:-1])
    pc = 0.5 * (grid.a_b[1:] + grid.a_b[:-1])
    R, T, P = np.meshgrid(rc, tc, pc, indexing="ij")
    return np.stack([R * np.sin(T) * np.cos(P), R * np.sin(T) * np.sin(P), R * np.cos(T)], -1), R


def exp_background(grid: Grid, scale=4.0):
    _, R = centroids(grid)
    return np.exp(-(R - 3.0) / scale)


def blob_phantom(grid: Grid, rng, n_blobs=5, scale=4.0, amp=(0.5, 2.0), width=(1.0, 3.0),
                 r_mu=(5.0, 20.0), cent=None):
    """exp(-(r-3)/scale) plus Gaussian blobs A exp(-|x - mu|^2 / (2 w^2)).
    cent: precomputed centroids(grid), to reuse across many phantoms."""
    X, R = centroids(grid) if cent is None else cent
    rho = np.exp(-(R - 3.0) / scale)
    R2 = R * R  # |x|^2 at the centroids
    for _ in range(n_blobs):
        A = rng.uniform(*amp)
        w = rng.uniform(*width)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        mu = rng.uniform(*r_mu) * u
        d2 = np.maximum(R2 - 2.0 * (X @ mu) + mu @ mu, 0.0)  # |x - mu|^2
        rho += A * np.exp(-d2 / (2 * w * w))
    return rho


def plume_phantom(grid: Grid, rng, cent=None):
    """Learned-workload phantom: exp(-(r-3)/s), s ~ U[2,6], + K ~ U{1..8} plumes."""
    s = rng.uniform(2.0, 6.0)
    k = int(rng.integers(1, 9))
    return blob_phantom(grid, rng, n_blobs=k, scale=s, cent=cent)


def tiny(noise_seed=0, noise=0.01) -> Workload:
    g = uniform_grid((20, 10, 12), log_r=True)
    v = views_at(circular_orbit(4, 50.0), (30.0, 30.0), 32, 32)
    rng = np.random.default_rng(noise_seed)
    rho = exp_background(g) + (noise * rng.normal(size=g.shape) if noise else 0.0)
    return Workload("tiny", g, v, rho[None].astype(np.float32), "csr")


def medium(seed=1) -> Workload:
    g = uniform_grid((50, 50, 50))
    v = views_at(circular_orbit(30, 40.0, incl=np.deg2rad(30.0)), (20.0, 20.0), 256, 256)
    rho = blob_phantom(g, np.random.default_rng(seed))
    return Workload("medium", g, v, rho[None].astype(np.float32), "csr")


def diff(orbit_seed=2, truth_seed=3) -> Workload:
    g = uniform_grid((100, 60, 120))
    r = np.random.default_rng(orbit_seed)
    v = views_at(circular_orbit(100, 60.0, incl=r.uniform(0, np.pi), node=r.uniform(0, TWO_PI)),
                 (50.0, 50.0), 512, 512)
    rho = blob_phantom(g, np.random.default_rng(truth_seed))
    return Workload("diff", g, v, rho[None].astype(np.float32), "csr")


def learned_geometry(orbit_seed=5, n_views=64, det=256):
    g = uniform_grid((64, 32, 64))
    r = np.random.default_rng(orbit_seed)
    v = views_at(circular_orbit(n_views, 60.0, incl=r.uniform(0, np.pi),
                                node=r.uniform(0, TWO_PI)), (50.0, 50.0), det, det)
    return g, v


def learned_phantoms(grid: Grid, n, seed):
    rng = np.random.default_rng(seed)
    cent = centroids(grid)
    out = np.empty((n, *grid.shape), np.float32)
    for i in range(n):
        out[i] = plume_phantom(grid, rng, cent)
    return out


def large(orbit_seed=9, obj_seeds=(10, 11, 12, 13)) -> Workload:
    g = uniform_grid((200, 90, 180))
    v = views_at(elliptical_orbit(180, 80.0, 30.0, np.random.default_rng(orbit_seed)),
                 (50.0, 50.0), 512, 512)
    rho = np.stack([blob_phantom(g, np.random.default_rng(s)) for s in obj_seeds])
    return Workload("large", g, v, rho.astype(np.float32), "onthefly")


def random_rays(n, rng, r_start=(30.0, 60.0), aim=8.0):
    """Explicit rays (Listing 4 style): starts on a sphere of random radius,
    directions towards a random point near the origin, left un-normalised."""
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    starts = u * rng.uniform(*r_start, size=(n, 1))
    target = rng.uniform(-aim, aim, size=(n, 3))
    dirs = (target - starts) * rng.uniform(0.2, 3.0, size=(n, 1))
    return starts, dirs
