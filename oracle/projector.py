"""ctypes front-end of the C FP64 oracle (test infrastructure only).

Every function takes plain numpy arrays:
  grid  = (r_b, e_b, a_b) float64 boundary arrays (TomoSphero Sec. 2.2, Sec. 4.1)
  views = pos (V,3), look (V,3), up (V,3), fov_deg (V,2) = (fov_h, fov_w), H, W
          (cone beam with the detector at the vertex, Sec. 4.2 / Sec. 4.6)
  rays  = starts (R,3), dirs (R,3) (explicit rays as in Listing 4; directions
          need not be unit length).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def load_library():
    """Load ``liboracle.so``, building it with gcc when it is missing.  The
    environment variable TSP_ORACLE_LIB names another build of the same
    source instead (the sanitised build of the host-side checks)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.environ.get("TSP_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
    if not os.path.exists(path):
        from . import build as _b  # noqa: WPS433
        _b.build()
    lib = ctypes.CDLL(path)
    lib.ora_num_threads.restype = ctypes.c_int
    lib.ora_set_num_threads.restype = None
    lib.ora_set_num_threads.argtypes = [ctypes.c_int]
    lib.ora_cone_rays.restype = None
    lib.ora_cone_rays.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int,
                                  _dp, _dp]
    grid_args = [_dp, ctypes.c_int, _dp, ctypes.c_int, _dp, ctypes.c_int]
    lib.ora_count.restype = ctypes.c_int
    lib.ora_count.argtypes = grid_args + [_dp, _dp, ctypes.c_int64, _i32p, _u8p]
    lib.ora_fill.restype = ctypes.c_int
    lib.ora_fill.argtypes = grid_args + [_dp, _dp, ctypes.c_int64, _i64p, _i32p, _dp, _dp]
    lib.ora_forward.restype = None
    lib.ora_forward.argtypes = [_i64p, _i32p, _dp, ctypes.c_int64, _dp, ctypes.c_int,
                                ctypes.c_int64, _dp]
    lib.ora_adjoint.restype = None
    lib.ora_adjoint.argtypes = [_i64p, _i32p, _dp, ctypes.c_int64, _dp, ctypes.c_int,
                                ctypes.c_int64, _dp]
    lib.ora_project.restype = ctypes.c_int
    lib.ora_project.argtypes = grid_args + [_dp, _dp, ctypes.c_int64, _dp, ctypes.c_int, _dp,
                                            _i64p]
    lib.ora_cone_ray_ids.restype = None
    lib.ora_cone_ray_ids.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int,
                                     _i64p, ctypes.c_int64, _dp, _dp]
    lib.ora_cone_data_grad.restype = ctypes.c_int
    lib.ora_cone_data_grad.argtypes = grid_args + [ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_int,
                                                   ctypes.c_int, _dp, _dp, ctypes.c_int, _i64p,
                                                   _dp, _dp, _dp, _i64p]
    _LIB = lib
    return lib


def _p(a, ptr):
    return a.ctypes.data_as(ptr)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(load_library().ora_num_threads())


def set_num_threads(n: int) -> None:
    load_library().ora_set_num_threads(int(n))


def cone_rays(pos, look, up, fov_deg, H, W):
    """Rays of a stack of cone-beam views; ray id = (view*H + i)*W + j."""
    lib = load_library()
    pos, look, up, fov = _f64(pos), _f64(look), _f64(up), _f64(fov_deg)
    nv = pos.shape[0]
    R = nv * H * W
    starts = np.empty((R, 3), np.float64)
    dirs = np.empty((R, 3), np.float64)
    lib.ora_cone_rays(nv, _p(pos, _dp), _p(look, _dp), _p(up, _dp), _p(fov, _dp), int(H), int(W),
                      _p(starts, _dp), _p(dirs, _dp))
    return starts, dirs


def cone_ray_ids(pos, look, up, fov_deg, H, W, ids):
    """Rays with the given ids of a stack of cone views (as cone_rays)."""
    lib = load_library()
    pos, look, up, fov = _f64(pos), _f64(look), _f64(up), _f64(fov_deg)
    ids = np.ascontiguousarray(ids, np.int64)
    starts = np.empty((len(ids), 3))
    dirs = np.empty((len(ids), 3))
    lib.ora_cone_ray_ids(pos.shape[0], _p(pos, _dp), _p(look, _dp), _p(up, _dp), _p(fov, _dp),
                         int(H), int(W), _p(ids, _i64p), len(ids), _p(starts, _dp), _p(dirs, _dp))
    return starts, dirs


def _grid_args(grid):
    rb, eb, ab = (_f64(g) for g in grid)
    return (rb, eb, ab), [_p(rb, _dp), len(rb) - 1, _p(eb, _dp), len(eb) - 1, _p(ab, _dp),
                          len(ab) - 1]


def trace(grid, starts, dirs):
    """Canonical segment lists of every ray.

    Returns a dict with row_ptr (R+1,) int64, vox (S,) int32 linear index
    (ir*Ne + ie)*Na + ia, len (S,) float64, t0 (S,) float64 segment start
    distance, tie (R,) bool (index list not decided robustly in FP64),
    sensitive (R,) bool (lengths ill-conditioned beyond FP32 rounding; implied
    by tie), counts (R,) int32.
    """
    lib = load_library()
    keep, gargs = _grid_args(grid)
    starts, dirs = _f64(starts), _f64(dirs)
    R = starts.shape[0]
    counts = np.empty(R, np.int32)
    ties = np.empty(R, np.uint8)
    err = lib.ora_count(*gargs, _p(starts, _dp), _p(dirs, _dp), R, _p(counts, _i32p),
                        _p(ties, _u8p))
    if err:
        raise MemoryError("oracle count failed")
    row_ptr = np.zeros(R + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    S = int(row_ptr[-1])
    vox = np.empty(max(S, 1), np.int32)
    ln = np.empty(max(S, 1), np.float64)
    t0 = np.empty(max(S, 1), np.float64)
    err = lib.ora_fill(*gargs, _p(starts, _dp), _p(dirs, _dp), R, _p(row_ptr, _i64p),
                       _p(vox, _i32p), _p(ln, _dp), _p(t0, _dp))
    if err:
        raise RuntimeError(f"oracle fill failed ({err})")
    del keep
    return dict(row_ptr=row_ptr, vox=vox[:S], len=ln[:S], t0=t0[:S], tie=(ties & 1) > 0,
                sensitive=(ties & 2) > 0, counts=counts)


def forward(tr, rho):
    """y[b, i] = sum_k len_k rho[b, vox_k] over the row of ray i (Eq. 5), FP64.

    rho: (V,) or (B, V) (any trailing shape flattened per batch)."""
    lib = load_library()
    rho = np.asarray(rho, np.float64)
    single = rho.ndim == 1 or (rho.ndim == 3)
    rho2 = np.ascontiguousarray(rho.reshape(1, -1) if single else rho.reshape(rho.shape[0], -1))
    B, V = rho2.shape
    R = len(tr["row_ptr"]) - 1
    y = np.empty((B, R), np.float64)
    vox = np.ascontiguousarray(tr["vox"], np.int32)
    ln = _f64(tr["len"])
    rp = np.ascontiguousarray(tr["row_ptr"], np.int64)
    if vox.size == 0:
        vox, ln = np.zeros(1, np.int32), np.zeros(1)
    lib.ora_forward(_p(rp, _i64p), _p(vox, _i32p), _p(ln, _dp), R, _p(rho2, _dp), B, V,
                    _p(y, _dp))
    return y[0] if single else y


def adjoint(tr, y, V):
    """x[b, v] = sum of len_k y[b, ray_k] over the segments of voxel v, FP64."""
    lib = load_library()
    y = np.asarray(y, np.float64)
    single = y.ndim == 1
    y2 = np.ascontiguousarray(y.reshape(1, -1) if single else y.reshape(y.shape[0], -1))
    B, R = y2.shape
    assert R == len(tr["row_ptr"]) - 1
    x = np.empty((B, V), np.float64)
    vox = np.ascontiguousarray(tr["vox"], np.int32)
    ln = _f64(tr["len"])
    rp = np.ascontiguousarray(tr["row_ptr"], np.int64)
    if vox.size == 0:
        vox, ln = np.zeros(1, np.int32), np.zeros(1)
    lib.ora_adjoint(_p(rp, _i64p), _p(vox, _i32p), _p(ln, _dp), R, _p(y2, _dp), B, int(V),
                    _p(x, _dp))
    return x[0] if single else x


def project(grid, starts, dirs, rho):
    """Fused trace + forward without storing segments (same arithmetic as
    trace() then forward()); returns (y (B, R), total segment count)."""
    lib = load_library()
    keep, gargs = _grid_args(grid)
    starts, dirs = _f64(starts), _f64(dirs)
    rho = np.asarray(rho, np.float64)
    rho2 = np.ascontiguousarray(rho.reshape(rho.shape[0], -1) if rho.ndim in (2, 4)
                                else rho.reshape(1, -1))
    B = rho2.shape[0]
    R = starts.shape[0]
    y = np.empty((B, R), np.float64)
    tot = ctypes.c_int64(0)
    err = lib.ora_project(*gargs, _p(starts, _dp), _p(dirs, _dp), R, _p(rho2, _dp), B, _p(y, _dp),
                          ctypes.byref(tot))
    if err:
        raise MemoryError("oracle project failed")
    del keep
    return y, int(tot.value)


def voxel_bounding_spheres(grid, targets):
    """Conservative bounding sphere (centre, radius) of each target voxel:
    5x5x5 samples over its (r, colatitude, azimuth) box, radius x 1.1."""
    rb, eb, ab = (np.asarray(a, np.float64) for a in grid)
    ne, na = len(eb) - 1, len(ab) - 1
    out = np.empty((len(targets), 4))
    s = np.linspace(0.0, 1.0, 5)
    for n, v in enumerate(targets):
        ir, ie, ia = v // (ne * na), (v // na) % ne, v % na
        r = rb[ir] + s * (rb[ir + 1] - rb[ir])
        th = eb[ie] + s * (eb[ie + 1] - eb[ie])
        ph = ab[ia] + s * (ab[ia + 1] - ab[ia])
        R, T, Ph = np.meshgrid(r, th, ph, indexing="ij")
        P = np.stack([R * np.sin(T) * np.cos(Ph), R * np.sin(T) * np.sin(Ph), R * np.cos(T)],
                     -1).reshape(-1, 3)
        c = P.mean(0)
        out[n, :3] = c
        out[n, 3] = 1.1 * np.sqrt(((P - c) ** 2).sum(1)).max() + 1e-9
    return out


def cone_data_grad(grid, pos, look, up, fov_deg, H, W, rho, y, targets):
    """Gradient of ||F rho - y||^2 at the target voxels for cone views, FP64,
    rays generated and traced on the fly (no segment storage).  Returns
    (grad, bound, rays traced); bound scales the FP32 rounding of the same
    quantity (2 sum_i (sum_k |rho| len + |y_i|) len_iv)."""
    lib = load_library()
    keep, gargs = _grid_args(grid)
    pos, look, up, fov = _f64(pos), _f64(look), _f64(up), _f64(fov_deg)
    rho = _f64(np.asarray(rho).reshape(-1))
    y = _f64(np.asarray(y).reshape(-1))
    t = np.ascontiguousarray(targets, np.int64)
    bs = _f64(voxel_bounding_spheres(grid, t))
    g = np.empty(len(t))
    b = np.empty(len(t))
    n = ctypes.c_int64(0)
    err = lib.ora_cone_data_grad(*gargs, pos.shape[0], _p(pos, _dp), _p(look, _dp), _p(up, _dp),
                                 _p(fov, _dp), int(H), int(W), _p(rho, _dp), _p(y, _dp), len(t),
                                 _p(t, _i64p), _p(bs, _dp), _p(g, _dp), _p(b, _dp), ctypes.byref(n))
    if err:
        raise MemoryError("oracle data gradient failed")
    del keep
    return g, b, int(n.value)
