"""Python face of the projector: geometry, forward, adjoint, autograd.

The HIP library does all the work; this layer converts arrays, picks the
stream and shapes outputs.  PyTorch is used only for device memory and
streams.

    P = Projector(grid, views)                  # steps 1-3 precomputed (TomoSphero Sec. 3, 4.4)
    y = P.forward(rho)                          # Eq. 5, rho: (B, Nr, Ne, Na) float32 on cuda
    x = P.backproject(y)                        # adjoint, deterministic by default
    y = ProjectorFn.apply(rho, P)               # differentiable: backward = adjoint
"""
import ctypes

import numpy as np
import torch

from . import native as N

MODES = {"csr": N.TSP_MODE_CSR, "onthefly": N.TSP_MODE_ONTHEFLY}
ADJ = {"deterministic": N.TSP_ADJ_DETERMINISTIC, "atomic": N.TSP_ADJ_ATOMIC,
       "fixedpoint": N.TSP_ADJ_FIXEDPOINT}


def _grid_arrays(grid):
    if hasattr(grid, "arrays"):
        return tuple(np.ascontiguousarray(a, np.float64) for a in grid.arrays())
    return tuple(np.ascontiguousarray(a, np.float64) for a in grid)


def _view_array(views):
    """tsp_view array from ConeViews / ParallelViews or a list of them (a
    collection of views of any kinds with one detector shape, Sec. 4.3)."""
    stacks = list(views) if isinstance(views, (list, tuple)) else [views]
    items = []
    for st in stacks:
        cone = hasattr(st, "fov_deg")
        ext = st.fov_deg if cone else st.size
        for v in range(st.pos.shape[0]):
            items.append((N.TSP_VIEW_CONE if cone else N.TSP_VIEW_PARALLEL, st.pos[v], st.look[v],
                          st.up[v], ext[v], int(st.H), int(st.W)))
    if len({(it[5], it[6]) for it in items}) != 1:
        raise ValueError("all views of a collection must share one detector shape")
    arr = (N.tsp_view * len(items))()
    for i, (kind, pos, look, up, ext, H, W) in enumerate(items):
        arr[i].kind = kind
        arr[i].shape[:] = [H, W]
        arr[i].pos[:] = [float(a) for a in pos]
        arr[i].look[:] = [float(a) for a in look]
        arr[i].up[:] = [float(a) for a in up]
        arr[i].extent[:] = [float(a) for a in ext]
    return arr, items[0][5], items[0][6]


class Projector:
    """Spherical-grid line-integral projector y = F rho on one GPU.

    grid   Grid (or (r_b, e_b, a_b))
    views  ConeViews (cone beam, detector at the vertex), ParallelViews, or a
           list of them (a collection with one detector shape), or
    rays   (starts, dirs) explicit rays (float64 (R, 3) each; may start inside the grid)
    sun_dir  one ray per voxel from its centroid along sun_dir (Sec. 9.3's F_1);
           its projections are shaped like the grid
    mode   "csr" (precomputed segment lists) or "onthefly" (recomputed per call)
    csc    build the voxel-major store for the deterministic adjoint (csr mode)
    frames dynamic object (Sec. 4.4): object frame of each cone view; objects
           are then (..., F, Nr, Ne, Na) with F = n_frames or max(frames) + 1
    """

    def __init__(self, grid, views=None, rays=None, mode="csr", csc=True, device=None,
                 frames=None, n_frames=None, sun_dir=None):
        if (views is not None) + (rays is not None) + (sun_dir is not None) != 1:
            raise ValueError("give one of views, rays or sun_dir")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        rb, eb, ab = _grid_arrays(grid)
        self.shape = (len(rb) - 1, len(eb) - 1, len(ab) - 1)
        self._keep = (rb, eb, ab)
        gd = N.tsp_grid_desc(self.shape[0], self.shape[1], self.shape[2],
                             rb.ctypes.data_as(N._dp), eb.ctypes.data_as(N._dp),
                             ab.ctypes.data_as(N._dp))
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            if views is not None:
                arr, H, W = _view_array(views)
                N.check(N.lib.tsp_geometry_create_views(ctypes.byref(gd), arr, len(arr),
                                                        ctypes.byref(handle)))
                self.out_shape = (len(arr), H, W)
            elif sun_dir is not None:
                # one sunward ray per voxel centroid (Sec. 9.3, F_1 of Eq. 17)
                sd = np.ascontiguousarray(sun_dir, np.float64).reshape(3)
                N.check(N.lib.tsp_geometry_create_sunward(ctypes.byref(gd),
                                                          sd.ctypes.data_as(N._dp),
                                                          ctypes.byref(handle)))
                self.out_shape = self.shape
            else:
                s = np.ascontiguousarray(rays[0], np.float64).reshape(-1, 3)
                d = np.ascontiguousarray(rays[1], np.float64).reshape(-1, 3)
                if s.shape != d.shape:
                    raise ValueError("starts and dirs must have the same shape")
                N.check(N.lib.tsp_geometry_create(ctypes.byref(gd), None, 0,
                                                  s.ctypes.data_as(N._dp),
                                                  d.ctypes.data_as(N._dp), s.shape[0],
                                                  ctypes.byref(handle)))
                self.out_shape = (s.shape[0],)
        self._h = handle
        self.mode = mode
        self.obj_shape = self.shape
        if frames is not None:
            fr = np.ascontiguousarray(frames, np.int32).reshape(-1)
            F = int(n_frames) if n_frames is not None else int(fr.max()) + 1
            N.check(N.lib.tsp_set_object_frames(
                self._h, fr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), F))
            self.obj_shape = (F, *self.shape)
        self.retrace(mode, csc)

    # ------------------------------------------------------------------ state
    def retrace(self, mode="csr", csc=True):
        m = MODES[mode] | (0 if csc or mode != "csr" else N.TSP_TRACE_NO_CSC)
        with torch.cuda.device(self.device):
            N.check(N.lib.tsp_trace(self._h, m, N.stream_handle()))
        self.mode = mode
        self.csc = mode == "csr" and bool(csc)

    def info(self):
        inf = N.tsp_info()
        N.check(N.lib.tsp_query(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in N.tsp_info._fields_}

    def set_timing_events(self, start, stop):
        """Measurement hook: the next forward or backproject call records
        the torch.cuda.Event pair (timing enabled, on this GPU) around its
        main kernel (tsp_set_timing_events); (None, None) clears it."""
        if (start is None) != (stop is None):
            raise ValueError("start and stop must both be events or both None")
        hs = [None, None]
        if start is not None:
            for i, ev in enumerate((start, stop)):
                if not ev.cuda_event:   # torch creates the handle on first use
                    with torch.cuda.device(self.device):
                        ev.record()
                hs[i] = ctypes.c_void_p(ev.cuda_event)
        N.check(N.lib.tsp_set_timing_events(self._h, hs[0], hs[1]))

    @property
    def n_rays(self):
        return int(np.prod(self.out_shape))

    @property
    def n_voxels(self):
        return int(np.prod(self.shape))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            N.lib.tsp_geometry_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 (interpreter shutdown)
            pass

    # ------------------------------------------------------------------ checks
    def _dev_f32(self, t, name):
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"{name} must be a torch tensor on {self.device}")
        if t.dtype != torch.float32:
            raise ValueError(f"{name} must be float32")
        return t.contiguous()

    # ------------------------------------------------------------------ compute
    def forward(self, rho, out=None):
        """y = F rho.  rho: (..., *obj_shape) float32 on the projector's GPU,
        obj_shape = (Nr, Ne, Na), or (F, Nr, Ne, Na) for a dynamic object.
        Returns (..., *out_shape) float32."""
        rho = self._dev_f32(rho, "rho")
        k = len(self.obj_shape)
        if tuple(rho.shape[rho.dim() - k:]) != self.obj_shape:
            raise ValueError(f"rho must end in {self.obj_shape}, got {tuple(rho.shape)}")
        lead = rho.shape[:rho.dim() - k]
        B = int(np.prod(lead)) if lead else 1
        y = out if out is not None else torch.empty((*lead, *self.out_shape),
                                                    dtype=torch.float32, device=self.device)
        if B:
            N.check(N.lib.tsp_forward(self._h, N.ptr(rho), B, N.ptr(y), N.stream_handle()))
        return y

    def backproject(self, y, method=None, out=None):
        """x = F^T y.  y: (..., *out_shape) float32.

        method: "deterministic" (bitwise reproducible; from the voxel-major
        store when the lists are stored with it, else traced chunk by chunk
        within the call, which costs a full trace), "atomic", "fixedpoint"
        (bitwise reproducible: traced within the call, sums in 64-bit fixed
        point, one pass), or None: the stored deterministic adjoint when there
        is one, else the atomic one."""
        y = self._dev_f32(y, "y")
        k = len(self.out_shape)
        if tuple(y.shape[y.dim() - k:]) != self.out_shape:
            raise ValueError(f"y must end in {self.out_shape}, got {tuple(y.shape)}")
        lead = y.shape[:y.dim() - k]
        B = int(np.prod(lead)) if lead else 1
        x = out if out is not None else torch.empty((*lead, *self.obj_shape),
                                                    dtype=torch.float32, device=self.device)
        if method is None:
            method = "deterministic" if self.csc else "atomic"
        if B:
            N.check(N.lib.tsp_backproject(self._h, N.ptr(y), B, N.ptr(x), ADJ[method],
                                          N.stream_handle()))
        return x

    __call__ = forward

    def segments(self):
        """Canonical per-ray segment lists (Sec. 4.4 .regs/.lens) as CSR:
        row_ptr int64 (R+1), vox int32 (S), len float32 (S)."""
        inf = self.info()
        S = inf["n_segments"]
        rp = torch.empty(self.n_rays + 1, dtype=torch.int64, device=self.device)
        vox = torch.empty(max(S, 1), dtype=torch.int32, device=self.device)
        ln = torch.empty(max(S, 1), dtype=torch.float32, device=self.device)
        N.check(N.lib.tsp_segments(self._h, N.ptr(rp), N.ptr(vox), N.ptr(ln), N.stream_handle()))
        return rp, vox[:S], ln[:S]

    def rays(self):
        """(starts, unit dirs) float64 (R, 3) as traced by the kernels."""
        s = torch.empty((self.n_rays, 3), dtype=torch.float64, device=self.device)
        d = torch.empty((self.n_rays, 3), dtype=torch.float64, device=self.device)
        N.check(N.lib.tsp_rays(self._h, N.ptr(s), N.ptr(d), N.stream_handle()))
        return s, d


class ProjectorFn(torch.autograd.Function):
    """Differentiable y = F rho.  F is linear, so the gradient with respect
    to rho is F^T grad_y, computed by the hand-written adjoint kernel; autograd
    never sees the ray tracer."""

    @staticmethod
    def forward(ctx, rho, proj, method=None):
        ctx.proj = proj
        ctx.method = method
        return proj.forward(rho)

    @staticmethod
    def backward(ctx, gy):
        gx = ctx.proj.backproject(gy.contiguous(), method=ctx.method)
        return gx, None, None
