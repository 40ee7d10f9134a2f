"""Error paths of the C ABI that need a device: state errors, the device-memory
cap (TSP_MAX_DEVICE_BYTES) with the on-the-fly fallback, unsupported
combinations.  Every case returns an error code; no kernel is made to fail.
Also the timing hook (tsp_set_timing_events): the events bracket the main
kernel only, once, and leave the results as they are."""
import ctypes
import os

import numpy as np
import pytest
import torch

from paper_2608_16960_amd import workloads as W

pytestmark = pytest.mark.gpu


def _geometry(N, w):
    g = w.grid
    arrs = [np.ascontiguousarray(a, np.float64) for a in g.arrays()]
    gd = N.tsp_grid_desc(*g.shape, *[a.ctypes.data_as(N._dp) for a in arrs])
    v = w.views
    views = (N.tsp_cone_view * v.n_views)()
    for i in range(v.n_views):
        views[i].pos[:] = list(v.pos[i])
        views[i].look[:] = list(v.look[i])
        views[i].up[:] = list(v.up[i])
        views[i].fov_deg[:] = list(v.fov_deg[i])
        views[i].shape[:] = [v.H, v.W]
    h = ctypes.c_void_p()
    assert N.lib.tsp_geometry_create(ctypes.byref(gd), views, v.n_views, None, None, 0,
                                     ctypes.byref(h)) == N.TSP_OK
    return h, arrs


def test_state_and_capacity_errors():
    assert torch.cuda.is_available()
    from paper_2608_16960_amd import native as N
    w = W.tiny()
    h, keep = _geometry(N, w)
    rho = torch.from_numpy(w.rho).cuda()
    y = torch.empty(w.views.n_rays, device="cuda")
    x = torch.empty(w.grid.size, device="cuda")
    s = N.stream_handle()
    try:
        assert N.lib.tsp_forward(h, N.ptr(rho), 1, N.ptr(y), s) == N.TSP_E_STATE
        assert N.lib.tsp_backproject(h, N.ptr(y), 1, N.ptr(x), N.TSP_ADJ_ATOMIC, s) == \
            N.TSP_E_STATE
        assert N.lib.tsp_forward(h, N.ptr(rho), 0, N.ptr(y), s) == N.TSP_E_INVALID
        os.environ["TSP_MAX_DEVICE_BYTES"] = str(200_000)  # below the segment store
        try:
            assert N.lib.tsp_trace(h, N.TSP_MODE_CSR, s) == N.TSP_E_NOMEM
            assert b"TSP_MAX_DEVICE_BYTES" in N.lib.tsp_last_error()
            assert N.lib.tsp_trace(h, N.TSP_MODE_ONTHEFLY, s) == N.TSP_OK
        finally:
            del os.environ["TSP_MAX_DEVICE_BYTES"]
        assert N.lib.tsp_forward(h, N.ptr(rho), 1, N.ptr(y), s) == N.TSP_OK
        # on the fly, the deterministic adjoint is traced chunk by chunk in the call
        assert N.lib.tsp_backproject(h, N.ptr(y), 1, N.ptr(x), N.TSP_ADJ_DETERMINISTIC, s) == \
            N.TSP_OK
        xd = x.clone()
        assert N.lib.tsp_backproject(h, N.ptr(y), 1, N.ptr(x), N.TSP_ADJ_ATOMIC, s) == N.TSP_OK
        assert torch.allclose(x, xd, rtol=1e-5, atol=1e-5)
        rp = torch.empty(w.views.n_rays + 1, dtype=torch.int64, device="cuda")
        assert N.lib.tsp_segments(h, N.ptr(rp), None, None, s) == N.TSP_E_STATE
        assert N.lib.tsp_backproject(h, N.ptr(y), 1, N.ptr(x), 7, s) == N.TSP_E_INVALID
        info = N.tsp_info()
        assert N.lib.tsp_query(h, ctypes.byref(info)) == N.TSP_OK
        assert info.mode == N.TSP_MODE_ONTHEFLY and info.n_segments > 0 and info.has_csc == 0
        # switch back to stored lists without the transposed store: the
        # deterministic adjoint is then traced in the call as well
        assert N.lib.tsp_trace(h, N.TSP_MODE_CSR | N.TSP_TRACE_NO_CSC, s) == N.TSP_OK
        assert N.lib.tsp_backproject(h, N.ptr(y), 1, N.ptr(x), N.TSP_ADJ_DETERMINISTIC, s) == \
            N.TSP_OK
        assert torch.equal(x, xd)
        torch.cuda.synchronize()
    finally:
        N.lib.tsp_geometry_destroy(h)


def test_projector_falls_back_to_onthefly_adjoint():
    """By default the Python layer uses the atomic adjoint in on-the-fly mode."""
    from paper_2608_16960_amd.projector import Projector
    w = W.tiny()
    P = Projector(w.grid, views=w.views, mode="onthefly")
    y = P.forward(torch.from_numpy(w.rho).cuda())
    x = P.backproject(y)  # no error: switches to the atomic adjoint
    assert torch.isfinite(x).all() and float(x.abs().sum()) > 0


def test_object_frame_errors():
    """tsp_set_object_frames: frame index out of range, too many frames,
    after tsp_trace (state), and on explicit rays (unsupported)."""
    assert torch.cuda.is_available()
    from paper_2608_16960_amd import native as N
    w = W.tiny()
    h, keep = _geometry(N, w)
    I32 = ctypes.c_int32 * w.views.n_views
    s = N.stream_handle()
    try:
        assert N.lib.tsp_set_object_frames(h, I32(0, 1, 2, 3), 3) == N.TSP_E_INVALID
        assert N.lib.tsp_set_object_frames(h, I32(0, 0, -1, 0), 2) == N.TSP_E_INVALID
        assert N.lib.tsp_set_object_frames(h, I32(0, 0, 0, 0), 0) == N.TSP_E_INVALID
        assert N.lib.tsp_set_object_frames(h, I32(0, 0, 0, 0), 1 << 30) == N.TSP_E_INVALID
        assert N.lib.tsp_set_object_frames(h, I32(0, 1, 1, 0), 2) == N.TSP_OK
        assert N.lib.tsp_set_object_frames(h, I32(1, 0, 1, 0), 2) == N.TSP_OK  # replace
        assert N.lib.tsp_trace(h, N.TSP_MODE_CSR, s) == N.TSP_OK
        inf = N.tsp_info()
        assert N.lib.tsp_query(h, ctypes.byref(inf)) == N.TSP_OK and inf.n_obj_frames == 2
        assert N.lib.tsp_set_object_frames(h, I32(0, 0, 0, 0), 1) == N.TSP_E_STATE
    finally:
        N.lib.tsp_geometry_destroy(h)
    g = w.grid
    arrs = [np.ascontiguousarray(a, np.float64) for a in g.arrays()]
    gd = N.tsp_grid_desc(*g.shape, *[a.ctypes.data_as(N._dp) for a in arrs])
    st, di = W.random_rays(10, np.random.default_rng(0))
    st, di = np.ascontiguousarray(st), np.ascontiguousarray(di)
    h2 = ctypes.c_void_p()
    assert N.lib.tsp_geometry_create(ctypes.byref(gd), None, 0, st.ctypes.data_as(N._dp),
                                     di.ctypes.data_as(N._dp), 10, ctypes.byref(h2)) == N.TSP_OK
    try:
        assert N.lib.tsp_set_object_frames(h2, (ctypes.c_int32 * 1)(0), 1) == \
            N.TSP_E_UNSUPPORTED
    finally:
        N.lib.tsp_geometry_destroy(h2)


def test_timing_events_bracket_the_main_kernel():
    """Medium workload, batch 1, stored lists.  The kernel's own time lies
    inside the call's (torch events on the same stream around the call), the
    events are recorded by one call only, and the results are bitwise those
    of calls without events.  On the fly they bracket the whole launch."""
    from paper_2608_16960_amd import native as N
    from paper_2608_16960_amd.projector import Projector
    w = W.medium()
    P = Projector(w.grid, views=w.views)
    rho = torch.from_numpy(w.rho[:1]).cuda()
    y0 = P.forward(rho)
    x0 = P.backproject(y0, "deterministic")

    def ev():
        return torch.cuda.Event(enable_timing=True)

    try:
        for op in ("forward", "adjoint"):
            ks, ke, cs, ce = ev(), ev(), ev(), ev()
            P.set_timing_events(ks, ke)
            cs.record()
            out = P.forward(rho) if op == "forward" else P.backproject(y0, "deterministic")
            ce.record()
            torch.cuda.synchronize()
            assert torch.equal(out, y0 if op == "forward" else x0)
            tk, tc = ks.elapsed_time(ke), cs.elapsed_time(ce)
            print(op, "kernel", tk, "call", tc, flush=True)
            assert 0 < tk <= tc
            # one-shot: the next call records nothing
            P.backproject(y0, "deterministic")
            torch.cuda.synchronize()
            assert ks.elapsed_time(ke) == tk
        # half a pair is refused, on the ABI and in the binding
        h = ks.cuda_event
        assert N.lib.tsp_set_timing_events(P._h, ctypes.c_void_p(h), None) == N.TSP_E_INVALID
        with pytest.raises(ValueError):
            P.set_timing_events(ks, None)
        # set and cleared: nothing recorded
        P.set_timing_events(ks, ke)
        P.set_timing_events(None, None)
        P.forward(rho)
        torch.cuda.synchronize()
        assert ks.elapsed_time(ke) == tk
        # on the fly: the events bracket the whole launch
        P.retrace("onthefly")
        ks, ke = ev(), ev()
        P.set_timing_events(ks, ke)
        yo = P.forward(rho)
        torch.cuda.synchronize()
        assert ks.elapsed_time(ke) > 0
        assert float((yo - y0).abs().max()) <= 1e-5 * float(y0.abs().max())
    finally:
        P.close()
