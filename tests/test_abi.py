"""The C-ABI libraries load and export every symbol their headers declare;
host-side argument validation fails before touching any GPU (runs on CPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2608_16960_amd")
DECL = re.compile(r"^\s*(?:[A-Za-z_][\w\s]*?[\s\*]+)(tsp\w+)\s*\(", re.M)


def _declared(header):
    with open(os.path.join(ROOT, "include", header)) as f:
        txt = f.read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(DECL.findall(txt)))


@pytest.mark.parametrize("header,lib", [("tsp.h", "libtsp.so"), ("tspnn.h", "libtspnn.so")])
def test_library_exports_every_declared_symbol(header, lib):
    if not os.path.exists(os.path.join(ROOT, "include", header)):
        pytest.skip(f"{header} not present")
    names = _declared(header)
    assert len(names) >= 5
    so = ctypes.CDLL(os.path.join(PKG, lib))
    missing = [n for n in names if not hasattr(so, n)]
    assert not missing, f"{lib} lacks {missing}"


def test_binding_names_match_header():
    from paper_2608_16960_amd import native as N
    assert sorted(N.SIGNATURES) == _declared("tsp.h")


def _grid(rb=(1.0, 2.0), eb=(0.0, np.pi), ab=(0.0, 2 * np.pi)):
    from paper_2608_16960_amd import native as N
    arrs = [np.asarray(a, np.float64) for a in (rb, eb, ab)]
    gd = N.tsp_grid_desc(len(rb) - 1, len(eb) - 1, len(ab) - 1,
                         *[a.ctypes.data_as(N._dp) for a in arrs])
    return gd, arrs


def _view(pos=(10.0, 0.0, 0.0), fov=(30.0, 30.0), shape=(4, 4)):
    from paper_2608_16960_amd import native as N
    v = N.tsp_cone_view()
    v.pos[:] = pos
    v.look[:] = (0.0, 0.0, 0.0)
    v.up[:] = (0.0, 0.0, 0.0)
    v.fov_deg[:] = fov
    v.shape[:] = shape
    return v


@pytest.mark.parametrize("case", ["null_grid", "rb_not_increasing", "eb_out_of_range",
                                  "ab_span", "detector_inside", "fov", "both_sources",
                                  "ray_nan", "zero_dir", "shape_mismatch",
                                  "tables_exceed_lds"])
def test_create_validation(case):
    from paper_2608_16960_amd import native as N
    out = ctypes.c_void_p()
    gd, keep = _grid()
    views = (N.tsp_cone_view * 2)(_view(), _view(pos=(0.0, 12.0, 1.0)))
    nv = 2
    starts = dirs = None
    nrays = 0
    if case == "null_grid":
        st = N.lib.tsp_geometry_create(None, views, nv, None, None, 0, ctypes.byref(out))
        assert st == N.TSP_E_INVALID
        return
    if case == "rb_not_increasing":
        gd, keep = _grid(rb=(1.0, 1.0))
    elif case == "eb_out_of_range":
        gd, keep = _grid(eb=(0.0, 3.5))
    elif case == "ab_span":
        gd, keep = _grid(ab=(0.0, 7.0))
    elif case == "detector_inside":
        views = (N.tsp_cone_view * 1)(_view(pos=(1.5, 0.0, 0.0)))
        nv = 1
    elif case == "fov":
        views = (N.tsp_cone_view * 1)(_view(fov=(180.0, 30.0)))
        nv = 1
    elif case == "shape_mismatch":
        views = (N.tsp_cone_view * 2)(_view(), _view(shape=(4, 5)))
    elif case == "tables_exceed_lds":  # nr + ne + 3 na = 5630 > 5627
        gd, keep = _grid(ab=np.linspace(0.0, 2 * np.pi, 1876 + 1))
    elif case in ("both_sources", "ray_nan", "zero_dir"):
        s = np.array([[10.0, 0, 0]] if case != "ray_nan" else [[np.nan, 0, 0]])
        d = np.array([[-1.0, 0, 0]] if case != "zero_dir" else [[0.0, 0, 0]])
        starts, dirs = s.ctypes.data_as(N._dp), d.ctypes.data_as(N._dp)
        nrays = 1
        if case != "both_sources":
            views, nv = None, 0
    st = N.lib.tsp_geometry_create(ctypes.byref(gd), views, nv, starts, dirs, nrays,
                                   ctypes.byref(out))
    assert st == N.TSP_E_INVALID, N.lib.tsp_last_error()
    assert not out.value
    assert len(N.lib.tsp_last_error()) > 0


@pytest.mark.parametrize("case", ["kind", "size", "reaches_in", "ok_off_axis"])
def test_view_kinds_validation(case):
    """tsp_geometry_create_views: unknown kind, non-positive parallel size,
    a parallel detector reaching into the outer sphere (rejected before any
    device call); a parallel detector beside the sphere passes validation."""
    from paper_2608_16960_amd import native as N
    gd, keep = _grid()  # outer radius 2
    v = N.tsp_view()
    v.kind = N.TSP_VIEW_PARALLEL
    v.shape[:] = (4, 4)
    v.pos[:] = (10.0, 0.0, 0.0)
    v.extent[:] = (3.0, 3.0)
    if case == "kind":
        v.kind = 7
    elif case == "size":
        v.extent[:] = (3.0, 0.0)
    elif case == "reaches_in":
        v.pos[:] = (2.5, 0.0, 0.0)
        v.look[:] = (2.5, 5.0, 0.0)  # looks sideways: the detector plane cuts the ball
    elif case == "ok_off_axis":  # closest detector point (1, 0, 2.5), radius 2.69
        v.pos[:] = (2.5, 0.0, 4.0)
        v.look[:] = (2.5, 5.0, 4.0)
    out = ctypes.c_void_p()
    st = N.lib.tsp_geometry_create_views(ctypes.byref(gd), (N.tsp_view * 1)(v), 1,
                                         ctypes.byref(out))
    if case == "ok_off_axis":
        assert st != N.TSP_E_INVALID, N.lib.tsp_last_error()
        if out.value:
            N.lib.tsp_geometry_destroy(out)
    else:
        assert st == N.TSP_E_INVALID and not out.value


def test_table_limit_is_inclusive():
    """nr + ne + 3 na = 5627 passes validation (without a GPU the call then
    fails in the HIP runtime, not in argument checking)."""
    from paper_2608_16960_amd import native as N
    out = ctypes.c_void_p()
    gd, keep = _grid(ab=np.linspace(0.0, 2 * np.pi, 1875 + 1))
    views = (N.tsp_cone_view * 1)(_view())
    st = N.lib.tsp_geometry_create(ctypes.byref(gd), views, 1, None, None, 0, ctypes.byref(out))
    assert st != N.TSP_E_INVALID, N.lib.tsp_last_error()
    if out.value:
        N.lib.tsp_geometry_destroy(out)


def test_null_geometry_calls():
    from paper_2608_16960_amd import native as N
    assert N.lib.tsp_trace(None, N.TSP_MODE_CSR, None) == N.TSP_E_INVALID
    fr = (ctypes.c_int32 * 1)(0)
    assert N.lib.tsp_set_object_frames(None, fr, 1) == N.TSP_E_INVALID
    assert N.lib.tsp_forward(None, None, 1, None, None) == N.TSP_E_INVALID
    assert N.lib.tsp_backproject(None, None, 1, None, 1, None) == N.TSP_E_INVALID
    info = N.tsp_info()
    assert N.lib.tsp_query(None, ctypes.byref(info)) == N.TSP_E_INVALID
    assert N.lib.tsp_set_timing_events(None, None, None) == N.TSP_E_INVALID
    N.lib.tsp_geometry_destroy(None)
