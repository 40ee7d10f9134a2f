"""ctypes binding of libtsp.so (include/tsp.h); argument marshalling only.

Every function here forwards to the C ABI of the same name.  There is no
fallback: if the native library is missing the import of this module raises,
and every computation runs in the HIP kernels behind the ABI.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtsp.so")

TSP_OK, TSP_E_INVALID, TSP_E_NOMEM, TSP_E_HIP, TSP_E_STATE, TSP_E_UNSUPPORTED = range(6)
TSP_MODE_CSR = 1
TSP_MODE_ONTHEFLY = 2
TSP_TRACE_NO_CSC = 0x10
TSP_ADJ_DETERMINISTIC = 1
TSP_ADJ_ATOMIC = 2
TSP_ADJ_FIXEDPOINT = 3

STATUS_NAMES = {0: "TSP_OK", 1: "TSP_E_INVALID", 2: "TSP_E_NOMEM", 3: "TSP_E_HIP",
                4: "TSP_E_STATE", 5: "TSP_E_UNSUPPORTED"}


class TspError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class tsp_grid_desc(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("ne", ctypes.c_int32), ("na", ctypes.c_int32),
                ("r_b", ctypes.POINTER(ctypes.c_double)),
                ("e_b", ctypes.POINTER(ctypes.c_double)),
                ("a_b", ctypes.POINTER(ctypes.c_double))]


class tsp_cone_view(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_double * 3), ("look", ctypes.c_double * 3),
                ("up", ctypes.c_double * 3), ("fov_deg", ctypes.c_double * 2),
                ("shape", ctypes.c_int32 * 2)]


TSP_VIEW_CONE = 0
TSP_VIEW_PARALLEL = 1


class tsp_view(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("shape", ctypes.c_int32 * 2),
                ("reserved", ctypes.c_int32), ("pos", ctypes.c_double * 3),
                ("look", ctypes.c_double * 3), ("up", ctypes.c_double * 3),
                ("extent", ctypes.c_double * 2)]


class tsp_info(ctypes.Structure):
    _fields_ = [("n_rays", ctypes.c_int64), ("n_voxels", ctypes.c_int64),
                ("n_segments", ctypes.c_int64), ("n_stored", ctypes.c_int64),
                ("max_per_ray", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("mode", ctypes.c_int32), ("has_csc", ctypes.c_int32),
                ("n_obj_frames", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_st = ctypes.c_int

# name -> (restype, argtypes)
SIGNATURES = {
    "tsp_geometry_create": (_st, [ctypes.POINTER(tsp_grid_desc), ctypes.POINTER(tsp_cone_view),
                                  ctypes.c_int32, _dp, _dp, ctypes.c_int64,
                                  ctypes.POINTER(_vp)]),
    "tsp_geometry_create_views": (_st, [ctypes.POINTER(tsp_grid_desc), ctypes.POINTER(tsp_view),
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "tsp_set_object_frames": (_st, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]),
    "tsp_geometry_create_sunward": (_st, [ctypes.POINTER(tsp_grid_desc), _dp,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "tsp_atten_forward": (_st, [_vp, _vp, _vp, _vp, ctypes.c_int32, _vp, _vp, _vp]),
    "tsp_atten_backward": (_st, [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32, _vp,
                                 ctypes.c_int32, _vp]),
    "tsp_trace": (_st, [_vp, ctypes.c_int32, _vp]),
    "tsp_forward": (_st, [_vp, _vp, ctypes.c_int32, _vp, _vp]),
    "tsp_backproject": (_st, [_vp, _vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp]),
    "tsp_backproject_noalloc": (_st, [_vp, _vp, ctypes.c_int32, _vp, _vp]),
    "tsp_segments": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "tsp_rays": (_st, [_vp, _vp, _vp, _vp]),
    "tsp_set_timing_events": (_st, [_vp, _vp, _vp]),
    "tsp_query": (_st, [_vp, ctypes.POINTER(tsp_info)]),
    "tsp_geometry_destroy": (None, [_vp]),
    "tsp_last_error": (ctypes.c_char_p, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2608_16960_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def check(status):
    if status != TSP_OK:
        raise TspError(status, lib.tsp_last_error().decode(errors="replace"))


def ptr(t):
    """Device address of a tensor (or None) as a c_void_p."""
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def stream_handle(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)
