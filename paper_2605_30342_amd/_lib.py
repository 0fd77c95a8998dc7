"""ctypes binding of libgavis.so (include/gavis.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
the library.  PyTorch provides device memory (tensor.data_ptr()) and the HIP
stream (torch.cuda.current_stream().cuda_stream).  Loading fails loudly when
the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgavis.so")

GV_OK, GV_ERR_INVALID_ARG, GV_ERR_OUT_OF_MEMORY, GV_ERR_HIP, GV_ERR_CAPACITY, GV_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
GV_F32, GV_F16, GV_BF16 = 0, 1, 2
GV_MAX_SH_DEGREE = 3

# every symbol the header declares
EXPORTS = (
    "gv_create", "gv_destroy", "gv_last_error", "gv_default_vf_params", "gv_default_uq_params",
    "vf_build_workspace_size", "vf_build", "vf_query_workspace_size", "vf_query_views",
    "gv_workspace_check", "gv_workspace_bytes", "select_next_view",
    "gv_profile_enable", "gv_profile_read", "gv_profile_stage_name", "vf_multiview_visibility",
    "gv_set_tuning", "gv_get_tuning", "vf_view_visibility", "vf_query_views_exact",
    "vf_query_views_color", "vf_query_views_noalloc", "vf_density_control_workspace_size", "vf_density_control",
    "vf_virtual_particle_count",
)
GV_PROFILE_STAGES = 9
GV_NOALLOC_SCRATCH_BYTES = 64 << 20
GV_NOALLOC_MAX_VIEWS = 4096


class GvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gavis error {status}: {msg}")
        self.status = status


class gv_camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class gv_gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_virtual", ctypes.c_int64), ("dtype", ctypes.c_int),
                ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("anchors", ctypes.c_void_p), ("anchor_block", ctypes.c_int32)]


class gv_vf_params(ctypes.Structure):
    _fields_ = [("sh_degree", ctypes.c_int32), ("kappa", ctypes.c_float), ("eps_T", ctypes.c_float),
                ("znear", ctypes.c_float), ("lowpass", ctypes.c_float), ("cut", ctypes.c_float),
                ("views_per_pass", ctypes.c_int32), ("accumulate", ctypes.c_int32)]


class gv_density_params(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_float * 3), ("hi", ctypes.c_float * 3), ("rho", ctypes.c_float),
                ("eta", ctypes.c_float), ("eps_v", ctypes.c_float)]


class gv_uq_params(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_float), ("o0", ctypes.c_float), ("half_logdet_Q0", ctypes.c_float),
                ("half_logdet_Qc", ctypes.c_float), ("eps_T", ctypes.c_float), ("znear", ctypes.c_float),
                ("lowpass", ctypes.c_float), ("cut", ctypes.c_float), ("write_maps", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("count_pairs", ctypes.c_int32), ("write_depth", ctypes.c_int32)]


class gv_tuning(ctypes.Structure):
    _fields_ = [("vis_batch", ctypes.c_int32), ("uq_batch", ctypes.c_int32), ("vis_order", ctypes.c_int32),
                ("uq_order", ctypes.c_int32)]


class gv_workspace(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_size_t), ("max_records", ctypes.c_int64), ("max_instances", ctypes.c_int64),
                ("n", ctypes.c_int64), ("n_views", ctypes.c_int32), ("total_tiles", ctypes.c_int32),
                ("total_pixels", ctypes.c_int64), ("kind", ctypes.c_int32), ("sh_degree", ctypes.c_int32),
                ("emit_mode", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Loads libgavis.so; raises if it is missing (build it with
    paper_2605_30342_amd.build.build_library())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run python -m paper_2605_30342_amd.build")
    L = ctypes.CDLL(path)
    P, vp = ctypes.POINTER, ctypes.c_void_p
    i32, i64, st = ctypes.c_int32, ctypes.c_int64, ctypes.c_int
    L.gv_create.argtypes = [ctypes.c_int, P(vp)]
    L.gv_create.restype = st
    L.gv_destroy.argtypes = [vp]
    L.gv_destroy.restype = None
    L.gv_last_error.argtypes = []
    L.gv_last_error.restype = ctypes.c_char_p
    L.gv_default_vf_params.argtypes = [P(gv_vf_params)]
    L.gv_default_vf_params.restype = None
    L.gv_default_uq_params.argtypes = [P(gv_uq_params)]
    L.gv_default_uq_params.restype = None
    L.vf_build_workspace_size.argtypes = [vp, P(gv_gaussians), P(gv_camera), i32, P(gv_vf_params),
                                          P(gv_workspace), vp]
    L.vf_build_workspace_size.restype = st
    L.vf_build.argtypes = [vp, P(gv_gaussians), P(gv_camera), i32, P(gv_vf_params), vp, ctypes.c_int,
                           P(gv_workspace), vp, vp]
    L.vf_build.restype = st
    L.vf_multiview_visibility.argtypes = [vp, P(gv_gaussians), P(gv_camera), i32, P(gv_vf_params), vp,
                                          P(gv_workspace), vp, vp]
    L.vf_multiview_visibility.restype = st
    L.vf_view_visibility.argtypes = [vp, P(gv_gaussians), P(gv_camera), i32, P(gv_vf_params), vp, vp,
                                     P(gv_workspace), vp, vp]
    L.vf_view_visibility.restype = st
    L.vf_density_control_workspace_size.argtypes = [vp, P(gv_gaussians), i64, vp, i64, P(gv_density_params),
                                                    P(gv_camera), i32, P(gv_vf_params), P(gv_workspace), P(i64), vp]
    L.vf_density_control_workspace_size.restype = st
    L.vf_density_control.argtypes = [vp, P(gv_gaussians), i64, vp, i64, P(gv_density_params), P(gv_camera), i32,
                                     P(gv_vf_params), vp, vp, P(i64), P(gv_workspace), vp, vp]
    L.vf_density_control.restype = st
    L.vf_virtual_particle_count.argtypes = [P(gv_density_params), P(i64), P(ctypes.c_float)]
    L.vf_virtual_particle_count.restype = st
    L.vf_query_views_exact.argtypes = [vp, P(gv_gaussians), vp, vp, i32, ctypes.c_float, P(gv_camera), i32,
                                       P(gv_uq_params), vp, vp, P(gv_workspace), vp, vp]
    L.vf_query_views_exact.restype = st
    L.vf_query_views_color.argtypes = [vp, P(gv_gaussians), vp, ctypes.c_int, i32, i64, vp, i32, P(gv_camera), i32,
                                       P(gv_uq_params), vp, vp, P(gv_workspace), vp, vp]
    L.vf_query_views_color.restype = st
    L.vf_query_workspace_size.argtypes = [vp, P(gv_gaussians), P(gv_camera), i32, P(gv_uq_params), i32,
                                          P(gv_workspace), vp]
    L.vf_query_workspace_size.restype = st
    L.vf_query_views.argtypes = [vp, P(gv_gaussians), vp, ctypes.c_int, i32, i64, P(gv_camera), i32,
                                 P(gv_uq_params), vp, vp, P(gv_workspace), vp, vp]
    L.vf_query_views.restype = st
    L.vf_query_views_noalloc.argtypes = [vp, P(gv_gaussians), vp, ctypes.c_int, i32, i64, P(gv_camera), i32,
                                         P(gv_uq_params), vp, vp, vp]
    L.vf_query_views_noalloc.restype = st
    L.gv_workspace_check.argtypes = [vp, P(gv_workspace), vp, P(i64), vp]
    L.gv_workspace_check.restype = st
    L.gv_workspace_bytes.argtypes = [P(gv_workspace)]
    L.gv_workspace_bytes.restype = ctypes.c_size_t
    L.select_next_view.argtypes = [vp, vp, i32, P(i32), vp]
    L.select_next_view.restype = st
    L.gv_set_tuning.argtypes = [vp, P(gv_tuning)]
    L.gv_set_tuning.restype = st
    L.gv_get_tuning.argtypes = [vp, P(gv_tuning)]
    L.gv_get_tuning.restype = st
    L.gv_profile_enable.argtypes = [vp, i32]
    L.gv_profile_enable.restype = st
    L.gv_profile_read.argtypes = [vp, P(ctypes.c_double), P(i64), vp]
    L.gv_profile_read.restype = st
    L.gv_profile_stage_name.argtypes = [i32]
    L.gv_profile_stage_name.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status: int) -> None:
    if status != GV_OK:
        msg = load().gv_last_error()
        raise GvError(status, msg.decode() if msg else "")


def default_vf_params(**kw) -> gv_vf_params:
    p = gv_vf_params()
    load().gv_default_vf_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def default_uq_params(**kw) -> gv_uq_params:
    p = gv_uq_params()
    load().gv_default_uq_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


_CAMERA_DTYPE = None


def cameras_to_c(cams) -> ctypes.Array:
    """Host gv_camera[] from a scenes.Cameras (filled column-wise with numpy)."""
    global _CAMERA_DTYPE
    if _CAMERA_DTYPE is None:
        import numpy as np
        _CAMERA_DTYPE = np.dtype([("R", np.float32, 9), ("t", np.float32, 3), ("K", np.float32, 4),
                                  ("wh", np.int32, 2)])
        assert _CAMERA_DTYPE.itemsize == ctypes.sizeof(gv_camera)
    import numpy as np
    arr = (gv_camera * cams.n)()
    view = np.frombuffer(arr, dtype=_CAMERA_DTYPE, count=cams.n)
    view["R"] = np.asarray(cams.R, dtype=np.float32).reshape(cams.n, 9)
    view["t"] = np.asarray(cams.t, dtype=np.float32).reshape(cams.n, 3)
    view["K"] = np.asarray(cams.K, dtype=np.float32).reshape(cams.n, 4)
    view["wh"] = np.asarray(cams.wh, dtype=np.int32).reshape(cams.n, 2)
    return arr
