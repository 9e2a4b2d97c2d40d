"""ctypes binding of librtg.so (the C ABI of include/rtg.h).

Argument marshalling only: every step runs in the HIP kernels of the
library.  Loading fails loudly when the library has not been built."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# RTG_LIB names another build of the same library (the sanitizer tests load
# an instrumented one)
LIB_PATH = os.environ.get("RTG_LIB") or os.path.join(HERE, "librtg.so")

RTG_OK, RTG_E_INVALID, RTG_E_CAPACITY, RTG_E_HIP, RTG_E_UNSUPPORTED, RTG_E_DEVICE = 0, -1, -2, -3, -4, -5
RTG_E_TOO_LARGE = -6
STATIC_SCRATCH_BYTES = 64 << 20
MAX_FRAMES = 32


class RtgError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (where, status_string(status), status))


class Config(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("cutoff2", ctypes.c_float), ("dilation", ctypes.c_float),
                ("z_near", ctypes.c_float), ("t_eps", ctypes.c_float),
                ("items_per_pop", ctypes.c_int32), ("tile_filter50", ctypes.c_int32),
                ("sort_cap", ctypes.c_int32), ("stage_cap", ctypes.c_int32), ("sh_degree", ctypes.c_int32),
                ("depth_mode", ctypes.c_int32), ("straggler_lanes", ctypes.c_int32),
                ("straggler_rest", ctypes.c_int32), ("static_share", ctypes.c_int32),
                ("fwd_items_per_pop", ctypes.c_int32), ("fwd_static_share", ctypes.c_int32)]


class AddingParams(ctypes.Structure):
    _fields_ = [("delta_T", ctypes.c_float), ("delta_d", ctypes.c_float), ("delta_c", ctypes.c_float),
                ("rate", ctypes.c_float), ("alpha_opaque", ctypes.c_float),
                ("alpha_transparent", ctypes.c_float), ("r_transparent", ctypes.c_float),
                ("thickness", ctypes.c_float), ("delta_eta", ctypes.c_int32), ("delta_e", ctypes.c_int32),
                ("delta_t", ctypes.c_int32), ("sh_degree", ctypes.c_int32)]


class IcpParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("iters", ctypes.c_int32 * 3), ("dist", ctypes.c_double),
                ("sin_angle", ctypes.c_double)]


class Intrinsics(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


_lib = None

# (name, restype, argtypes) of every exported entry point
_P, _I32, _I64, _F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
SIGNATURES = [
    ("rtg_config_default", None, [_P]),
    ("rtg_plan_create", _I32, [_P, _P, _I64, _I32, _I64, _P]),
    ("rtg_plan_destroy", None, [_P]),
    ("rtg_plan_workspace_bytes", ctypes.c_size_t, [_P]),
    ("rtg_plan_layout", _I32, [_P, _P, _I32]),
    ("rtg_project", _I32, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    ("rtg_unstable_mask", _I32, [_P, _P, _P, _P]),
    ("rtg_bin", _I32, [_P, _P, _P, _P]),
    ("rtg_render", _I32, [_P, _P, _P, _P, _P, _P, _P]),
    ("rtg_forward_static", _I32, [_P] * 15),
    ("rtg_backward", _I32, [_P] * 20),
    ("rtg_backward_raster", _I32, [_P] * 8),
    ("rtg_backward_project", _I32, [_P] * 14),
    ("rtg_loss_l1", _I32, [_P, _P, _P, _P, _P, _P, _F, _F, _P, _P, _P, _P]),
    ("rtg_backward_raster_l1", _I32, [_P] * 9),
    ("rtg_backward_project_l1", _I32, [_P] * 8 + [_F, _F] + [_P] * 7),
    ("rtg_adam", _I32, [_P] * 13 + [_F] * 8 + [_P]),
    ("rtg_read_status", _I32, [_P, _P, _P, _P]),
    ("rtg_adding_params_default", None, [_P]),
    ("rtg_adding_workspace_bytes", ctypes.c_size_t, [_P]),
    ("rtg_add_gaussians", _I32, [_P] * 10 + [_I32, _I64, _I64] + [_P] * 12 + [ctypes.c_size_t, _P]),
    ("rtg_confidence_count", _I32, [_I64, _I32, _P, _P, _P, _P]),
    ("rtg_reg_l2", _I32, [_I64, _F] + [_P] * 13),
    ("rtg_fuse", _I32, [_I64, _I32] + [_P] * 11),
    ("rtg_select_workspace_bytes", ctypes.c_size_t, [_I32, _I32, _I32]),
    ("rtg_select_top_error", _I32, [_I32, _I32, _I32, ctypes.c_double, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    ("rtg_render_normals", _I32, [_P, _P, _P, _P]),
    ("rtg_icp_params_default", None, [_P]),
    ("rtg_icp_workspace_bytes", ctypes.c_size_t, [_P, _I32]),
    ("rtg_icp", _I32, [_P] * 10 + [ctypes.c_size_t, _P]),
    ("rtg_state_update", _I32, [_P] * 7 + [_I32, _I64] + [_P] * 7),
    ("rtg_compact_workspace_bytes", ctypes.c_size_t, [_I64]),
    ("rtg_compact_rows", _I32, [_I64, _P, _I32, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    ("rtg_status_string", ctypes.c_char_p, [_I32]),
    ("rtg_version", ctypes.c_char_p, []),
]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librtg.so is not built (%s); run __graft_entry__.build() or "
                               "python paper_2404_19706_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(s):
    try:
        return lib().rtg_status_string(int(s)).decode()
    except Exception:
        return "status %d" % s


def check(status, where):
    if status != RTG_OK:
        raise RtgError(status, where)


def default_config(**kw):
    c = Config()
    lib().rtg_config_default(ctypes.byref(c))
    for k, v in kw.items():
        if not hasattr(c, k):
            raise TypeError("unknown config field %r" % k)
        setattr(c, k, v)
    return c
