"""ctypes view of the C ABI in include/wect.h (libwect.so, built in-tree).

Loading fails loudly when the library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_void_p

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libwect.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "wect.h")

WECT_OK, WECT_ERR_ARG, WECT_ERR_INDEX, WECT_ERR_THRESHOLDS, WECT_ERR_NONFINITE, \
    WECT_ERR_WORKSPACE, WECT_ERR_UNSUPPORTED, WECT_ERR_DEVICE = range(8)
WECT_W_ONES, WECT_W_EXPLICIT, WECT_W_VERTEX_MAX = 0, 1, 2
WECT_I32, WECT_F32 = 0, 1
WECT_SIMPLICIAL, WECT_CUBICAL = 0, 1


class WectComplex(ctypes.Structure):
    _fields_ = [
        ("kind", c_int32), ("n", c_int32), ("B", c_int32), ("top_dim", c_int32),
        ("wmode", c_int32), ("dtype", c_int32),
        ("coords", c_void_p), ("vert_off", c_void_p), ("count", c_int64 * 4),
        ("simplices", c_void_p * 4), ("simp_off", c_void_p * 4), ("weights", c_void_p * 4),
        ("shape", c_void_p), ("grid_off", c_void_p), ("intensity", c_void_p), ("axis", c_void_p),
        ("axis_off", c_void_p), ("total_voxels", c_int64), ("include_above", c_int32), ("reserved", c_int32),
    ]


class WectGrid(ctypes.Structure):
    _fields_ = [("dirs", c_void_p), ("d", c_int32), ("T", c_int32), ("thr", c_void_p)]


class WectLaunch(ctypes.Structure):
    _fields_ = [("block", c_int32), ("blocks_per_cu", c_int32), ("min_items_per_block", c_int32),
                ("decomposition", c_int32), ("threshold_tile", c_int32), ("directions_per_lane", c_int32),
                ("cubical_records", c_int32), ("cell_packing", c_int32),
                ("stage_entries", c_int32)]


class WectError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        detail = ""
        if status == WECT_ERR_DEVICE:
            detail = " [" + lib().wect_last_error().decode() + "]"
        super().__init__(f"{what}: {status_string(status)} (status {status}){detail}")


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libwect.so not found at {LIB_PATH}; build it with "
                           "`python -m paper_2511_03909_amd.build` (no fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    P = POINTER
    L.wect_workspace_bytes.argtypes = [P(WectComplex), P(WectGrid), c_int]
    L.wect_workspace_bytes.restype = c_size_t
    L.wect_forward.argtypes = [P(WectComplex), P(WectGrid), c_void_p, c_void_p, c_size_t, c_void_p]
    L.wect_forward.restype = c_int
    L.wect_forward_noalloc.argtypes = [P(WectComplex), P(WectGrid), c_void_p, c_void_p]
    L.wect_forward_noalloc.restype = c_int
    L.wect_backward.argtypes = [P(WectComplex), P(WectGrid), c_void_p, P(c_void_p), c_void_p, c_void_p,
                                c_size_t, c_void_p]
    L.wect_backward.restype = c_int
    L.wect_batched.argtypes = [P(WectComplex), P(WectGrid), c_void_p, c_void_p, P(c_void_p), c_void_p,
                               c_void_p, c_size_t, c_void_p]
    L.wect_batched.restype = c_int
    L.wect_validate.argtypes = [P(WectComplex), P(WectGrid), c_void_p]
    L.wect_validate.restype = c_int
    L.wect_status_string.argtypes = [c_int]
    L.wect_status_string.restype = c_char_p
    L.wect_set_launch.argtypes = [P(WectLaunch)]
    L.wect_set_launch.restype = c_int
    L.wect_get_launch.argtypes = [P(WectLaunch)]
    L.wect_get_launch.restype = c_int
    L.wect_profile_enable.argtypes = [c_int]
    L.wect_profile_enable.restype = c_int
    L.wect_profile_read.argtypes = [P(c_double), P(c_int64), P(c_double), P(c_int64), c_int]
    L.wect_profile_read.restype = c_int
    L.wect_calib_copy.argtypes = [c_void_p, c_void_p, c_size_t, c_void_p]
    L.wect_calib_copy.restype = c_int
    L.wect_calib_lds_atomics.argtypes = [c_int32, c_int32, c_int32, c_void_p, c_void_p]
    L.wect_calib_lds_atomics.restype = c_int
    L.wect_version.argtypes = []
    L.wect_version.restype = c_char_p
    L.wect_last_error.argtypes = []
    L.wect_last_error.restype = c_char_p
    L.wect_wecf_workspace_bytes.argtypes = [P(WectComplex), c_int32, c_int32]
    L.wect_wecf_workspace_bytes.restype = c_size_t
    L.wect_wecf_forward.argtypes = [P(WectComplex), c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_void_p,
                                    c_size_t, c_void_p]
    L.wect_wecf_forward.restype = c_int
    L.wect_wecf_backward.argtypes = [P(WectComplex), c_void_p, c_int32, c_void_p, c_int32, c_void_p, P(c_void_p),
                                     c_void_p, c_void_p, c_size_t, c_void_p]
    L.wect_wecf_backward.restype = c_int
    L.wect_freudenthal_counts.argtypes = [c_int32, c_void_p, P(c_int64)]
    L.wect_freudenthal_counts.restype = c_int
    L.wect_freudenthal_build.argtypes = [P(WectComplex)] + [c_void_p] * 8
    L.wect_freudenthal_build.restype = c_int
    L.wect_image_ecf_workspace_bytes.argtypes = [P(WectComplex)]
    L.wect_image_ecf_workspace_bytes.restype = c_size_t
    L.wect_image_ecf.argtypes = [P(WectComplex), c_void_p, c_int32, c_void_p, c_void_p, c_size_t, c_void_p]
    L.wect_image_ecf.restype = c_int
    L.wect_smooth_workspace_bytes.argtypes = [P(WectComplex), P(WectGrid), c_float]
    L.wect_smooth_workspace_bytes.restype = c_size_t
    L.wect_smooth_forward.argtypes = [P(WectComplex), P(WectGrid), c_float, c_void_p, c_void_p, c_size_t, c_void_p]
    L.wect_smooth_forward.restype = c_int
    L.wect_smooth_backward.argtypes = [P(WectComplex), P(WectGrid), c_float, c_void_p, c_void_p, c_void_p,
                                       P(c_void_p), c_void_p, c_void_p]
    L.wect_smooth_backward.restype = c_int
    L.wect_lower_star_bytes.argtypes = [P(WectComplex)]
    L.wect_lower_star_bytes.restype = c_size_t
    L.wect_lower_star_build.argtypes = [P(WectComplex), c_void_p, c_size_t, c_void_p]
    L.wect_lower_star_build.restype = c_int
    L.wect_smooth_ls_workspace_bytes.argtypes = [P(WectComplex), P(WectGrid), c_float]
    L.wect_smooth_ls_workspace_bytes.restype = c_size_t
    L.wect_smooth_ls_forward.argtypes = [P(WectComplex), P(WectGrid), c_float, c_void_p, c_size_t, c_void_p,
                                         c_void_p, c_size_t, c_void_p]
    L.wect_smooth_ls_forward.restype = c_int
    L.wect_smooth_ls_backward.argtypes = [P(WectComplex), P(WectGrid), c_float, c_void_p, c_size_t, c_void_p,
                                          c_void_p, c_void_p, P(c_void_p), c_void_p, c_void_p]
    L.wect_smooth_ls_backward.restype = c_int
    _lib = L
    return L


def status_string(status: int) -> str:
    return lib().wect_status_string(int(status)).decode()


def check(status: int, what: str) -> None:
    if status != WECT_OK:
        raise WectError(status, what)


def declared_functions() -> list:
    """Names of the functions include/wect.h declares."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wect_[a-z_]+)\s*\(", text)))
