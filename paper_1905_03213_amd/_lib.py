"""ctypes declarations of libwproj.so (include/wproj.h).

Loading fails loudly when the library has not been built: there is no other
implementation to fall back to.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwproj.so")

F64, F32, F32_F16TABLE = 0, 1, 2
ALGO_TILED, ALGO_PLAIN = 0, 1
W_LINEAR, W_FOLD, W_FOLD_SQRT, W_STACK = 0, 1, 2, 3
GRID_TO_IMAGE, IMAGE_TO_GRID, GRID_TO_IMAGE_RAW = 0, 1, 2
EXPORT_TABLES, EXPORT_TABLE_OFFSETS, EXPORT_KAPPA, EXPORT_TAPER, EXPORT_SUPPORTS = range(5)

STATUS = {0: "WPROJ_OK", -1: "WPROJ_EINVAL", -2: "WPROJ_ENOMEM", -3: "WPROJ_EHIP",
          -4: "WPROJ_EUNSUPPORTED", -5: "WPROJ_EWORKSPACE", -6: "WPROJ_EFFT", -7: "WPROJ_EEMPTY"}

EXPORTED = ("wproj_make_kernels", "wproj_free_kernels", "wproj_export", "wproj_workspace_size",
            "wproj_grid", "wproj_degrid", "wproj_image", "wproj_autotune", "wproj_tuning",
            "wproj_profile", "wproj_profile_read", "wproj_last_error", "wproj_version",
            "wproj_footprints", "wproj_regroup_workspace_size", "wproj_regroup_rows",
            "wproj_gather_rows", "wproj_plan_create", "wproj_plan_free", "wproj_grid_planned",
            "wproj_degrid_planned", "wproj_plan_rows", "wproj_chi2", "wproj_chi2_workspace_size",
            "wproj_grid_noalloc", "wproj_noalloc_scratch_bytes",
            "wproj_check_weights", "wproj_measure_lds", "wproj_measure_vmem", "wproj_regroup_channels")
PHASES = ("bin", "grid", "plain", "fft", "correct", "degrid", "reduce")


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("n_wplanes", ctypes.c_int32),
        ("cell_rad", ctypes.c_double),
        ("w_max", ctypes.c_double),
        ("support", ctypes.c_int32),
        ("oversample", ctypes.c_int32),
        ("support_per_plane", ctypes.POINTER(ctypes.c_int32)),
        ("kernel_image_size", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("n_images", ctypes.c_int32),
        ("algorithm", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("chunk", ctypes.c_int32),
        ("w_mode", ctypes.c_int32),
        ("accumulate_runs", ctypes.c_int32),
        ("n_wlayers", ctypes.c_int32),
        ("bin_aggregate", ctypes.c_int32),
        ("stable_bins", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 1),
    ]


class WprojError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} -> {STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1905_03213_amd.build` "
            "(hipcc, gfx950). There is no fallback implementation.")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.wproj_make_kernels.argtypes = [ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    L.wproj_free_kernels.argtypes = [vp]
    L.wproj_export.argtypes = [vp, i32, vp, i64, ctypes.POINTER(i64), vp]
    L.wproj_workspace_size.argtypes = [vp, i64]
    L.wproj_workspace_size.restype = i64
    L.wproj_grid.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, i64, vp]
    L.wproj_degrid.argtypes = [vp, i64, vp, vp, vp, vp, vp, i64, vp]
    L.wproj_image.argtypes = [vp, i32, vp, vp, vp, vp, i64, vp]
    L.wproj_autotune.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, i64, vp]
    L.wproj_tuning.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32)]
    L.wproj_profile.argtypes = [vp, i32]
    L.wproj_profile_read.argtypes = [vp, vp, vp]
    L.wproj_last_error.restype = ctypes.c_char_p
    L.wproj_last_error.argtypes = []
    L.wproj_version.argtypes = []
    L.wproj_footprints.argtypes = [vp, i64, vp, vp, vp, vp]
    L.wproj_plan_create.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, i64, vp, ctypes.POINTER(vp)]
    L.wproj_plan_free.argtypes = [vp]
    L.wproj_grid_planned.argtypes = [vp, vp, vp, vp]
    L.wproj_degrid_planned.argtypes = [vp, vp, vp, vp]
    L.wproj_plan_rows.argtypes = [vp, vp, vp]
    L.wproj_chi2.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp, i64, vp]
    L.wproj_chi2_workspace_size.argtypes = []
    L.wproj_chi2_workspace_size.restype = i64
    L.wproj_regroup_workspace_size.argtypes = [i64, ctypes.c_int32]
    L.wproj_regroup_workspace_size.restype = i64
    L.wproj_regroup_rows.argtypes = [i64, vp, vp, ctypes.c_int32, vp, vp, vp, vp, i64, vp]
    L.wproj_gather_rows.argtypes = [i64, i64, vp, i64, vp, vp, vp, vp]
    L.wproj_grid_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    L.wproj_noalloc_scratch_bytes.argtypes = []
    L.wproj_noalloc_scratch_bytes.restype = i64
    L.wproj_check_weights.argtypes = [vp, vp, vp]
    L.wproj_regroup_channels.argtypes = [i64, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp]
    L.wproj_measure_lds.argtypes = [i32, ctypes.c_int32, vp, vp, vp]
    L.wproj_measure_vmem.argtypes = [i32, ctypes.c_int32, vp, vp, vp]
    for name in ("wproj_make_kernels", "wproj_free_kernels", "wproj_export", "wproj_grid",
                 "wproj_degrid", "wproj_image", "wproj_autotune", "wproj_tuning", "wproj_profile",
                 "wproj_profile_read", "wproj_version", "wproj_footprints", "wproj_regroup_rows",
                 "wproj_gather_rows", "wproj_plan_create", "wproj_plan_free", "wproj_grid_planned",
                 "wproj_degrid_planned", "wproj_plan_rows", "wproj_chi2", "wproj_grid_noalloc",
                 "wproj_check_weights",
                 "wproj_measure_lds",
                 "wproj_measure_vmem", "wproj_regroup_channels"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def check(fn: str, rc: int):
    if rc != 0:
        raise WprojError(fn, rc, lib().wproj_last_error().decode())
    return rc
