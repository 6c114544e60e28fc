"""ctypes declarations of the libisx C ABI (include/isx.h).

Loading fails loudly: there is no fallback path.  Build the library with
``python -m paper_2402_13861_amd.build`` first.
"""

from __future__ import annotations

import ctypes as C
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libisx.so"

OK, EINVAL, ESHAPE, ENOMEM, ECAPACITY, EHIP, ENAN, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {
    0: "ISX_OK", -1: "ISX_EINVAL", -2: "ISX_ESHAPE", -3: "ISX_ENOMEM", -4: "ISX_ECAPACITY",
    -5: "ISX_EHIP", -6: "ISX_ENAN", -7: "ISX_EUNSUPPORTED",
}
AA, UP, RAUA, RAFIXED = 0, 1, 2, 3
RELU, SINE, ELU = 0, 1, 2
FP32, BF16, FP64 = 0, 1, 2
(KEEP_LEVELS, HIDDEN_KERNEL, PROFILE, SCRATCH_BYTES, VERBOSE, BF16_VARIANT, UP_FORM, LIN_PRECISION,
 AA_MARGIN, BATCH_WORKERS, CANCEL_CHECK, AUTOTUNE, BF16_READOFF, RECHECK_CASCADE, DENSE_FROM_LEVEL,
 RECHECK_SPLIT) = (1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16)
MAX_LINEAR, MAX_WIDTH, MAX_ISO = 16, 1024, 32
NOALLOC_MAX_CELLS = 1 << 22
(KERNEL_HIDDEN_FP32, KERNEL_HIDDEN_BF16, KERNEL_HIDDEN_SIMT_FP32, KERNEL_HIDDEN_FP64, KERNEL_DENSE,
 KERNEL_OUTPUT, KERNEL_HIDDEN_COV_BF16, KERNEL_LINEARIZE) = range(8)


class SurrogateCalibration(C.Structure):
    _fields_ = [
        ("n_levels", C.c_int32),
        ("n_cells", C.c_int64 * 16),
        ("kept", C.c_int64 * 16),
        ("err_mu", C.c_float * 16),
        ("err_logsig", C.c_float * 16),
        ("z", C.c_float * 16),
        ("z_accept", C.c_float * 16),
        ("z_global", C.c_float),
        ("z_accept_global", C.c_float),
        ("holdout_miss", C.c_double),
        ("holdout_false_accept", C.c_double),
    ]


class SurrogateFitParams(C.Structure):
    _fields_ = [
        ("n_pairs", C.c_int64),
        ("n_holdout", C.c_int64),
        ("steps", C.c_int32),
        ("batch", C.c_int32),
        ("lr", C.c_float),
        ("seed", C.c_uint64),
        ("depth", C.c_int32),
        ("hidden_width", C.c_int32),
        ("hidden_layers", C.c_int32),
        ("use_base", C.c_int32),
        ("mu_bar", C.c_float),
        ("scale", C.c_float),
        ("k", C.c_float),
        ("miss_target", C.c_float),
        ("accept_target", C.c_float),
        ("min_level_kept", C.c_int64),
        ("accept_leaves", C.c_int32),
    ]


class RayParams(C.Structure):
    _fields_ = [
        ("method", C.c_int),
        ("precision", C.c_int),
        ("k", C.c_float),
        ("iso", C.c_float),
        ("step0", C.c_float),
        ("step_min", C.c_float),
        ("step_max", C.c_float),
        ("max_iter", C.c_int32),
    ]


class Params(C.Structure):
    _fields_ = [
        ("method", C.c_int),
        ("precision", C.c_int),
        ("k", C.c_float),
        ("max_depth", C.c_int32),
        ("fp64_band", C.c_float),
        ("max_cells", C.c_int64),
        ("chunk_cells", C.c_int64),
        ("use_surrogate", C.c_int32),
        ("tree", C.c_int32),
        ("fp64_band_rel", C.c_float),
    ]


# (name, restype, argtypes)
_SIGS = [
    ("isx_create", C.c_int, [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("isx_destroy", C.c_int, [C.c_void_p]),
    ("isx_last_error", C.c_char_p, [C.c_void_p]),
    ("isx_load_mlp", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_void_p),
                               C.POINTER(C.c_void_p), C.POINTER(C.c_int32)]),
    ("isx_unload_mlp", C.c_int, [C.c_void_p, C.c_int32]),
    ("isx_set_activation", C.c_int, [C.c_void_p, C.c_int32, C.c_int]),
    ("isx_set_domain", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    ("isx_set_isovalues", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_float)]),
    ("isx_propagate", C.c_int, [C.c_void_p, C.c_int32, C.c_int, C.c_int, C.c_int64, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_void_p]),
    ("isx_classify_compact", C.c_int, [C.c_void_p, C.c_int32, C.c_float, C.c_int64, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p]),
    ("isx_classify_compact_noalloc", C.c_int, [C.c_void_p, C.c_int32, C.c_float, C.c_int64, C.c_void_p,
                                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("isx_eval_points", C.c_int, [C.c_void_p, C.c_int32, C.c_int, C.c_int64, C.c_void_p, C.c_void_p]),
    ("isx_linearize", C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("isx_propagate_segments", C.c_int, [C.c_void_p, C.c_int32, C.c_int, C.c_int, C.c_int64, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_void_p]),
    ("isx_raycast", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(RayParams), C.c_int64, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)]),
    ("isx_distribution_kl", C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                                      C.c_int32, C.c_int32, C.c_uint64, C.c_void_p, C.c_void_p]),
    ("isx_extract", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(Params), C.POINTER(C.c_void_p)]),
    ("isx_extract_dense", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int, C.POINTER(C.c_void_p)]),
    ("isx_extract_batch", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(Params),
                                    C.POINTER(C.c_void_p)]),
    ("isx_mesh_info", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                C.POINTER(C.c_int32)]),
    ("isx_mesh_level", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    ("isx_mesh_level_cancelled", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]),
    ("isx_mesh_level_rechecked_fp64", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]),
    ("isx_mesh_times", C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_float), C.POINTER(C.c_float),
                                 C.POINTER(C.c_float)]),
    ("isx_mesh_copy_tris", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("isx_mesh_copy_leaves", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("isx_mesh_copy_level", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("isx_mesh_free", C.c_int, [C.c_void_p]),
    ("isx_mc_case_table", C.c_int, [C.c_void_p, C.c_void_p]),
    ("isx_set_option", C.c_int, [C.c_void_p, C.c_int, C.c_int64]),
    ("isx_surrogate_load", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_void_p), C.POINTER(C.c_int32)]),
    ("isx_surrogate_get", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
    ("isx_surrogate_set_norm", C.c_int, [C.c_void_p, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float]),
    ("isx_surrogate_set_base", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_float]),
    ("isx_surrogate_train", C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_int64, C.c_int32, C.c_int32, C.c_float, C.c_void_p]),
    ("isx_surrogate_grad", C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_int64, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                     C.POINTER(C.c_float)]),
    ("isx_surrogate_predict", C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("isx_surrogate_attach", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_float),
                                       C.POINTER(C.c_float), C.POINTER(C.c_float), C.POINTER(C.c_float),
                                       C.c_int32]),
    ("isx_surrogate_free", C.c_int, [C.c_void_p, C.c_int32]),
    ("isx_surrogate_partition", C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_float,
                                          C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("isx_surrogate_sample_cells", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                             C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("isx_surrogate_calibrate", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.c_float, C.c_float,
                                          C.c_int64, C.c_int32, C.POINTER(SurrogateCalibration)]),
    ("isx_surrogate_fit", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(SurrogateFitParams),
                                    C.POINTER(C.c_int32), C.POINTER(SurrogateCalibration), C.c_void_p]),
    ("isx_surrogate_save_file", C.c_int, [C.c_void_p, C.c_int32, C.c_char_p]),
    ("isx_surrogate_load_file", C.c_int, [C.c_void_p, C.c_char_p, C.c_int32, C.POINTER(C.c_int32)]),
    ("isx_get_profile", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32]),
]

EXPORTED = [name for name, _, _ in _SIGS]

_lib = None


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2402_13861_amd.build` "
                "(there is no non-HIP fallback)"
            )
        L = C.CDLL(str(LIB_PATH))
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
