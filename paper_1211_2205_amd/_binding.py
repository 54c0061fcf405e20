"""ctypes binding of libstarmap.so (include/starmap.h).

Argument marshalling only: every step of the solver runs in the native
library and its HIP kernels.  Loading fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstarmap.so")

OK = 0
EINVAL, ENOMEM, EHIP, EUNSTABLE, ESTATE = -1, -2, -3, -4, -5
BC_PERIODIC, BC_EXTRAPOLATION = 0, 1
FP64, FP32, BF16 = 0, 1, 2
CLOSURE_PN, CLOSURE_LEARNED = 0, 1
CLOSURE_PARAMS = 33798
FIELD_ABSORPTION, FIELD_SCATTERING, FIELD_SOURCE, FIELD_INITIAL = 0, 1, 2, 3
FIELD_SCATTERING_ORDER = 4
MAX_FIELD_TERMS = 32
FUSED_MAX_ORDER = 7

_ERRNAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHIP: "EHIP", EUNSTABLE: "EUNSTABLE", ESTATE: "ESTATE"}


class StarmapError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"starmap error {_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("ax", ctypes.c_double * 4), ("n", ctypes.c_int32 * 2), ("bc", ctypes.c_int32 * 2),
                ("N", ctypes.c_int32), ("cfl", ctypes.c_double), ("t_final", ctypes.c_double),
                ("precision", ctypes.c_int32), ("closure", ctypes.c_int32)]


FIELD_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.c_int64,
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double))

TIME_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_void_p, ctypes.c_double)

_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)
_szp = ctypes.POINTER(ctypes.c_size_t)
_fp = ctypes.POINTER(ctypes.c_float)

# (name, argtypes, restype)
SIGNATURES = [
    ("starmap_num_moments", [ctypes.c_int32], ctypes.c_int),
    ("starmap_moment_info", [ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, _i32p, _i32p, _i32p], ctypes.c_int),
    ("starmap_closure_pn", [ctypes.c_int32, ctypes.c_int32, _i32p, _dp], ctypes.c_int),
    ("starmap_spectral_radius", [ctypes.c_int32, _dp], ctypes.c_int),
    ("starmap_direction_moments", [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp],
     ctypes.c_int),
    ("starmap_plan_check", [ctypes.c_int32] * 4, ctypes.c_int),
    ("starmap_create", [ctypes.POINTER(Problem), ctypes.POINTER(_vp)], ctypes.c_int),
    ("starmap_destroy", [_vp], None),
    ("starmap_set_absorption", [_vp, FIELD_FN, _vp, ctypes.c_int32], ctypes.c_int),
    ("starmap_set_scattering", [_vp, FIELD_FN, _vp, ctypes.c_int32], ctypes.c_int),
    ("starmap_set_scattering_order", [_vp, ctypes.c_int32, FIELD_FN, _vp, ctypes.c_int32], ctypes.c_int),
    ("starmap_set_source", [_vp, ctypes.c_int32, FIELD_FN, _vp, ctypes.c_int32], ctypes.c_int),
    ("starmap_set_initial", [_vp, ctypes.c_int32, FIELD_FN, _vp], ctypes.c_int),
    ("starmap_set_filter_damping", [_vp, _dp], ctypes.c_int),
    ("starmap_set_diffusion", [_vp, FIELD_FN, _vp], ctypes.c_int),
    ("starmap_set_fused", [_vp, ctypes.c_int32], ctypes.c_int),
    ("starmap_add_field_term", [_vp, ctypes.c_int32, ctypes.c_int32, FIELD_FN, _vp, TIME_FN, _vp], ctypes.c_int),
    ("starmap_set_field_array", [_vp, ctypes.c_int32, ctypes.c_int32, _dp], ctypes.c_int),
    ("starmap_moment_shape", [_vp, ctypes.c_int32, _i32p, _i32p, _dp, _dp], ctypes.c_int),
    ("starmap_time", [_vp, _dp, _dp, _i64p, _i64p], ctypes.c_int),
    ("starmap_workspace_bytes", [_vp, _szp], ctypes.c_int),
    ("starmap_bind_device", [_vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    ("starmap_advance", [_vp, ctypes.c_int64], ctypes.c_int),
    ("starmap_run", [_vp], ctypes.c_int),
    ("starmap_sweep", [_vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32], ctypes.c_int),
    ("starmap_synchronize", [_vp], ctypes.c_int),
    ("starmap_get_moment", [_vp, ctypes.c_int32, _dp], ctypes.c_int),
    ("starmap_state_bytes", [_vp, _szp], ctypes.c_int),
    ("starmap_get_state", [_vp, _vp, ctypes.c_size_t, _dp, _i64p], ctypes.c_int),
    ("starmap_set_state", [_vp, _vp, ctypes.c_size_t, ctypes.c_double, ctypes.c_int64], ctypes.c_int),
    ("starmap_diagnostics", [_vp, _dp, _dp, _dp, _i32p], ctypes.c_int),
    ("starmap_variant_count", [], ctypes.c_int),
    ("starmap_set_variant", [_vp, ctypes.c_int32], ctypes.c_int),
    ("starmap_get_variant", [_vp, _i32p, _i32p, _i32p], ctypes.c_int),
    ("starmap_autotune", [_vp, ctypes.c_int32], ctypes.c_int),
    ("starmap_set_range_width", [_vp, ctypes.c_int32], ctypes.c_int),
    ("starmap_set_graphs", [_vp, ctypes.c_int32], ctypes.c_int),
    ("starmap_closure_set_fused", [_vp, ctypes.c_int32], ctypes.c_int),
    ("starmap_diagnostics_noalloc", [_vp, _dp, _dp, _dp, _i32p], ctypes.c_int),
    ("starmap_get_range_width", [_vp, _i32p], ctypes.c_int),
    ("starmap_sweep_bytes", [_vp, ctypes.c_int32, _dp], ctypes.c_int),
    ("starmap_profile_begin", [_vp], ctypes.c_int),
    ("starmap_profile_end", [_vp, _dp, _i64p, _dp], ctypes.c_int),
    ("starmap_closure_load", [_vp, _fp, ctypes.c_size_t], ctypes.c_int),
    ("starmap_closure_samples", [_vp, _i32p, ctypes.c_int32, _vp, _vp], ctypes.c_int),
    ("starmap_closure_features", [_vp, _i32p, ctypes.c_int32, _vp, _vp], ctypes.c_int),
    ("starmap_mlp_create", [ctypes.c_int32, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    ("starmap_mlp_destroy", [_vp], None),
    ("starmap_mlp_set_params", [_vp, _fp, ctypes.c_size_t], ctypes.c_int),
    ("starmap_mlp_get_params", [_vp, _fp, ctypes.c_size_t], ctypes.c_int),
    ("starmap_mlp_forward", [_vp, _vp, ctypes.c_int32, _vp], ctypes.c_int),
    ("starmap_mlp_gradients", [_vp, _vp, _vp, ctypes.c_int32, _fp, _dp], ctypes.c_int),
    ("starmap_mlp_train_step", [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_double, _dp], ctypes.c_int),
    ("starmap_mlp_adam_step", [_vp, _fp, ctypes.c_double], ctypes.c_int),
    ("starmap_reset", [_vp], ctypes.c_int),
    ("starmap_batch_create", [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.POINTER(_vp)], ctypes.c_int),
    ("starmap_batch_destroy", [_vp], None),
    ("starmap_batch_run", [_vp, ctypes.c_int32], ctypes.c_int),
    ("starmap_batch_last_run", [_vp, _dp, _i64p, _dp, _i64p], ctypes.c_int),
    ("starmap_batch_set_variant", [_vp, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    ("starmap_batch_get_variant", [_vp, _i32p, _i32p], ctypes.c_int),
    ("starmap_batch_autotune", [_vp, ctypes.c_int32], ctypes.c_int),
    ("starmap_batch_group_count", [_vp], ctypes.c_int),
    ("starmap_batch_set_merged", [_vp, ctypes.c_int32], ctypes.c_int),
    ("starmap_batch_get_merged", [_vp], ctypes.c_int),
    ("starmap_batch_set_group_variant", [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    ("starmap_batch_get_group", [_vp, ctypes.c_int32, _i32p, _i32p, _i32p, _i32p], ctypes.c_int),
    ("starmap_last_error", [], ctypes.c_char_p),
]

_lib = None


def lib():
    """Load libstarmap.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1211_2205_amd.build.build() "
                              "(hipcc, gfx950); there is no fallback implementation")
        # PyTorch ships its own HIP runtime under the same soname as the system
        # one the library links against.  Loading torch first makes the library
        # bind to torch's copy, so the process has one runtime (shared device
        # context and streams); the other order leaves torch on a mismatched
        # runtime that finds no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, args, res in SIGNATURES:
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(rc):
    if rc is not None and rc < 0:
        msg = lib().starmap_last_error()
        raise StarmapError(rc, msg.decode() if msg else "")
    return rc
