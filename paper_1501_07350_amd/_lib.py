"""ctypes binding of libofft.so (the C ABI declared in include/offt.h).

Argument marshalling only: every step of the transform runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libofft.so")

C2C_F64 = 0
C2C_F32 = 1

SUCCESS = 0
ERR_INVALID_ARG = -1
ERR_UNSUPPORTED_SIZE = -2
ERR_OUT_OF_MEMORY = -3
ERR_NO_DEVICE = -4
ERR_HIP = -5
ERR_BAD_PLAN = -6
ERR_IO = -7

TUNE_NONE = 0
TUNE_EXHAUSTIVE = 1
TUNE_LEARNED = 2
TUNE_FORCED = 3

FORWARD = -1
BACKWARD = +1

# launch forms of offt_exec_many
MANY_SEPARATE_TUNED = -2
MANY_SEPARATE_HEURISTIC = -1
MANY_PERSISTENT = 0
MANY_PERSISTENT_GRAPH = 1
MANY_LEVELS_GRAPH = 2
MANY_LEVELS = 3
MANY_SYNC = 4
MANY_SYNC_GRAPH = 5
MANY_LEVELS_GROUPED_GRAPH = 6
MAX_AXIS = 1024
MAX_DIMS = 5

# communication methods of the distributed flow (offt_plan_dist)
COMM_AUTO = -1
COMM_ISEND_WAITALL = 0
COMM_ALLTOALLV = 1
COMM_ISEND_WAITALL_BLOCK = 2
COMM_ISEND_WAITSOME = 3
COMM_ISEND_WAITSOME_BLOCK = 4
COMM_SENDRECV = 5
COMM_METHODS = ["Isend_Waitall", "Alltoallv", "Isend_Waitall_Block", "Isend_Waitsome", "Isend_Waitsome_Block",
                "Sendrecv"]
ORDER_ABC, ORDER_CAB, ORDER_CBA = 0, 1, 2

# order of transformed grids (offt_opts.layout)
LAYOUT_NATURAL = 0
LAYOUT_REVERSED = 1


class Opts(ctypes.Structure):
    _fields_ = [
        ("tune", ctypes.c_int),
        ("reps", ctypes.c_int),
        ("normalize_inverse", ctypes.c_int),
        ("forced_plan", ctypes.c_char_p),
        ("cache_path", ctypes.c_char_p),
        ("weights_path", ctypes.c_char_p),
        ("stream", ctypes.c_void_p),
        ("tune_inplace", ctypes.c_int),
        ("use_graph", ctypes.c_int),
        ("layout", ctypes.c_int),
    ]


# name -> (restype, argtypes); every symbol the header declares
_i64 = ctypes.c_int64
_vp = ctypes.c_void_p
_ci = ctypes.c_int
SIGNATURES = {
    "offt_opts_default": (None, [ctypes.POINTER(Opts)]),
    "offt_plan": (_vp, [_i64, _i64, _i64, _ci, _i64]),
    "offt_plan_ex": (_vp, [_i64, _i64, _i64, _ci, _i64, ctypes.POINTER(Opts)]),
    "offt_exec_fwd": (_ci, [_vp, _vp, _vp, _vp]),
    "offt_exec_bwd": (_ci, [_vp, _vp, _vp, _vp]),
    "offt_exec_bwd_norm": (_ci, [_vp, _vp, _vp, _ci, _vp]),
    "offt_destroy": (_ci, [_vp]),
    "offt_plan_passes": (_ci, [_vp]),
    "offt_exec_pass": (_ci, [_vp, _ci, _ci, _vp, _vp, _vp]),
    "offt_exec_range": (_ci, [_vp, _ci, _ci, _ci, _vp, _vp, _vp]),
    "offt_copy_pass": (_ci, [_vp, _ci, _vp, _vp, _vp]),
    "offt_exec_noalloc": (_ci, [_i64, _i64, _i64, _ci, _i64, _ci, _ci, _vp, _vp, _vp]),
    "offt_plan_describe": (_ci, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    "offt_workspace_bytes": (_i64, [_vp]),
    "offt_last_error": (_ci, []),
    "offt_error_string": (ctypes.c_char_p, [_ci]),
    "offt_twiddles": (_ci, [_i64, _ci, _vp]),
    "offt_default_plan_string": (_ci, [_i64, _i64, _i64, _ci, ctypes.c_char_p, ctypes.c_size_t]),
    "offt_plan_string": (_ci, [_i64, _i64, _i64, _ci, _ci, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_size_t]),
    "offt_plan_nd": (_vp, [_ci, ctypes.POINTER(_i64), _ci, _i64, ctypes.POINTER(Opts)]),
    "offt_plan_string_nd": (_ci, [_ci, ctypes.POINTER(_i64), _ci, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_size_t]),
    "offt_feature_dim": (_ci, []),
    "offt_candidates": (_ci, [_i64, _i64, _i64, _ci, _i64, ctypes.c_char_p, ctypes.c_size_t,
                              ctypes.POINTER(ctypes.c_float), _ci]),
    "offt_tune_table": (_ci, [_i64, _i64, _i64, _ci, _i64, _ci, _vp, ctypes.c_size_t, _vp,
                              ctypes.POINTER(ctypes.c_float), _ci]),
    "offt_selector_choose": (_ci, [_i64, _i64, _i64, _ci, _i64, ctypes.c_char_p, ctypes.c_char_p,
                                   ctypes.c_size_t]),
    "offt_plan_features": (_ci, [_i64, _i64, _i64, _ci, _i64, ctypes.c_char_p, ctypes.POINTER(ctypes.c_float)]),
    "offt_selector_scores": (_ci, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_float), _ci,
                                   ctypes.POINTER(ctypes.c_float)]),
    "offt_mlp_nparams": (_i64, [_ci, _ci]),
    "offt_mlp_init_params": (None, [_ci, _ci, ctypes.c_uint64, ctypes.POINTER(ctypes.c_float)]),
    "offt_mlp_create": (_vp, [_ci, _ci, _ci, ctypes.POINTER(ctypes.c_float), ctypes.c_uint64]),
    "offt_mlp_destroy": (_ci, [_vp]),
    "offt_mlp_get_params": (_ci, [_vp, ctypes.POINTER(ctypes.c_float)]),
    "offt_mlp_set_params": (_ci, [_vp, ctypes.POINTER(ctypes.c_float)]),
    "offt_mlp_forward": (_ci, [_vp, _vp, _vp, _ci, _vp, _vp]),
    "offt_mlp_gradient": (_ci, [_vp, _vp, _vp, _vp, _ci, _vp, _vp, _vp]),
    "offt_mlp_adam": (_ci, [_vp, _vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp]),
    "offt_plan_many": (_vp, [_ci, ctypes.POINTER(_i64), _ci, ctypes.POINTER(Opts)]),
    "offt_many_offset": (_i64, [_vp, _ci]),
    "offt_exec_many": (_ci, [_vp, _vp, _vp, _ci, _ci, _vp]),
    "offt_exec_many_fwd": (_ci, [_vp, _vp, _vp, _vp]),
    "offt_exec_many_bwd": (_ci, [_vp, _vp, _vp, _vp]),
    "offt_many_status": (_ci, [_vp]),
    "offt_plan_dist": (_vp, [_i64, _i64, _i64, _ci, _ci, _ci, _ci, ctypes.POINTER(Opts)]),
    "offt_dist_method": (_ci, [_vp]),
    "offt_dist_method_times": (_ci, [_vp, ctypes.POINTER(ctypes.c_float)]),
    "offt_dist_count": (_i64, [_vp, _ci, _ci, _ci, _ci]),
    "offt_dist_block": (_i64, [_vp, _ci, _ci, ctypes.POINTER(_i64)]),
    "offt_dist_exec_steps": (_ci, [_vp, _ci, _ci, _ci, _vp, _vp, _vp]),
    "offt_pass_bytes": (_i64, [_i64, _i64, _i64, _ci, _i64]),
    "offt_decomp_start": (_i64, [_i64, _i64, _i64, _i64, _i64]),
    "offt_transpose_count": (_i64, [_i64, _i64, _i64, _i64, _ci, _i64, _i64]),
    "offt_transpose_volume": (_i64, [_i64, _i64, _i64, _i64, _ci]),
}

_lib = None


class OfftError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = error_string(code) if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


def load():
    """Load libofft.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it first (python -m paper_1501_07350_amd.build "
            "or __graft_entry__.build()); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def error_string(code: int) -> str:
    return load().offt_error_string(code).decode()


def last_error() -> int:
    return load().offt_last_error()


def check(rc: int, what: str = ""):
    if rc < 0:
        raise OfftError(rc, what)
    return rc


def default_opts() -> Opts:
    o = Opts()
    load().offt_opts_default(ctypes.byref(o))
    return o
