"""ctypes binding of the C ABI in ``include/lct.h``.

Argument marshalling only: every transform step runs in the HIP library
``liblct_mi355x.so`` built in-tree by ``paper_0912_1379_amd/build.py``.  When
the library is missing this module raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# LCT_LIBRARY names another build of the same ABI (the host-only sanitized
# library of build.py --sanitize, for the CPU suite); unset, the in-tree library.
LIBPATH = os.environ.get("LCT_LIBRARY") or os.path.join(HERE, "liblct_mi355x.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lct.h")

LCT_OK = 0
LCT_ERR_ARG = -1
LCT_ERR_NOT_UNIMODULAR = -2
LCT_ERR_UNSUPPORTED_N = -3
LCT_ERR_DOMAIN = -4
LCT_ERR_WORKSPACE = -5
LCT_ERR_HIP = -6
LCT_ERR_UNSUPPORTED = -7

LCT_FP32 = 0
LCT_FP64 = 1
LCT_FP32_SPLITBF16 = 2

LCT_TUNE_LCT = 0
LCT_TUNE_FRFT = 1


class TuneResult(ctypes.Structure):
    """lct_tune_result of include/lct.h."""
    _fields_ = [("kind", ctypes.c_int32), ("candidates", ctypes.c_int32), ("best_us", ctypes.c_double),
                ("default_us", ctypes.c_double), ("batch", ctypes.c_int64), ("config", ctypes.c_char * 160)]

_lib = None

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_d = ctypes.c_double
_int = ctypes.c_int
_dp = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes); mirrors include/lct.h
SIGNATURES = {
    "lct_plan_create": (_int, [ctypes.POINTER(_vp), _i64, _d, _d, _d, _d]),
    "lct_plan_create_ex": (_int, [ctypes.POINTER(_vp), _i64, _d, _d, _d, _d, _int]),
    "lct_plan_create_scaled": (_int, [ctypes.POINTER(_vp), _i64, _d, _d, _d, _d, _d, _int]),
    "lct_plan_destroy": (None, [_vp]),
    "lct_exec": (_int, [_vp, _vp, _vp, _i64, _vp]),
    "lct_exec_many": (_int, [_i64, _int, _vp, _vp, _vp, _i64, _vp]),
    "lct_exec_adjoint": (_int, [_vp, _vp, _vp, _i64, _vp]),
    "lct_exec_many_adjoint": (_int, [_i64, _int, _vp, _vp, _vp, _i64, _vp]),
    "lct_param_grad_many": (_int, [_i64, _int, _vp, _vp, _vp, _vp, _i64, _vp]),
    "frft_exec": (_int, [_vp, _d, _d, _vp, _vp, _i64, _vp]),
    "frft_exec_many": (_int, [_i64, _int, _vp, _vp, _vp, _i64, _vp]),
    "frft_workspace_size": (ctypes.c_size_t, [_i64, _int, _i64]),
    "frft_exec_ws": (_int, [_vp, _d, _d, _vp, _vp, _i64, _vp, ctypes.c_size_t, _vp]),
    "frft_exec_many_ws": (_int, [_i64, _int, _vp, _vp, _vp, _i64, _vp, ctypes.c_size_t, _vp]),
    "frft_exec_noalloc": (_int, [_vp, _d, _d, _vp, _vp, _i64, _vp]),
    "lct_oversampled_workspace_size": (ctypes.c_size_t, [_i64, _int, _int, _i64]),
    "lct_exec_oversampled": (_int, [_vp, _int, _vp, _vp, _i64, _vp, ctypes.c_size_t, _vp]),
    "lct_complex_exec": (_int, [_i64, _int, _d, _d, _d, _d, _d, _d, _vp, _vp, _i64, _vp]),
    "lct_complex_nodes": (_int, [_i64, _d, _d, _dp]),
    "lct_same_grid_exec": (_int, [_i64, _int, _d, _d, _d, _d, _d, _d, _vp, _vp, _i64, _vp, ctypes.c_size_t, _vp]),
    "lct_ragged_plan_create": (_int, [ctypes.POINTER(_vp), _vp, _i64, _int]),
    "lct_ragged_workspace_size": (ctypes.c_size_t, [_vp]),
    "lct_ragged_info": (_int, [_vp, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(ctypes.c_size_t)]),
    "lct_exec_ragged": (_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "lct_ragged_plan_destroy": (None, [_vp]),
    "lct_workspace_size": (_int, [_vp, _i64, ctypes.POINTER(ctypes.c_size_t)]),
    "lct_check_params": (_int, [_int, _vp, _i64, _vp, _vp]),
    "lct_check_desc": (_int, [_vp, _i64, _vp, _vp]),
    "lct_autotune": (_int, [_i64, _int, _int, _i64, _vp, _vp]),
    "lct_tune_candidates": (_int, [_i64, _int, _int, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(_int)]),
    "lct_tune_get": (_int, [_i64, _int, _int, ctypes.c_char_p, ctypes.c_size_t]),
    "lct_tune_set": (_int, [ctypes.c_char_p]),
    "lct_tune_load": (_int, [ctypes.c_char_p]),
    "lct_tune_save": (_int, [ctypes.c_char_p]),
    "lct_tune_clear": (None, []),
    "lct_nodes": (_int, [_i64, _d, _d, _dp, _dp]),
    "xft_plan_create": (_int, [ctypes.POINTER(_vp), _i64, _int]),
    "xft_plan_destroy": (None, [_vp]),
    "xft_workspace_size": (ctypes.c_size_t, [_i64, _int, _i64]),
    "xft_exec": (_int, [_vp, _d, _d, _vp, _vp, _i64, _vp, ctypes.c_size_t, _vp]),
    "xft_nodes": (_int, [_i64, _dp]),
    "xft_vectors": (_int, [_i64, _dp]),
    "lct_nodes_scaled": (_int, [_i64, _d, _d, _d, _dp, _dp]),
    "lct_strerror": (ctypes.c_char_p, [_int]),
    "lct_max_single_pass": (_i64, [_int]),
}


class LctError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = load().lct_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} ({code})")


def load():
    """Loads the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError(
            f"{LIBPATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "or `python paper_0912_1379_amd/build.py`")
    lib = ctypes.CDLL(LIBPATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int, where: str) -> None:
    if rc != LCT_OK:
        raise LctError(rc, where)
