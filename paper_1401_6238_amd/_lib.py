"""ctypes binding of libhankel.so (argument marshalling only).

The library is built in-tree by ``paper_1401_6238_amd.build``.  There is no
fallback: if the shared library is missing, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import List

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhankel.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hankel.h")

HK_C64, HK_C128, HK_F32, HK_F64 = 0, 1, 2, 3
HK_MAX_ORDER = 8
HK_PLAN_PERSISTENT = 0x1
HK_PLAN_MULTIKERNEL = 0x2
HK_PLAN_GRAPH = 0x4
HK_PLAN_AUTOTUNE = 0x8
HK_PLAN_POW2 = 0x10

STATUS_NAMES = {
    0: "HK_SUCCESS", 1: "HK_ERR_INVALID_VALUE", 2: "HK_ERR_NULL_POINTER", 3: "HK_ERR_MISALIGNED",
    4: "HK_ERR_WORKSPACE", 5: "HK_ERR_SIZE_LIMIT", 6: "HK_ERR_DEVICE", 7: "HK_ERR_HIP",
    8: "HK_ERR_DEVICE_FAULT", 9: "HK_ERR_NOT_SUPPORTED",
}


class HankelError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        self.code = code
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)} ({detail})")


class hk_problem_t(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32), ("is_block", ctypes.c_int32),
        ("reserved0", ctypes.c_int32), ("reserved1", ctypes.c_int32),
        ("dims", ctypes.c_int64 * HK_MAX_ORDER), ("block_dims", ctypes.c_int64 * HK_MAX_ORDER),
        ("h", ctypes.c_void_p), ("vectors", ctypes.c_void_p * HK_MAX_ORDER),
        ("y", ctypes.c_void_p), ("alpha", ctypes.c_void_p),
    ]


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_PSZ = ctypes.POINTER(ctypes.c_size_t)
_PI64 = ctypes.POINTER(ctypes.c_int64)

_SIGS = {
    "hankel_tvp_workspace_size": [_I, _I, _I64, _PSZ],
    "hankel_tvp": [_I, _P, _I, _I64, _P, _P, _P, _P, _SZ, _P],
    "hankel_tvp_noalloc": [_I, _P, _I, _I64, _P, _P, _P, _P],
    "hankel_mode_products_workspace_size": [_I, _I, _PI64, _P, _I, _I, _PSZ],
    "hankel_mode_products": [_I, _P, _I, _PI64, _P, _P, _P, _P, _SZ, _P],
    "hankel_spectrum_layout": [_I, _I, _PI64, _PI64, _PI64],
    "hankel_spectrum_workspace_size": [_I, _I, _PI64, _I, _PSZ],
    "hankel_spectrum": [_I, _I, _PI64, _I, _P, _P, _P, _SZ, _P],
    "hankel_mode_products_spectral_workspace_size": [_I, _I, _PI64, _P, _P, _I, _I, _PSZ],
    "hankel_mode_products_spectral": [_I, _P, _I, _PI64, _P, _P, _P, _P, _P, _SZ, _P],
    "hankel_tvp_spectral_strided_batched_workspace_size": [_I, _I, _I64, _I64, _PSZ],
    "hankel_tvp_backward_spectral_workspace_size": [_I, _I, _I64, _PSZ],
    "hankel_tvp_backward_spectral": [_I, _P, _I, _I64, _P, _P, _P, _P, _P, _P, _SZ, _P],
    "hankel_tvp_spectral_strided_batched": [_I, _P, _I, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _SZ, _P],
    "block_hankel_tvp_workspace_size": [_I, _I, _PI64, _PI64, _P, _I, _I, _PSZ],
    "block_hankel_tvp_layout": [_I, _I, _PI64, _PI64, _I64, _PI64, _PI64],
    "block_hankel_tvp": [_I, _P, _I, _PI64, _PI64, _P, _P, _P, _P, _SZ, _P],
    "block_hankel_tvp_levels_workspace_size": [_I, _I, _I, _PI64, _P, _I, _I, _PSZ],
    "block_hankel_tvp_levels": [_I, _P, _I, _I, _PI64, _P, _P, _P, _P, _SZ, _P],
    "hk_plan_create": [ctypes.POINTER(_P), _I, _P, _I64, ctypes.c_uint],
    "hk_plan_workspace_size": [_P, _PSZ],
    "hk_plan_execute": [_P, _P, _SZ, _P],
    "hk_plan_status": [_P],
    "hk_plan_destroy": [_P],
    "hankel_tvp_batched_workspace_size": [_I, _P, _I64, _PSZ],
    "hankel_tvp_batched": [_I, _P, _I64, _P, _SZ, _P],
    "hankel_mode_products_batched_workspace_size": [_I, _P, _I64, _PSZ],
    "hankel_mode_products_batched": [_I, _P, _I64, _P, _SZ, _P],
    "block_hankel_tvp_batched_workspace_size": [_I, _P, _I64, _PSZ],
    "block_hankel_tvp_batched": [_I, _P, _I64, _P, _SZ, _P],
    "hankel_tvp_backward_workspace_size": [_I, _I, _I64, _PSZ],
    "hankel_tvp_save_spectrum_workspace_size": [_I, _I, _I64, _I64, _PSZ],
    "hankel_mode_products_backward_workspace_size": [_I, _I, _PI64, _I, _I, _PSZ],
    "hankel_mode_products_backward": [_I, _P, _I, _PI64, _P, _P, _P, _P, _P, _P, _SZ, _P],
    "block_hankel_tvp_backward_workspace_size": [_I, _I, _PI64, _PI64, _I, _I, _PSZ],
    "block_hankel_tvp_backward": [_I, _P, _I, _PI64, _PI64, _P, _P, _P, _P, _P, _P, _SZ, _P],
    "hankel_tvp_save_spectrum": [_I, _P, _I64, _I, _I64, _P, _I64, _P, _I64, _P, _P, _I64, _I64, _P, _SZ, _P],
    "hankel_tvp_backward_spectral_strided_batched_workspace_size": [_I, _I, _I64, _I64, _PSZ],
    "hankel_tvp_backward_spectral_strided_batched": [_I, _P, _I64, _I, _I64, _P, _I64, _P, _I64, _P, _P, _I64, _P,
                                                     _I64, _I64, _P, _SZ, _P],
    "hankel_tvp_backward": [_I, _P, _I, _I64, _P, _P, _P, _P, _P, _P, _SZ, _P],
    "hankel_tvp_strided_batched_workspace_size": [_I, _I, _I64, _I64, _PSZ],
    "hankel_tvp_strided_batched": [_I, _P, _I64, _I, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _SZ, _P],
    "hankel_tvp_backward_strided_batched_workspace_size": [_I, _I, _I64, _I64, _PSZ],
    "hankel_tvp_backward_strided_batched": [_I, _P, _I64, _I, _I64, _P, _I64, _P, _I64, _P, _P, _I64, _P,
                                            _I64, _I64, _P, _SZ, _P],
    "block_hankel_tvp_strided_batched_workspace_size": [_I, _I, _PI64, _PI64, _I64, _PSZ],
    "block_hankel_tvp_strided_batched": [_I, _P, _I64, _I, _PI64, _PI64, _P, _I64, _P, _I64, _P, _I64, _P,
                                         _SZ, _P],
    "hk_fft_layout": [_I64, _PI64, _PI64, _PI64],
    "hk_set_fft_lengths": [_I],
    "hk_get_fft_lengths": [],
    "hk_autotune_tvp": [_I, _I, _I64, _I],
    "hk_autotune": [_I, _I, _I, _I64, _PI64, _PI64, _I64, _I],
    "hk_tune_save": [ctypes.c_char_p],
    "hankel_tensor_matrix_workspace_size": [_I, _I, _I64, _I64, ctypes.POINTER(ctypes.c_size_t)],
    "hankel_tensor_matrix": [_I, _P, _I, _I64, _I64, _P, _P, _P, ctypes.c_size_t, _P],
    "hk_plan_set_wait_bound": [ctypes.c_void_p, ctypes.c_uint32],
    "hk_plan_pass_bytes": [ctypes.c_void_p, _PI64],
    "hk_plan_tune_times": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_uint32)],
    "hk_tune_load": [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)],
    "hk_last_launch_count": [],
    "hk_profile_start": [],
    "hk_profile_stop": [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
    "hk_status_string": [_I],
    "hk_last_error": [],
    "hk_version": [],
}

_lib = None
TUNE_DB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_db.txt")


def lib():
    """Loads libhankel.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_1401_6238_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.hk_status_string.restype = ctypes.c_char_p
        L.hk_last_error.restype = ctypes.c_char_p
        _lib = L
        # schedules measured on MI355X and shipped with the package
        if os.path.exists(TUNE_DB_PATH) and not os.environ.get("HK_NO_TUNE_DB"):
            n = ctypes.c_int(0)
            rc = L.hk_tune_load(TUNE_DB_PATH.encode(), ctypes.byref(n))
            if rc != 0:
                raise RuntimeError(f"{TUNE_DB_PATH}: " + L.hk_last_error().decode(errors="replace"))
    return _lib


def check(code: int, where: str):
    if code != 0:
        detail = lib().hk_last_error().decode(errors="replace")
        raise HankelError(code, where, detail)


def header_functions() -> List[str]:
    """Names of the functions declared in include/hankel.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(?:hk_status_t|const char \*|int)\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", text)
    return sorted(set(names))
