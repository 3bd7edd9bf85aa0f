"""ctypes loader for ``libmoff.so``: argument marshalling only, no computation."""
from __future__ import annotations

import ctypes as C
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmoff.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "moff.h")

MOFF_OK, MOFF_E_INVALID, MOFF_E_BUDGET, MOFF_E_DEVICE, MOFF_E_UNSUPPORTED, MOFF_E_STATE = range(6)
FFT_FP32, FFT_SPLIT_FP16, FFT_SPLIT_BF16, FFT_GEMM_FP16 = range(4)
ACC_FP32, ACC_FP64_COMP = range(2)
VOLT_INT8, VOLT_C64 = range(2)
KERNEL_DIAG, KERNEL_JONES = range(2)
PIPELINE_TWO_PASS, PIPELINE_STREAM = range(2)


class PlanDesc(C.Structure):
    _fields_ = [
        ("n_ant", C.c_int32), ("n_pol", C.c_int32), ("n_chan", C.c_int32), ("ksize", C.c_int32),
        ("ant_xy_m", C.POINTER(C.c_double)), ("freq_hz", C.POINTER(C.c_double)),
        ("grid_n", C.POINTER(C.c_int32)), ("cell_lambda", C.c_double),
        ("fft_mode", C.c_int32), ("acc_mode", C.c_int32), ("time_block", C.c_int32), ("volt_format", C.c_int32),
        ("chans_per_block", C.c_int32), ("time_group", C.c_int32), ("kernel_mode", C.c_int32),
        ("n_tap", C.c_int32),
    ]


_P = C.c_void_p
_SIGS = {
    "moff_plan": ([C.POINTER(PlanDesc), C.POINTER(_P)], C.c_int),
    "moff_workspace_size": ([_P, C.POINTER(C.c_size_t)], C.c_int),
    "moff_acc_size": ([_P, C.POINTER(C.c_size_t)], C.c_int),
    "moff_image_size": ([_P, C.POINTER(C.c_size_t)], C.c_int),
    "moff_grid_n": ([_P, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
    "moff_chan_offset": ([_P, C.c_int32, C.POINTER(C.c_int64)], C.c_int),
    "moff_bind": ([_P, _P, C.c_size_t, _P], C.c_int),
    "moff_set_kernels": ([_P, _P, _P], C.c_int),
    "moff_set_kernels_phased": ([_P, _P, _P, _P], C.c_int),
    "moff_set_pipeline": ([_P, C.c_int32], C.c_int),
    "moff_set_taps": ([_P, C.POINTER(C.c_int32), _P], C.c_int),
    "moff_correlate_tap": ([_P, _P, C.c_int64, _P, _P, _P], C.c_int),
    "moff_cal_size": ([_P, C.POINTER(C.c_size_t)], C.c_int),
    "moff_cal_accumulate": ([_P, _P, _P, C.c_int64, _P, _P], C.c_int),
    "moff_cal_solve": ([_P, _P, _P, _P, _P], C.c_int),
    "moff_stream_status": ([_P, C.POINTER(C.c_int32)], C.c_int),
    "moff_grid": ([_P, _P, C.c_int64, _P, _P], C.c_int),
    "moff_fft": ([_P, _P, C.c_int64, _P], C.c_int),
    "moff_accumulate": ([_P, _P, C.c_int64, _P, _P], C.c_int),
    "moff_correlate": ([_P, _P, C.c_int64, _P, _P], C.c_int),
    "moff_read_image": ([_P, _P, C.c_int64, C.c_int32, _P, _P], C.c_int),
    "moff_debug_unpack": ([_P, _P, _P, _P], C.c_int),
    "moff_probe": ([C.c_int32, C.c_int32, C.c_int32, _P, _P], C.c_int),
    "moff_debug_tile_counts": ([_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32)], C.c_int),
    "moff_debug_tiles": ([_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "moff_workspace_size_for": ([_P, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)], C.c_int),
    "moff_set_launch_shape": ([_P, C.c_int32, C.c_int32, C.c_int32], C.c_int),
    "moff_get_launch_shape": ([_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "moff_autotune": ([_P, _P, C.c_int64, _P, _P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                       C.POINTER(C.c_double)], C.c_int),
    "moff_autotune_cached": ([_P, C.c_char_p, _P, C.c_int64, _P, _P, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                              C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_int32)], C.c_int),
    "moff_autotune_key": ([_P, C.c_char_p, C.c_size_t], C.c_int),
    "moff_correlate_graph": ([_P, _P, C.c_int64, _P, _P], C.c_int),
    "moff_correlate_noalloc": ([_P, _P, C.c_int64, _P, _P], C.c_int),
    "moff_profile": ([_P, C.c_int32], C.c_int),
    "moff_profile_read": ([_P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
                          C.c_int),
    "moff_plan_destroy": ([_P], None),
    "moff_status_str": ([C.c_int], C.c_char_p),
    "moff_last_error": ([], C.c_char_p),
}

_lib = None


def header_functions():
    """Names of the functions declared in include/moff.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(moff_[a-z_0-9]+)\s*\(", text)))


def load():
    """Loads the built library (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib
