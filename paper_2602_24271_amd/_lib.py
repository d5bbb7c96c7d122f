"""ctypes binding of libnshe.so (argument marshalling only).

The library is the only compute path: there is no fallback.  Loading fails
loudly when libnshe.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnshe.so")

NSHE_MAX_L = 24


class NsheParams(ctypes.Structure):
    _fields_ = [("log2_n", ctypes.c_uint32), ("t", ctypes.c_uint64), ("L", ctypes.c_int32),
                ("q_host", ctypes.POINTER(ctypes.c_uint64)), ("P", ctypes.c_uint64),
                ("alpha", ctypes.c_int32), ("P1", ctypes.c_uint64), ("P2", ctypes.c_uint64)]


class NsheInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("L", ctypes.c_int32), ("L_ext", ctypes.c_int32),
                ("squarings", ctypes.c_int32), ("ext_primes", ctypes.c_uint64 * 32),
                ("ct_words", ctypes.c_size_t), ("relin_key_words", ctypes.c_size_t),
                ("depth_budget", ctypes.c_int32), ("lt_depth", ctypes.c_int32),
                ("fresh_bits", ctypes.c_double), ("level_bits", ctypes.c_double),
                ("alpha", ctypes.c_int32), ("dnum", ctypes.c_int32)]


class NsheBudget(ctypes.Structure):
    _fields_ = [("depth_budget", ctypes.c_int32), ("lt_depth", ctypes.c_int32),
                ("fresh_bits", ctypes.c_double), ("level_bits", ctypes.c_double)]


# error codes and constants of include/nshe.h
NSHE_EINVAL, NSHE_ESHAPE, NSHE_ENOMEM, NSHE_EDEVICE = -1, -2, -3, -4
NSHE_EDEPTH, NSHE_ENOKEY, NSHE_EUNSUPPORTED = -5, -6, -7
OPS = {"add": 0, "mul": 1, "mul_plain": 2, "eq": 3, "in": 4, "lt": 5, "between": 6, "join": 7}
NSHE_MARGIN_SITES = 6
NSHE_DEBUG_WIDE_LIFT_WINDOW = 1
NSHE_DEBUG_CHECK_INPUTS = 2


class NsheItem(ctypes.Structure):
    _fields_ = [("x_dev", ctypes.c_void_p), ("y_dev", ctypes.c_void_p),
                ("out_dev", ctypes.c_void_p), ("n_ct", ctypes.c_int32),
                ("y_broadcast", ctypes.c_int32)]


class NsheKernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double), ("work", ctypes.c_double)]


class NsheTuning(ctypes.Structure):
    _fields_ = [("ks_chunk", ctypes.c_int32), ("split_forward", ctypes.c_int32),
                ("ew_block", ctypes.c_int32), ("wave_ct", ctypes.c_int32),
                ("ks_fused", ctypes.c_int32), ("streams", ctypes.c_int32)]


class NsheModmulProbe(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("products_per_s", ctypes.c_double),
                ("fp64_ops_per_s", ctypes.c_double)]


class NsheOverlapProbe(ctypes.Structure):
    _fields_ = [("ms_valu", ctypes.c_double), ("ms_mfma", ctypes.c_double),
                ("ms_both", ctypes.c_double), ("fma_per_s_valu", ctypes.c_double),
                ("fma_per_s_mfma", ctypes.c_double)]


class NsheConvProbe(ctypes.Structure):
    _fields_ = [("coefficients", ctypes.c_uint64), ("ms_fma", ctypes.c_double),
                ("ms_mfma", ctypes.c_double), ("mismatches", ctypes.c_uint64)]


# name -> (restype, argtypes)
_P = ctypes.c_void_p
_I = ctypes.c_int
_SZ = ctypes.c_size_t
SIGNATURES = {
    "nshe_ctx_create": (_I, [ctypes.POINTER(NsheParams), _I, ctypes.POINTER(_P)]),
    "nshe_ctx_destroy": (_I, [_P]),
    "nshe_ctx_info": (_I, [_P, ctypes.POINTER(NsheInfo)]),
    "nshe_set_relin_key": (_I, [_P, _P, _SZ, _P]),
    "nshe_budget_of": (_I, [ctypes.POINTER(NsheParams), ctypes.POINTER(NsheBudget)]),
    "nshe_op_depth": (_I, [_P, _I, _I, ctypes.POINTER(_I)]),
    "nshe_depth_after": (_I, [_P, _I, _I, _I, ctypes.POINTER(_I)]),
    "nshe_set_debug": (_I, [_P, ctypes.c_uint32]),
    "nshe_margin_sites": (_I, [_P, ctypes.POINTER(ctypes.c_uint64), _I, ctypes.POINTER(_I), _P]),
    "nshe_workspace_bytes": (_SZ, [_P, _I]),
    "nshe_sub": (_I, [_P, _P, _P, _P, _I, _P]),
    "nshe_square_relin": (_I, [_P, _P, _P, _I, _P, _SZ, _P]),
    "nshe_mul_relin": (_I, [_P, _P, _P, _P, _I, _P, _SZ, _P]),
    "nshe_multiply": (_I, [_P, _P, _P, _P, _I, _P, _SZ, _P]),
    "nshe_relinearize": (_I, [_P, _P, _P, _I, _P, _SZ, _P]),
    "nshe_eq_mask": (_I, [_P, _P, _P, _P, _I, _I, _P, _SZ, _P]),
    "nshe_eq_mask_noalloc": (_I, [_P, _P, _P, _P, _I, _I, _P]),
    "nshe_batched_workspace_bytes": (_SZ, [_P, _I, ctypes.c_longlong]),
    "nshe_eq_mask_batched": (_I, [_P, ctypes.POINTER(NsheItem), _I, _I, _I, _P, _SZ, _P]),
    "nshe_add": (_I, [_P, _P, _P, _P, _I, _P]),
    "nshe_sum": (_I, [_P, _P, _I, _P, _I, _P]),
    "nshe_in_workspace_bytes": (_SZ, [_P, _I, _I, _I]),
    "nshe_in_mask": (_I, [_P, _P, _P, _I, _P, _I, _I, _I, _P, _SZ, _P]),
    "nshe_compare_workspace_bytes": (_SZ, [_P, _I]),
    "nshe_compare": (_I, [_P, _P, _P, _I, _I, _P, _I, _P, _SZ, _P]),
    "nshe_between": (_I, [_P, _P, _P, _P, _I, _P, _I, _P, _SZ, _P]),
    "nshe_mul_plain": (_I, [_P, _P, _P, _P, _I, _P, _SZ, _P]),
    "nshe_extract": (_I, [_P, _P, _I, _I, _P, _I, _P, _SZ, _P]),
    "nshe_join_workspace_bytes": (_SZ, [_P, _I]),
    "nshe_join_sum": (_I, [_P, _P, _P, _P, ctypes.POINTER(ctypes.c_int32), _I, _P, _I, _P, _SZ,
                           _P]),
    "nshe_set_galois_key": (_I, [_P, ctypes.c_uint32, _P, _SZ, _P]),
    "nshe_galois_elements": (_I, [_P, ctypes.POINTER(ctypes.c_uint32), _I, ctypes.POINTER(_I)]),
    "nshe_rotate": (_I, [_P, _P, ctypes.c_uint32, _P, _I, _P, _SZ, _P]),
    "nshe_sum_slots": (_I, [_P, _P, _P, _I, _P, _SZ, _P]),
    "nshe_get_tuning": (_I, [_P, ctypes.POINTER(NsheTuning)]),
    "nshe_set_tuning": (_I, [_P, ctypes.POINTER(NsheTuning)]),
    "nshe_autotune": (_I, [_P, _P, _I, _I, _P, _SZ, _P, ctypes.POINTER(NsheTuning),
                           ctypes.POINTER(ctypes.c_double)]),
    "nshe_ntt": (_I, [_P, _P, _P, _I, _I, _P, _SZ, _P]),
    "nshe_margin_events": (_I, [_P, ctypes.POINTER(ctypes.c_uint64), _P]),
    "nshe_reset_margin_events": (_I, [_P, _P]),
    "nshe_profile": (_I, [_P, _I]),
    "nshe_profile_read": (_I, [_P, ctypes.POINTER(NsheKernelStat), _I, ctypes.POINTER(_I)]),
    "nshe_last_error": (ctypes.c_char_p, []),
    # measurement entry points (include/nshe_probe.h)
    "nshe_probe_modmul": (_I, [_I, _I, ctypes.POINTER(NsheModmulProbe)]),
    "nshe_probe_fp64_overlap": (_I, [_I, _I, ctypes.POINTER(NsheOverlapProbe)]),
    "nshe_probe_conversion": (_I, [_I, ctypes.POINTER(ctypes.c_uint64), _I,
                                   ctypes.POINTER(ctypes.c_uint64), _I, _SZ, _I,
                                   ctypes.POINTER(NsheConvProbe)]),
    "nshe_probe_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load() -> ctypes.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2602_24271_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class NsheError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nshe error {code}: {msg}")
        self.code = code


def check(rc: int) -> None:
    if rc != 0:
        raise NsheError(rc, load().nshe_last_error().decode())
