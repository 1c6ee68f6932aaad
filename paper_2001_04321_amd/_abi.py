"""ctypes declarations of the C ABI in include/ntf.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libntf.so")

NTF_MAX_ORDER = 8
NTF_MAX_RANK = 256

NTF_OK, NTF_EINVAL, NTF_ENOMEM, NTF_EDEVICE, NTF_EUNSUPPORTED, NTF_ENUMERIC = range(6)
NTF_F32, NTF_BF16 = 0, 1
NTF_HER_INIT, NTF_HER_EXTRAPOLATE, NTF_HER_DECIDE = 0, 1, 2
NTF_FLAG_WAIT_TIMEOUT = 0x1
NTF_FLAG_NONFINITE = 0x2


class NtfTensor(C.Structure):
    _fields_ = [("order", C.c_int32), ("dtype", C.c_int32),
                ("dims", C.c_int64 * NTF_MAX_ORDER), ("data", C.c_void_p)]


class NtfTucker(C.Structure):
    _fields_ = [("core", NtfTensor), ("U", C.c_void_p * NTF_MAX_ORDER),
                ("dims", C.c_int64 * NTF_MAX_ORDER)]


class NtfHerParams(C.Structure):
    _fields_ = [("beta0", C.c_double), ("gamma", C.c_double), ("gamma_bar", C.c_double),
                ("eta", C.c_double), ("max_inner", C.c_int32), ("inner_solver", C.c_int32),
                ("inner_tol", C.c_double), ("scheme", C.c_int32), ("reserved", C.c_int32)]


class NtfHerState(C.Structure):
    _fields_ = [("beta", C.c_double), ("beta_bar", C.c_double), ("fhat_prev", C.c_double),
                ("fhat", C.c_double), ("k", C.c_int64), ("restart", C.c_int32),
                ("nrestarts", C.c_int32), ("it", C.c_int64)]


class NtfTrace(C.Structure):
    _fields_ = [("fhat", C.c_void_p), ("beta", C.c_void_p), ("beta_bar", C.c_void_p),
                ("restart", C.c_void_p), ("sweeps", C.c_void_p)]


class NtfProblem(C.Structure):
    _fields_ = [("T", NtfTensor), ("r", C.c_int32), ("reserved", C.c_int32),
                ("A", C.c_void_p * 3), ("state", C.c_void_p), ("trace_fhat", C.c_void_p),
                ("trace_restart", C.c_void_p), ("trace_sweeps", C.c_void_p)]


PTR = C.c_void_p
PTRS = C.POINTER(C.c_void_p)
I64S = C.POINTER(C.c_int64)

# name -> (restype, argtypes); mirrors include/ntf.h
SIGNATURES = {
    "ntf_handle_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    "ntf_handle_destroy": (None, [PTR]),
    "ntf_last_error": (C.c_char_p, []),
    "ntf_status_string": (C.c_char_p, [C.c_int]),
    "ntf_version": (C.c_char_p, []),
    "ntf_device_flags": (C.c_int, [PTR, PTR, C.POINTER(C.c_uint32)]),
    "ntf_handle_set_wait_limit": (C.c_int, [PTR, C.c_double]),
    "ntf_norm2": (C.c_int, [PTR, C.POINTER(NtfTensor), PTR, PTR]),
    "ntf_cast_bf16": (C.c_int, [PTR, PTR, PTR, C.c_int64, PTR]),
    "ntf_mttkrp": (C.c_int, [PTR, C.POINTER(NtfTensor), PTRS, C.c_int32, C.c_int32, PTR, PTR]),
    "ntf_mttkrp_noalloc": (C.c_int, [PTR, C.POINTER(NtfTensor), PTRS, C.c_int32, C.c_int32, PTR,
                                     PTR]),
    "ntf_gram": (C.c_int, [PTR, PTRS, I64S, C.c_int32, C.c_int32, C.c_int32, PTR, PTR, PTR]),
    "ntf_hals_update": (C.c_int, [PTR, PTR, PTR, PTR, C.c_int64, C.c_int32, C.c_int32,
                                  C.c_double, PTR, PTR]),
    "ntf_her_step": (C.c_int, [PTR, C.c_int, PTR, C.POINTER(NtfHerParams), C.c_int32, I64S,
                               C.c_int32, PTRS, PTRS, PTRS, C.c_int32, PTR, PTR]),
    "ntf_error": (C.c_int, [PTR, PTR, PTR, PTR, PTR, C.c_int64, C.c_int32, PTR, PTR]),
    "ntf_solve": (C.c_int, [PTR, C.POINTER(NtfTensor), C.c_int32, PTRS,
                            C.POINTER(NtfHerParams), C.c_int32, PTR, C.c_int32,
                            C.POINTER(NtfTrace), PTR]),
    "ntf_cp_loss": (C.c_int, [PTR, PTR, PTR, PTR, PTR, C.c_int64, C.c_int32, PTR, PTR]),
    "ntf_cp_grad": (C.c_int, [PTR, PTR, PTR, PTR, C.c_int64, C.c_int32, PTR, C.c_float, PTR,
                              PTR]),
    "ntf_solve_batched": (C.c_int, [PTR, C.c_int32, C.POINTER(NtfProblem),
                                    C.POINTER(NtfHerParams), C.c_int32, C.c_int32, PTR]),
    "ntf_residual_norm2": (C.c_int, [PTR, C.POINTER(NtfTensor), PTRS, C.c_int32, PTR, PTR]),
    "ntf_mttkrp_autotune": (C.c_int, [PTR, C.POINTER(NtfTensor), PTRS, C.c_int32, C.c_int32,
                                      PTR, C.c_int32, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_float), PTR]),
    "ntf_tune_export": (C.c_int64, [PTR, C.c_char_p, C.c_int64]),
    "ntf_tune_import": (C.c_int, [PTR, C.c_char_p]),
    "ntf_pgd_update": (C.c_int, [PTR, PTR, PTR, PTR, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                 PTR, PTR]),
    "ntf_solve_apg": (C.c_int, [PTR, C.POINTER(NtfTensor), C.c_int32, PTRS, C.c_int32,
                                C.c_double, PTR, PTR, PTR]),
    "ntf_solve_ibpg": (C.c_int, [PTR, C.POINTER(NtfTensor), C.c_int32, PTRS, C.c_int32,
                                 C.c_int32, C.c_double, C.c_double, PTR, PTR]),
    "ntf_tucker_mttkrp": (C.c_int, [PTR, C.POINTER(NtfTucker), PTRS, C.c_int32, C.c_int32, PTR,
                                    PTR]),
    "ntf_tucker_norm2": (C.c_int, [PTR, C.POINTER(NtfTucker), PTR, PTR]),
    "ntf_solve_tucker": (C.c_int, [PTR, C.POINTER(NtfTucker), C.c_int32, PTRS,
                                   C.POINTER(NtfHerParams), C.c_int32, PTR, C.c_int32,
                                   C.POINTER(NtfTrace), PTR]),
    "ntf_admm_update": (C.c_int, [PTR, PTR, PTR, PTR, C.c_int64, C.c_int32, C.c_int32,
                                  C.c_double, PTR, PTR]),
    "ntf_mttkrp_multi": (C.c_int, [PTR, C.POINTER(NtfTensor), PTRS, C.c_int32, C.c_int32, PTRS,
                                   PTR]),
}

_lib = None


class NtfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_status_name(status)}: {msg}")
        self.status = status


def _status_name(s: int) -> str:
    names = ["NTF_OK", "NTF_EINVAL", "NTF_ENOMEM", "NTF_EDEVICE", "NTF_EUNSUPPORTED",
             "NTF_ENUMERIC"]
    return names[s] if 0 <= s < len(names) else f"status {s}"


def lib():
    """Load libntf.so (built in-tree). Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing; build it with `python -m paper_2001_04321_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != NTF_OK:
        msg = lib().ntf_last_error()
        raise NtfError(status, msg.decode() if msg else "")


def ptr_array(ptrs) -> C.Array:
    arr = (C.c_void_p * len(ptrs))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr


def i64_array(vals) -> C.Array:
    arr = (C.c_int64 * len(vals))()
    for i, v in enumerate(vals):
        arr[i] = int(v)
    return arr
