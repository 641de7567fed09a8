"""ctypes declarations of the C ABI in include/ens.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libensdns.so")

ENS_OK, ENS_E_INVALID, ENS_E_OOM, ENS_E_HIP, ENS_E_UNSUPPORTED, ENS_E_STATE, ENS_E_DIVERGED = 0, -1, -2, -3, -4, -5, -6
ENS_FP64, ENS_FP32 = 0, 1
ENS_NPASS = 7
ENS_NMOM = 32
ENS_MIX_STATIC_MAX = 1023
PASS_NAMES = ("band", "zinv", "yinv", "xpass", "yfwd", "zfwd_update", "end_step")

# every symbol the header declares
EXPORTS = ("ens_create", "ens_destroy", "ens_last_error", "ens_set_graphs", "ens_member_workspace_bytes",
           "ens_member_init", "ens_member_set_state", "ens_member_get_state", "ens_step", "ens_profile_step",
           "ens_get_diag", "ens_accumulate_stats", "ens_stats_len", "ens_get_stats", "ens_reset_stats",
           "ens_member_set_diag", "ens_set_stats",
           "ens_mix_len", "ens_mix", "ens_mix_noalloc", "ens_mix_table", "ens_lambda_pdf_from_cf", "ens_scale_gap", "ens_spectrum", "ens_integral_scales", "ens_member_refine",
           "ens_fft_pencils", "ens_autotune", "ens_set_variant", "ens_get_variant")


class MemberDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("precision", ctypes.c_int32), ("box", ctypes.c_double),
                ("nu", ctypes.c_double), ("eps_ref", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("kf_lo", ctypes.c_double), ("kf_hi", ctypes.c_double), ("dt", ctypes.c_double),
                ("cfl", ctypes.c_double), ("seed", ctypes.c_uint64), ("k_peak", ctypes.c_double),
                ("e0", ctypes.c_double), ("visc_mode", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class HistDesc(ctypes.Structure):
    _fields_ = [("qr_bins", ctypes.c_int32), ("q_lo", ctypes.c_double), ("q_hi", ctypes.c_double),
                ("r_lo", ctypes.c_double), ("r_hi", ctypes.c_double),
                ("log_bins", ctypes.c_int32), ("log10_lo", ctypes.c_double), ("log10_hi", ctypes.c_double),
                ("a_bins", ctypes.c_int32), ("a_lo", ctypes.c_double), ("a_hi", ctypes.c_double),
                ("eps_ref", ctypes.c_double), ("nu_ref", ctypes.c_double)]


class Diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double), ("E", ctypes.c_double), ("D", ctypes.c_double),
                ("inj", ctypes.c_double), ("E_f", ctypes.c_double), ("umax", ctypes.c_double),
                ("cfl", ctypes.c_double), ("rlambda", ctypes.c_double), ("kmax_eta", ctypes.c_double),
                ("step", ctypes.c_int64), ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class EnsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ens status {status}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libensdns.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(the HIP library is the only implementation of this package)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sz = ctypes.c_size_t
    P = ctypes.POINTER
    proto = {
        "ens_create": [P(vp), ctypes.c_int, P(HistDesc)],
        "ens_destroy": [vp],
        "ens_set_graphs": [vp, i32],
        "ens_member_workspace_bytes": [vp, P(MemberDesc), P(sz)],
        "ens_member_init": [vp, P(MemberDesc), vp, sz, vp, P(i32)],
        "ens_member_set_state": [vp, i32, vp, vp],
        "ens_member_get_state": [vp, i32, vp, vp],
        "ens_step": [vp, P(i32), i32, i32, vp],
        "ens_profile_step": [vp, P(i32), i32, vp, P(dp)],
        "ens_get_diag": [vp, i32, P(Diag)],
        "ens_accumulate_stats": [vp, P(i32), i32, vp],
        "ens_stats_len": [vp, P(sz)],
        "ens_get_stats": [vp, i32, P(ctypes.c_uint64), P(dp), P(ctypes.c_uint64)],
        "ens_reset_stats": [vp, i32, vp],
        "ens_member_set_diag": [vp, i32, P(Diag), vp],
        "ens_set_stats": [vp, i32, P(ctypes.c_uint64), P(dp), vp],
        "ens_mix_len": [vp, i32, P(sz)],
        "ens_mix": [vp, P(i32), i32, dp, dp, i32, dp, vp, vp],
        "ens_mix_noalloc": [vp, P(i32), i32, dp, dp, i32, dp, vp, vp],
        "ens_mix_table": [vp, P(i32), i32, vp, i32, dp, dp, vp, vp],
        "ens_lambda_pdf_from_cf": [vp, i32, dp, dp, vp, vp],
        "ens_scale_gap": [vp, P(i32), i32, dp, P(dp), P(dp), P(dp)],
        "ens_spectrum": [vp, i32, i32, vp, vp],
        "ens_integral_scales": [vp, i32, vp, vp],
        "ens_member_refine": [vp, i32, i32, vp],
        "ens_fft_pencils": [i32, i32, i32, i64, vp, vp, vp],
        "ens_autotune": [vp, P(i32), i32, vp, ctypes.c_char_p],
        "ens_set_variant": [vp, i32, i32, i32, i32],
        "ens_get_variant": [vp, i32, i32, i32, P(i32)],
    }
    for name, args in proto.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.ens_last_error.argtypes = []
    L.ens_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status: int) -> int:
    if status != ENS_OK:
        raise EnsError(status, lib().ens_last_error().decode(errors="replace"))
    return status
