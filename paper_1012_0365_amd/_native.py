"""ctypes binding of libblws.so (the C ABI in include/blws.h).

Argument marshalling only: every step of the computation runs in the library's
HIP kernels. Loading fails loudly when the library has not been built; there is
no fallback path.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libblws.so")

BLWS_FP64, BLWS_FP32, BLWS_BF16, BLWS_BF16X3 = 0, 1, 2, 3
# start blocks of blws_svt_lanczos (include/blws.h, BLWS_START_*)
STARTS = {"split": 0, "aug": 1, "left": 2, "right": 3}
STATUS = {0: "ok", 1: "not converged", -1: "invalid argument", -2: "out of device memory",
          -3: "device error", -4: "NaN or Inf encountered", -5: "unsupported"}


class SvtOpts(ctypes.Structure):
    _fields_ = [("pow_steps", ctypes.c_int), ("seed", ctypes.c_ulonglong)]


class AlmOpts(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("rho", ctypes.c_double),
        ("mu0_scale", ctypes.c_double),
        ("mu_max_factor", ctypes.c_double),
        ("sv0", ctypes.c_int),
        ("sv_step_frac", ctypes.c_double),
        ("b_round", ctypes.c_int),
        ("pow_steps", ctypes.c_int),
        ("seed", ctypes.c_ulonglong),
        ("norm_steps", ctypes.c_int),
        ("norm_rtol", ctypes.c_double),
        ("b_max", ctypes.c_int),
        ("ladder_tol", ctypes.c_double),
        ("svt_start", ctypes.c_int),
        ("k_blocks", ctypes.c_int),
        ("ladder3_tol", ctypes.c_double),
    ]


class SvtMcOpts(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("rank_step", ctypes.c_int),
        ("b_round", ctypes.c_int),
        ("b_max", ctypes.c_int),
        ("pow_steps", ctypes.c_int),
        ("seed", ctypes.c_ulonglong),
        ("norm_steps", ctypes.c_int),
        ("norm_rtol", ctypes.c_double),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("iters", ctypes.c_int),
        ("rank", ctypes.c_int),
        ("b_final", ctypes.c_int),
        ("fallbacks", ctypes.c_int),
        ("nnz_E", ctypes.c_longlong),
        ("rel_residual", ctypes.c_double),
        ("norm2_D", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("iters_bf16", ctypes.c_int),
        ("refined", ctypes.c_int),
        ("iters_bf16x3", ctypes.c_int),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int), ("mem_budget", ctypes.c_size_t),
                ("group_products", ctypes.c_int), ("group_window_us", ctypes.c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_longlong),
        ("completed", ctypes.c_longlong),
        ("failed", ctypes.c_longlong),
        ("active", ctypes.c_int),
        ("queued", ctypes.c_int),
        ("max_active", ctypes.c_int),
        ("mem_in_use", ctypes.c_size_t),
        ("mem_peak", ctypes.c_size_t),
        ("mem_budget", ctypes.c_size_t),
        ("grouped_launches", ctypes.c_longlong),
        ("grouped_products", ctypes.c_longlong),
        ("max_group", ctypes.c_int),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


# (name, restype, argtypes) for every exported entry point
_vp, _i, _d, _ll, _ull = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong, \
    ctypes.c_ulonglong
SIGNATURES = {
    "blws_create": (_i, [ctypes.POINTER(_vp), _i]),
    "blws_destroy": (_i, [_vp]),
    "blws_status_string": (ctypes.c_char_p, [_i]),
    "blws_last_error": (ctypes.c_char_p, [_vp]),
    "blws_default_alm_opts": (None, [ctypes.POINTER(AlmOpts)]),
    "blws_default_svt_opts": (None, [ctypes.POINTER(SvtOpts)]),
    "blws_svt": (_i, [_vp, _vp, _i, _i, _i, _vp, _i, _d, _i, _vp, _i, _vp, _i, _i, _vp, _vp, _vp,
                      _i, ctypes.POINTER(SvtOpts)]),
    "blws_svt_lanczos": (_i, [_vp, _vp, _i, _i, _vp, _i, _d, _i, _i, _i, _vp, _i, _vp, _i, _vp,
                              _vp, _vp, _i]),
    "blws_svt_noalloc": (_i, [_vp, _vp, _i, _i, _i, _vp, _i, _d, _i, _vp, _i, _vp, _i, _i, _vp,
                              _vp, _vp, _i, ctypes.POINTER(SvtOpts)]),
    "blws_rpca_solve": (_i, [_vp, _vp, _i, _i, _i, _vp, _i, _d, ctypes.POINTER(AlmOpts), _vp, _i,
                             _vp, _i, ctypes.POINTER(SolveInfo)]),
    "blws_default_mc_opts": (None, [ctypes.POINTER(AlmOpts)]),
    "blws_mc_solve": (_i, [_vp, _vp, _i, _i, _i, _i, _vp, _vp, _vp, ctypes.POINTER(AlmOpts), _i,
                           _vp, _i, _vp, _vp, _i, ctypes.POINTER(SolveInfo)]),
    "blws_default_svt_mc_opts": (None, [ctypes.POINTER(SvtMcOpts)]),
    "blws_mc_svt_solve": (_i, [_vp, _vp, _i, _i, _i, _i, _vp, _vp, _vp, ctypes.POINTER(SvtMcOpts),
                               _i, _vp, _i, _vp, _vp, _i, ctypes.POINTER(SolveInfo)]),
    "blws_fill_uniform": (_i, [_vp, _vp, _i, _i, _vp, _i, _ull, _ull]),
    "blws_gemm_f64": (_i, [_vp, _vp, _i, _i, _i, _i, _d, _vp, _i, _vp, _i, _d, _vp, _i]),
    "blws_gemm_lp": (_i, [_vp, _vp, _i, _i, _i, _i, _i, _vp, _i, _vp, _i, _vp, _i]),
    "blws_gemm_bf16x3": (_i, [_vp, _vp, _i, _i, _i, _i, _vp, _vp, _i, _vp, _i, _vp, _i]),
    "blws_small_svd_f64": (_i, [_vp, _vp, _i, _vp, _i, _vp, _vp, _vp]),
    "blws_cold_block": (_i, [_vp, _vp, _i, _i, _i, _vp, _i, _i, _i, _ull, _ull, _vp, _i, _vp,
                             _i]),
    "blws_default_server_opts": (None, [ctypes.POINTER(ServerOpts)]),
    "blws_server_create": (_i, [ctypes.POINTER(_vp), _i, ctypes.POINTER(ServerOpts)]),
    "blws_server_destroy": (_i, [_vp]),
    "blws_server_submit_rpca": (_i, [_vp, _i, _i, _i, _vp, _i, _d, ctypes.POINTER(AlmOpts), _vp,
                                     _i, _vp, _i, ctypes.POINTER(_ll)]),
    "blws_server_submit_mc": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp, ctypes.POINTER(AlmOpts),
                                   _i, _vp, _i, _vp, _vp, _i, ctypes.POINTER(_ll)]),
    "blws_server_poll": (_i, [_vp, _ll, ctypes.POINTER(_i), ctypes.POINTER(SolveInfo)]),
    "blws_server_wait": (_i, [_vp, _ll, ctypes.POINTER(SolveInfo)]),
    "blws_server_get_stats": (_i, [_vp, ctypes.POINTER(ServerStats)]),
    "blws_server_last_error": (ctypes.c_char_p, [_vp]),
    "blws_set_plan_target": (_i, [_i]),
    "blws_timing_enable": (_i, [_vp, _i]),
    "blws_timing_list": (_i, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    "blws_timing_only": (_i, [_vp, ctypes.c_char_p]),
    "blws_timing_get": (_i, [_vp, ctypes.c_char_p, ctypes.POINTER(_ll), ctypes.POINTER(_d),
                             ctypes.POINTER(_d), ctypes.POINTER(_d)]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libblws.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python paper_1012_0365_amd/build.py` "
                "(or __graft_entry__.build()); the library has no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class BlwsError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status


def check(status: int, ctx=None) -> int:
    if status < 0:
        detail = lib().blws_last_error(ctx).decode() if ctx is not None else ""
        raise BlwsError(status, detail)
    return status
