"""CPU oracle (test infrastructure only).

Plain FP64 C implementation of BLWS singular value thresholding and of the
inexact-ALM RPCA / matrix-completion loops that host it, loaded with ctypes.
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the GPU library never does and shares no
code with it.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "blws_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (generic x86-64, OpenMP)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
               "-Wno-unused-result", _SRC, "-o", _SO + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


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
        ("seed", ctypes.c_uint64),
        ("norm_steps", ctypes.c_int),
        ("norm_rtol", ctypes.c_double),
        ("svt_start", ctypes.c_int),
        ("k_blocks", ctypes.c_int),
    ]


# start blocks of the literal block Lanczos on [[0, W], [W^T, 0]] (Sec. 4.1)
START_SPLIT, START_AUG, START_LEFT, START_RIGHT = 0, 1, 2, 3
STARTS = {"split": START_SPLIT, "aug": START_AUG, "left": START_LEFT, "right": START_RIGHT}


class SvtMcOpts(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("rank_step", ctypes.c_int),
        ("b_round", ctypes.c_int),
        ("pow_steps", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("norm_steps", ctypes.c_int),
        ("norm_rtol", ctypes.c_double),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("rank", ctypes.c_int),
        ("b_final", ctypes.c_int),
        ("nnz_E", ctypes.c_longlong),
        ("rel_residual", ctypes.c_double),
        ("norm2_D", ctypes.c_double),
        ("status", ctypes.c_int),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        d = ctypes.POINTER(ctypes.c_double)
        i = ctypes.POINTER(ctypes.c_int)
        L.orc_splitmix64.restype = ctypes.c_uint64
        L.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_predict_rank.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int]
        L.orc_block_width.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_resize_block.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, d,
                                       ctypes.c_uint64, ctypes.c_uint64, d]
        L.orc_rpca_snapshot.argtypes = [ctypes.c_int, ctypes.c_int, d, ctypes.c_double,
                                        ctypes.POINTER(AlmOpts), ctypes.c_int, d, d, d,
                                        ctypes.c_int, i, d]
        L.orc_uniform.restype = ctypes.c_double
        L.orc_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_fill_uniform.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                       ctypes.c_uint64, d]
        L.orc_jacobi_svd.argtypes = [ctypes.c_int, ctypes.c_int, d, d, d, d]
        L.orc_svt_exact.argtypes = [ctypes.c_int, ctypes.c_int, d, ctypes.c_double, d, d, i]
        L.orc_blws_step.argtypes = [ctypes.c_int, ctypes.c_int, d, ctypes.c_double,
                                    ctypes.c_int, d, d, d, d, i]
        L.orc_lanczos_svt.argtypes = [ctypes.c_int, ctypes.c_int, d, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, d, d, d, d, i]
        L.orc_cold_block.argtypes = [ctypes.c_int, ctypes.c_int, d, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, d, d]
        L.orc_spectral_norm_blws.restype = ctypes.c_double
        L.orc_spectral_norm_blws.argtypes = [ctypes.c_int, ctypes.c_int, d, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_uint64, ctypes.c_double,
                                             ctypes.c_int, i]
        L.orc_default_opts.argtypes = [ctypes.POINTER(AlmOpts)]
        L.orc_rpca.argtypes = [ctypes.c_int, ctypes.c_int, d, ctypes.c_double,
                               ctypes.POINTER(AlmOpts), ctypes.c_int, d, d, d, i,
                               ctypes.POINTER(Info)]
        L.orc_mc.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, i, i, d,
                             ctypes.POINTER(AlmOpts), ctypes.c_int, ctypes.c_int, d, d, d, i,
                             ctypes.POINTER(Info)]
        L.orc_default_svt_mc_opts.argtypes = [ctypes.POINTER(SvtMcOpts)]
        L.orc_mc_svt.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, i, i, d,
                                 ctypes.POINTER(SvtMcOpts), ctypes.c_int, ctypes.c_int, d, d, d,
                                 i, ctypes.POINTER(Info)]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def default_opts(**kw) -> AlmOpts:
    o = AlmOpts()
    lib().orc_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def splitmix64(seed: int, counter: int) -> int:
    """The (counter + 1)-th 64-bit output of SplitMix64 seeded with `seed`."""
    return int(lib().orc_splitmix64(seed, counter))


def predict_rank(svp: int, sv: int, step_frac: float, p: int) -> int:
    return int(lib().orc_predict_rank(svp, sv, step_frac, p))


def block_width(sv: int, b_round: int, p: int) -> int:
    return int(lib().orc_block_width(sv, b_round, p))


def resize_block(X, b_new: int, seed: int, stream: int) -> np.ndarray:
    X = _f64(X)
    rows, b_old = X.shape
    Y = np.empty((rows, b_new))
    rc = lib().orc_resize_block(rows, b_old, b_new, _dp(X), seed, stream, _dp(Y))
    if rc < 0:
        raise RuntimeError(f"orc_resize_block failed: {rc}")
    return Y


def rpca_snapshot(D, it: int, lam: float | None = None, b_cap: int = 1024, **opts):
    """State at the start of BLWS-mode RPCA iteration `it` (1-based): returns
    (W, U, V, eps) with U, V the warm block of that iteration."""
    D = _f64(D)
    m, n = D.shape
    o = default_opts(**opts)
    W = np.empty((m, n))
    U = np.empty(m * b_cap)
    V = np.empty(n * b_cap)
    b = ctypes.c_int(0)
    eps = ctypes.c_double(0.0)
    rc = lib().orc_rpca_snapshot(m, n, _dp(D), -1.0 if lam is None else float(lam),
                                 ctypes.byref(o), it, _dp(W), _dp(U), _dp(V), b_cap,
                                 ctypes.byref(b), ctypes.byref(eps))
    if rc < 0:
        raise RuntimeError(f"orc_rpca_snapshot failed: {rc}")
    bb = b.value
    return W, U[: m * bb].reshape(m, bb).copy(), V[: n * bb].reshape(n, bb).copy(), eps.value


def uniform(seed: int, counter: int) -> float:
    return lib().orc_uniform(seed, counter)


def fill_uniform(rows: int, cols: int, seed: int, stream: int) -> np.ndarray:
    X = np.empty((rows, cols))
    lib().orc_fill_uniform(rows, cols, seed, stream, _dp(X))
    return X


def jacobi_svd(W):
    """Thin SVD by one-sided Jacobi: returns U (m x p), S (p,), V (n x p)."""
    W = _f64(W)
    m, n = W.shape
    p = min(m, n)
    U = np.empty((m, p))
    S = np.empty(p)
    V = np.empty((n, p))
    rc = lib().orc_jacobi_svd(m, n, _dp(W), _dp(U), _dp(S), _dp(V))
    if rc < 0:
        raise RuntimeError(f"orc_jacobi_svd failed: {rc}")
    return U, S, V


def svt_exact(W, eps: float):
    """Eq. (4) from the full Jacobi SVD: returns (A, all singular values, rank)."""
    W = _f64(W)
    m, n = W.shape
    A = np.empty((m, n))
    S = np.empty(min(m, n))
    r = ctypes.c_int(0)
    rc = lib().orc_svt_exact(m, n, _dp(W), eps, _dp(A), _dp(S), ctypes.byref(r))
    if rc < 0:
        raise RuntimeError(f"orc_svt_exact failed: {rc}")
    return A, S, r.value


def blws_step(W, eps: float, U, V, want_A: bool = True):
    """One BLWS step from the orthonormal warm block (U, V); returns
    (U_new, V_new, S, A or None, rank)."""
    W = _f64(W)
    m, n = W.shape
    U = np.array(U, dtype=np.float64, order="C", copy=True)
    V = np.array(V, dtype=np.float64, order="C", copy=True)
    b = U.shape[1]
    S = np.empty(b)
    A = np.empty((m, n)) if want_A else None
    r = ctypes.c_int(0)
    rc = lib().orc_blws_step(m, n, _dp(W), eps, b, _dp(U), _dp(V), _dp(S),
                             _dp(A) if want_A else None, ctypes.byref(r))
    if rc < 0:
        raise RuntimeError(f"orc_blws_step failed: {rc}")
    return U, V, S, A, r.value


def lanczos_svt(W, eps: float, U, V, start: str = "aug", k: int = 2, want_A: bool = True):
    """Algorithms 2-3 taken literally on the augmented matrix from the start
    block `start` ("split", "aug", "left", "right") built from (U, V), with k
    blocks; returns (U_new, V_new, S, A or None, rank) as blws_step does."""
    W = _f64(W)
    m, n = W.shape
    U = np.array(U, dtype=np.float64, order="C", copy=True)
    V = np.array(V, dtype=np.float64, order="C", copy=True)
    b = U.shape[1]
    S = np.empty(b)
    A = np.empty((m, n)) if want_A else None
    r = ctypes.c_int(0)
    rc = lib().orc_lanczos_svt(m, n, _dp(W), eps, b, STARTS[start], k, _dp(U), _dp(V), _dp(S),
                               _dp(A) if want_A else None, ctypes.byref(r))
    if rc != 0:
        raise RuntimeError(f"orc_lanczos_svt failed: {rc}")
    return U, V, S, A, r.value


def cold_block(W, b: int, pow_steps: int, seed: int, stream_v: int = 1):
    W = _f64(W)
    m, n = W.shape
    U = np.empty((m, b))
    V = np.empty((n, b))
    rc = lib().orc_cold_block(m, n, _dp(W), b, pow_steps, seed, stream_v, _dp(U), _dp(V))
    if rc < 0:
        raise RuntimeError(f"orc_cold_block failed: {rc}")
    return U, V


def spectral_norm_blws(W, bs: int = 16, pow_steps: int = 2, seed: int = 20101202,
                       rtol: float = 1e-13, max_steps: int = 5000):
    W = _f64(W)
    m, n = W.shape
    steps = ctypes.c_int(0)
    s = lib().orc_spectral_norm_blws(m, n, _dp(W), bs, pow_steps, seed, rtol, max_steps,
                                     ctypes.byref(steps))
    return s, steps.value


def rpca(D, lam: float | None = None, mode: str = "exact", want_Y: bool = False, **opts):
    """Inexact-ALM RPCA. mode 'exact' (full Jacobi SVT, the plain form) or 'blws'."""
    D = _f64(D)
    m, n = D.shape
    o = default_opts(**opts)
    A = np.empty((m, n))
    E = np.empty((m, n))
    Y = np.empty((m, n)) if want_Y else None
    trace = np.zeros(o.max_iter, dtype=np.int32)
    info = Info()
    rc = lib().orc_rpca(m, n, _dp(D), -1.0 if lam is None else float(lam), ctypes.byref(o),
                        {"exact": 0, "blws": 1}[mode], _dp(A), _dp(E),
                        _dp(Y) if want_Y else None, _ip(trace), ctypes.byref(info))
    if rc < 0:
        raise RuntimeError(f"orc_rpca failed: {rc}")
    out = {"A": A, "E": E, "info": info.as_dict(), "svp": trace[: info.iters].copy()}
    if want_Y:
        out["Y"] = Y
    return out


def mc(m: int, n: int, row_ptr, col_idx, values, mode: str = "blws", r_cap: int = 256,
       **opts):
    """ALM matrix completion; returns factors (U, S, V) of the completed matrix."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    values = _f64(values)
    o = default_opts(**opts)
    U = np.zeros((m, r_cap))
    V = np.zeros((n, r_cap))
    S = np.zeros(r_cap)
    rank = ctypes.c_int(0)
    info = Info()
    rc = lib().orc_mc(m, n, values.size, _ip(row_ptr), _ip(col_idx), _dp(values),
                      ctypes.byref(o), {"exact": 0, "blws": 1}[mode], r_cap, _dp(U), _dp(S),
                      _dp(V), ctypes.byref(rank), ctypes.byref(info))
    if rc < 0:
        raise RuntimeError(f"orc_mc failed: {rc}")
    r = min(rank.value, r_cap)
    return {"U": U[:, :r], "S": S[:r], "V": V[:, :r], "rank": rank.value,
            "info": info.as_dict()}


def default_svt_mc_opts(**kw) -> SvtMcOpts:
    o = SvtMcOpts()
    lib().orc_default_svt_mc_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def mc_svt(m: int, n: int, row_ptr, col_idx, values, mode: str = "blws", r_cap: int = 256,
           **opts):
    """The SVT algorithm for matrix completion (exact or BLWS thresholding);
    returns factors (U, S, V) of the completed matrix."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    values = _f64(values)
    o = default_svt_mc_opts(**opts)
    U = np.zeros((m, r_cap))
    V = np.zeros((n, r_cap))
    S = np.zeros(r_cap)
    rank = ctypes.c_int(0)
    info = Info()
    rc = lib().orc_mc_svt(m, n, values.size, _ip(row_ptr), _ip(col_idx), _dp(values),
                          ctypes.byref(o), {"exact": 0, "blws": 1}[mode], r_cap, _dp(U), _dp(S),
                          _dp(V), ctypes.byref(rank), ctypes.byref(info))
    if rc < 0:
        raise RuntimeError(f"orc_mc_svt failed: {rc}")
    r = min(rank.value, r_cap)
    return {"U": U[:, :r], "S": S[:r], "V": V[:, :r], "rank": rank.value,
            "info": info.as_dict()}
