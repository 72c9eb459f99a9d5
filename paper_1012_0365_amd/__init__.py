"""MI355X-native BLWS singular value thresholding and the nuclear-norm solvers
that host it (Lin & Wei, block Lanczos with warm start).

Python surface over the C ABI of libblws.so: torch tensors supply device memory
and the current HIP stream; every computation runs in the library's kernels.

    import torch, paper_1012_0365_amd as blws
    ctx = blws.Context()
    A, E, info = ctx.rpca_solve(D)                 # robust PCA (inexact ALM + BLWS)
    U, S, V, info = ctx.mc_solve(m, n, row_ptr, col_idx, values)  # matrix completion
    S, rank = ctx.svt(W, eps, U, V, A=A_out)       # one BLWS SVT step, U/V updated in place
"""

from __future__ import annotations

import ctypes

from . import _native
from ._native import (AlmOpts, BlwsError, ServerOpts, ServerStats, SolveInfo, SvtMcOpts,
                      SvtOpts)

__all__ = ["Context", "Server", "BlwsError", "AlmOpts", "SvtOpts", "SvtMcOpts", "SolveInfo",
           "default_alm_opts", "default_mc_opts", "default_svt_mc_opts"]


def _torch():
    import torch  # plumbing only: device memory and streams

    return torch


def _prec_of(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return _native.BLWS_FP64
    if t.dtype == torch.float32:
        return _native.BLWS_FP32
    raise TypeError(f"unsupported dtype {t.dtype}: use float64 or float32")


# start blocks of svt_lanczos and of the svt_start option (Sec. 4.1)
STARTS = _native.STARTS


def _check_mat(t, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D row-major tensor (unit column stride)")
    return t.stride(0)


def default_alm_opts(**kw) -> AlmOpts:
    o = AlmOpts()
    _native.lib().blws_default_alm_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def default_svt_mc_opts(**kw) -> SvtMcOpts:
    o = SvtMcOpts()
    _native.lib().blws_default_svt_mc_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def default_mc_opts(**kw) -> AlmOpts:
    o = AlmOpts()
    _native.lib().blws_default_mc_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Context:
    """One library context on a HIP device (owns the device workspace)."""

    def __init__(self, device: int = 0):
        self._lib = _native.lib()
        h = ctypes.c_void_p()
        _native.check(self._lib.blws_create(ctypes.byref(h), device))
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            self._lib.blws_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return ctypes.c_void_p(_torch().cuda.current_stream(self.device).cuda_stream)

    def _check(self, status):
        return _native.check(status, self.handle)

    # -- the BLWS SVT step ---------------------------------------------------
    def svt(self, W, eps: float, U, V, warm: bool = True, A=None, S=None, seed: int = 20101202,
            pow_steps: int = 2, rank=None, noalloc: bool = False, bf16x3: bool = False):
        """A = T_eps(W) by one BLWS step. U (m x b), V (n x b) are updated in
        place with the top-b Ritz vectors. Returns (S, rank) as device tensors
        (S: float64 [b], rank: int32 [1]; pass them in to reuse buffers).
        noalloc=True calls blws_svt_noalloc (the library's static scratch, no
        device allocation inside the call). bf16x3=True (float32 W) runs the W
        products in split-precision BF16 x 3 (BLWS_BF16X3)."""
        torch = _torch()
        prec = _prec_of(W)
        if bf16x3:
            if prec != _native.BLWS_FP32:
                raise TypeError("BF16 x 3 products take float32 W")
            prec = _native.BLWS_BF16X3
        ldw = _check_mat(W, "W")
        ldu = _check_mat(U, "U")
        ldv = _check_mat(V, "V")
        m, n = W.shape
        b = U.shape[1]
        if U.shape != (m, b) or V.shape != (n, b) or U.dtype != W.dtype or V.dtype != W.dtype:
            raise ValueError("U must be m x b and V n x b, with W's dtype")
        if S is None:
            S = torch.empty(b, dtype=torch.float64, device=W.device)
        if rank is None:
            rank = torch.zeros(1, dtype=torch.int32, device=W.device)
        if S.dtype != torch.float64 or S.numel() < b or rank.dtype != torch.int32:
            raise ValueError("S must be float64 with b entries and rank int32")
        lda = 0
        if A is not None:
            lda = _check_mat(A, "A")
            if A.shape != (m, n) or A.dtype != W.dtype:
                raise ValueError("A must be m x n with W's dtype")
        o = SvtOpts(pow_steps, seed)
        fn = self._lib.blws_svt_noalloc if noalloc else self._lib.blws_svt
        self._check(fn(
            self.handle, self._stream(), prec, m, n, W.data_ptr(), ldw, float(eps), b,
            U.data_ptr(), ldu, V.data_ptr(), ldv, int(bool(warm)), S.data_ptr(),
            rank.data_ptr(), A.data_ptr() if A is not None else None, lda, ctypes.byref(o)))
        return S, rank

    def svt_lanczos(self, W, eps: float, U, V, start: str = "aug", k: int = 2, A=None, S=None,
                    rank=None):
        """One SVT step by the literal block Lanczos on [[0, W], [W^T, 0]]
        (blws_svt_lanczos) from the start block `start` ("split", "aug",
        "left", "right") with k blocks; float64 only. U, V are updated in place
        (sqrt(2) times the halves of the top-b Ritz vectors). Returns (S, rank)."""
        torch = _torch()
        if W.dtype != torch.float64:
            raise TypeError("svt_lanczos takes float64 W")
        ldw = _check_mat(W, "W")
        ldu = _check_mat(U, "U")
        ldv = _check_mat(V, "V")
        m, n = W.shape
        b = U.shape[1]
        if U.shape != (m, b) or V.shape != (n, b) or U.dtype != W.dtype or V.dtype != W.dtype:
            raise ValueError("U must be m x b and V n x b, with W's dtype")
        if S is None:
            S = torch.empty(b, dtype=torch.float64, device=W.device)
        if rank is None:
            rank = torch.zeros(1, dtype=torch.int32, device=W.device)
        lda = 0
        if A is not None:
            lda = _check_mat(A, "A")
            if A.shape != (m, n) or A.dtype != W.dtype:
                raise ValueError("A must be m x n with W's dtype")
        self._check(self._lib.blws_svt_lanczos(
            self.handle, self._stream(), m, n, W.data_ptr(), ldw, float(eps), b,
            _native.STARTS[start], int(k), U.data_ptr(), ldu, V.data_ptr(), ldv, S.data_ptr(),
            rank.data_ptr(), A.data_ptr() if A is not None else None, lda))
        return S, rank

    # -- robust PCA ----------------------------------------------------------
    def rpca_solve(self, D, lam: float | None = None, opts: AlmOpts | None = None, A=None,
                   E=None, bf16: bool = False):
        """min ||A||_* + lam ||E||_1 s.t. D = A + E by inexact ALM with BLWS.
        bf16=True (float32 D only) selects the precision ladder: BF16 W products
        while the residual is large, then FP32, with a final FP32 refinement.
        Returns (A, E, info dict)."""
        torch = _torch()
        prec = _prec_of(D)
        if bf16:
            if prec != _native.BLWS_FP32:
                raise TypeError("the BF16 ladder takes float32 D")
            prec = _native.BLWS_BF16
        ldd = _check_mat(D, "D")
        m, n = D.shape
        if A is None:
            A = torch.empty_like(D)
        if E is None:
            E = torch.empty_like(D)
        lda = _check_mat(A, "A")
        lde = _check_mat(E, "E")
        info = SolveInfo()
        st = self._lib.blws_rpca_solve(
            self.handle, self._stream(), prec, m, n, D.data_ptr(), ldd,
            -1.0 if lam is None else float(lam), ctypes.byref(opts) if opts is not None else None,
            A.data_ptr(), lda, E.data_ptr(), lde, ctypes.byref(info))
        self._check(st)
        return A, E, info.as_dict()

    # -- matrix completion -----------------------------------------------------
    def mc_solve(self, m: int, n: int, row_ptr, col_idx, values, opts: AlmOpts | None = None,
                 r_cap: int = 256):
        """min ||A||_* s.t. A agrees with the samples on Omega (CSR: row_ptr int32[m+1],
        col_idx int32[nnz], values float64/float32[nnz], all device tensors), by
        inexact ALM with BLWS. Returns (U, S, V, info) with A = U diag(S) V^T."""
        return self._mc(self._lib.blws_mc_solve, m, n, row_ptr, col_idx, values, opts, r_cap)

    def mc_svt_solve(self, m: int, n: int, row_ptr, col_idx, values,
                     opts: SvtMcOpts | None = None, r_cap: int = 256):
        """Matrix completion by the SVT algorithm (Y_k = Y_{k-1} + delta P_Omega(M - X_k),
        X_k = T_tau(Y_{k-1}) by BLWS). Arguments and results as mc_solve."""
        return self._mc(self._lib.blws_mc_svt_solve, m, n, row_ptr, col_idx, values, opts, r_cap)

    def _mc(self, fn, m, n, row_ptr, col_idx, values, opts, r_cap):
        torch = _torch()
        prec = _prec_of(values)
        for t, name in ((row_ptr, "row_ptr"), (col_idx, "col_idx"), (values, "values")):
            if not t.is_cuda or t.dim() != 1 or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous 1-D device tensor")
        if row_ptr.dtype != torch.int32 or col_idx.dtype != torch.int32:
            raise TypeError("row_ptr and col_idx must be int32")
        if row_ptr.numel() != m + 1 or col_idx.numel() != values.numel():
            raise ValueError("row_ptr must hold m + 1 entries and col_idx one per value")
        nnz = values.numel()
        U = torch.zeros(m, r_cap, dtype=values.dtype, device=values.device)
        V = torch.zeros(n, r_cap, dtype=values.dtype, device=values.device)
        S = torch.zeros(r_cap, dtype=torch.float64, device=values.device)
        info = SolveInfo()
        st = fn(
            self.handle, self._stream(), prec, m, n, nnz, row_ptr.data_ptr(), col_idx.data_ptr(),
            values.data_ptr(), ctypes.byref(opts) if opts is not None else None, r_cap,
            U.data_ptr(), r_cap, S.data_ptr(), V.data_ptr(), r_cap, ctypes.byref(info))
        self._check(st)
        d = info.as_dict()
        r = min(d["rank"], r_cap)
        return U[:, :r], S[:r], V[:, :r], d

    # -- diagnostics -----------------------------------------------------------
    def fill_uniform(self, X, seed: int, stream_id: int):
        ld = _check_mat(X, "X")
        self._check(self._lib.blws_fill_uniform(self.handle, self._stream(), X.shape[0],
                                                X.shape[1], X.data_ptr(), ld, seed, stream_id))

    def gemm_f64(self, A, B, C, trans_a: bool = False, alpha: float = 1.0, beta: float = 0.0):
        lda, ldb, ldc = _check_mat(A, "A"), _check_mat(B, "B"), _check_mat(C, "C")
        M, N = C.shape
        K = B.shape[0]
        self._check(self._lib.blws_gemm_f64(self.handle, self._stream(), int(trans_a), M, N, K,
                                            alpha, A.data_ptr(), lda, B.data_ptr(), ldb, beta,
                                            C.data_ptr(), ldc))

    def gemm_lp(self, A, B, C, trans_a: bool = False):
        """C = op(A) B on the FP32 (A float32) or BF16 (A int16 holding BF16 bits)
        matrix cores, FP32 accumulation (B, C float32)."""
        torch = _torch()
        lda, ldb, ldc = _check_mat(A, "A"), _check_mat(B, "B"), _check_mat(C, "C")
        bf = A.dtype == torch.int16
        if not bf and A.dtype != torch.float32:
            raise TypeError("A must be float32 or int16 (BF16 bits)")
        M, N = C.shape
        K = B.shape[0]
        self._check(self._lib.blws_gemm_lp(self.handle, self._stream(), int(bf), int(trans_a),
                                           M, N, K, A.data_ptr(), lda, B.data_ptr(), ldb,
                                           C.data_ptr(), ldc))

    def gemm_bf16x3(self, A_hi, A_lo, B, C, trans_a: bool = False):
        """C = op(A) B in split-precision BF16 x 3 (A_hi, A_lo int16 tensors
        holding the BF16 halves of A; B, C float32)."""
        torch = _torch()
        lda, ldb, ldc = _check_mat(A_hi, "A_hi"), _check_mat(B, "B"), _check_mat(C, "C")
        if _check_mat(A_lo, "A_lo") != lda or A_lo.shape != A_hi.shape:
            raise ValueError("A_hi and A_lo must have the same shape and layout")
        if A_hi.dtype != torch.int16 or A_lo.dtype != torch.int16:
            raise TypeError("A_hi and A_lo hold BF16 bits as int16")
        M, N = C.shape
        K = B.shape[0]
        self._check(self._lib.blws_gemm_bf16x3(self.handle, self._stream(), int(trans_a), M, N,
                                               K, A_hi.data_ptr(), A_lo.data_ptr(), lda,
                                               B.data_ptr(), ldb, C.data_ptr(), ldc))

    def small_svd_f64(self, B):
        torch = _torch()
        ldb = _check_mat(B, "B")
        N = B.shape[0]
        UB = torch.empty(N, N, dtype=torch.float64, device=B.device)
        VB = torch.empty_like(UB)
        S = torch.empty(N, dtype=torch.float64, device=B.device)
        self._check(self._lib.blws_small_svd_f64(self.handle, self._stream(), N, B.data_ptr(),
                                                 ldb, UB.data_ptr(), S.data_ptr(), VB.data_ptr()))
        return UB, S, VB

    def cold_block(self, W, b: int, pow_steps: int = 2, seed: int = 20101202,
                   stream_v: int = 1):
        """The cold start block of svt(warm=False): returns (U, V)."""
        torch = _torch()
        ldw = _check_mat(W, "W")
        m, n = W.shape
        U = torch.empty(m, b, dtype=W.dtype, device=W.device)
        V = torch.empty(n, b, dtype=W.dtype, device=W.device)
        self._check(self._lib.blws_cold_block(self.handle, self._stream(), _prec_of(W), m, n,
                                              W.data_ptr(), ldw, b, pow_steps, seed, stream_v,
                                              U.data_ptr(), b, V.data_ptr(), b))
        return U, V

    def timing(self, enable: bool, only=None):
        """Start (clearing the totals) or stop per-kernel timing; `only` names
        the families to record (default: all)."""
        if enable:
            names = ",".join(only) if only else ""
            self._check(self._lib.blws_timing_only(self.handle, names.encode()))
        self._check(self._lib.blws_timing_enable(self.handle, int(enable)))

    def timing_families(self) -> list:
        """Names of the kernel families recorded since timing was enabled."""
        buf = ctypes.create_string_buffer(1 << 16)
        self._check(self._lib.blws_timing_list(self.handle, buf, len(buf)))
        v = buf.value.decode()
        return v.split(",") if v else []

    def timing_get(self, name: str) -> dict:
        n = ctypes.c_longlong()
        ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.blws_timing_get(self.handle, name.encode(), ctypes.byref(n),
                                              ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by)))
        return {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}


class Server:
    """Request server: RPCA and MC solves submitted at any time and run with
    continuous batching (up to max_slots in flight, each on its own stream,
    admitted by workspace footprint against mem_budget bytes; 0 = 80% of free
    device memory). With group_products the dense W-products of the solves
    stepping together go out as grouped launches (a solve waits up to
    group_window_us for others to be ready). Results are those of
    Context.rpca_solve / mc_solve, bit for bit."""

    def __init__(self, device: int = 0, max_slots: int = 4, mem_budget: int = 0,
                 group_products: bool = True, group_window_us: int = 200):
        self._lib = _native.lib()
        o = ServerOpts()
        self._lib.blws_default_server_opts(ctypes.byref(o))
        o.max_slots = max_slots
        o.mem_budget = mem_budget
        o.group_products = 1 if group_products else 0
        o.group_window_us = group_window_us
        h = ctypes.c_void_p()
        st = self._lib.blws_server_create(ctypes.byref(h), device, ctypes.byref(o))
        if st < 0:
            raise BlwsError(st, self._lib.blws_server_last_error(None).decode())
        self.handle = h
        self.device = device
        self._keep = {}  # ticket -> (kind, tensors kept alive until retrieved)

    def _check(self, st):
        if st < 0:
            raise BlwsError(st, self._lib.blws_server_last_error(self.handle).decode())
        return st

    def close(self):
        if getattr(self, "handle", None):
            self._lib.blws_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit_rpca(self, D, lam: float | None = None, opts: AlmOpts | None = None,
                    bf16: bool = False) -> int:
        torch = _torch()
        prec = _prec_of(D)
        if bf16:
            if prec != _native.BLWS_FP32:
                raise TypeError("the BF16 ladder takes float32 D")
            prec = _native.BLWS_BF16
        ldd = _check_mat(D, "D")
        m, n = D.shape
        A = torch.empty(m, n, dtype=D.dtype, device=D.device)
        E = torch.empty(m, n, dtype=D.dtype, device=D.device)
        torch.cuda.current_stream(D.device).synchronize()  # inputs ready before the server reads
        t = ctypes.c_longlong()
        self._check(self._lib.blws_server_submit_rpca(
            self.handle, prec, m, n, D.data_ptr(), ldd, -1.0 if lam is None else float(lam),
            ctypes.byref(opts) if opts is not None else None, A.data_ptr(), n, E.data_ptr(), n,
            ctypes.byref(t)))
        self._keep[t.value] = ("rpca", D, A, E)
        return t.value

    def submit_mc(self, m: int, n: int, row_ptr, col_idx, values, opts: AlmOpts | None = None,
                  r_cap: int = 256) -> int:
        torch = _torch()
        prec = _prec_of(values)
        if row_ptr.dtype != torch.int32 or col_idx.dtype != torch.int32:
            raise TypeError("row_ptr and col_idx must be int32")
        if row_ptr.numel() != m + 1 or col_idx.numel() != values.numel():
            raise ValueError("row_ptr must hold m + 1 entries and col_idx one per value")
        U = torch.zeros(m, r_cap, dtype=values.dtype, device=values.device)
        V = torch.zeros(n, r_cap, dtype=values.dtype, device=values.device)
        S = torch.zeros(r_cap, dtype=torch.float64, device=values.device)
        torch.cuda.current_stream(values.device).synchronize()
        t = ctypes.c_longlong()
        self._check(self._lib.blws_server_submit_mc(
            self.handle, prec, m, n, values.numel(), row_ptr.data_ptr(), col_idx.data_ptr(),
            values.data_ptr(), ctypes.byref(opts) if opts is not None else None, r_cap,
            U.data_ptr(), r_cap, S.data_ptr(), V.data_ptr(), r_cap, ctypes.byref(t)))
        self._keep[t.value] = ("mc", row_ptr, col_idx, values, U, S, V)
        return t.value

    def _result(self, ticket, st, info):
        kept = self._keep.pop(ticket)
        self._check(st)
        d = info.as_dict()
        if kept[0] == "rpca":
            return kept[2], kept[3], d
        U, S, V = kept[4], kept[5], kept[6]
        r = min(d["rank"], U.shape[1])
        return U[:, :r], S[:r], V[:, :r], d

    def poll(self, ticket: int):
        """None while the request runs, else its result (as wait)."""
        done = ctypes.c_int()
        info = SolveInfo()
        st = self._lib.blws_server_poll(self.handle, ticket, ctypes.byref(done),
                                        ctypes.byref(info))
        if st < 0 and not done.value:
            self._check(st)
        if not done.value:
            return None
        return self._result(ticket, st, info)

    def wait(self, ticket: int):
        """(A, E, info) for RPCA, (U, S, V, info) for MC."""
        info = SolveInfo()
        st = self._lib.blws_server_wait(self.handle, ticket, ctypes.byref(info))
        return self._result(ticket, st, info)

    def stats(self) -> dict:
        st = ServerStats()
        self._check(self._lib.blws_server_get_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()
