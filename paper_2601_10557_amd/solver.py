"""Python binding of the C ABI: argument marshalling only.

Matrices cross the boundary column-major.  A column-major ``rows x cols``
block is represented by a torch tensor of shape ``(rows, cols)`` with
strides ``(1, ld)`` (see :func:`colmajor` / :func:`empty_cm`).  The blocks
``A`` (Hermitian) and ``B`` (complex symmetric) are taken as C-contiguous
``(m, m)`` complex128 tensors: read column-major such a buffer holds
``conj(A)`` and ``B``, which the library is told through ``a_conj``.
PyTorch provides device memory and the stream; every numerical step runs in
libchase_ph's kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = _lib.load()
    return _LIB


class ChasePHError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_lib.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def colmajor(t: torch.Tensor) -> torch.Tensor:
    """Column-major (Fortran-order) version of a 2-D tensor."""
    if t.dim() == 1:
        t = t[:, None]
    if t.stride(0) == 1 and t.stride(1) >= max(1, t.shape[0]):
        return t
    return t.t().contiguous().t()


def empty_cm(rows: int, cols: int, dtype=torch.complex128, device="cuda") -> torch.Tensor:
    return torch.empty((cols, rows), dtype=dtype, device=device).t()


def _ld(t: torch.Tensor) -> int:
    assert t.stride(0) == 1, "expected a column-major tensor"
    return max(t.stride(1), t.shape[0]) if t.shape[1] > 1 else max(t.shape[0], t.stride(1), 1)


def _ptr(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def mfma_probe(kind: int, iters: int = 10000) -> float:
    """Measured matrix-core throughput in TFLOP/s (kind 0: FP32
    v_mfma_f32_32x32x2f32, 1: FP64 v_mfma_f64_16x16x4f64) on the current
    device; see chase_ph_mfma_probe."""
    out = C.c_double(0.0)
    st = lib().chase_ph_mfma_probe(int(kind), int(iters), C.byref(out))
    if st != 0:
        raise ChasePHError(_lib.ERR_HIP, f"chase_ph_mfma_probe failed ({st})")
    return out.value


def eigval_backward_noalloc(V: torch.Tensor, g, GA: torch.Tensor, GB: torch.Tensor, stream=None) -> None:
    """Eigenvalue adjoint into caller-allocated ``GA``, ``GB`` (m x m
    column-major complex128) with no handle and no device allocation
    (chase_ph_eigval_backward_noalloc); ``V`` is the 2m x nev block of unit
    right eigenvectors on the current device, ``g`` the nev host weights."""
    V = colmajor(V)
    m, nev = V.shape[0] // 2, V.shape[1]
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64))
    assert g.shape == (nev,) and GA.shape == (m, m) and GB.shape == (m, m)
    assert _ld(GA) == _ld(GB), "GA and GB must share one leading dimension"
    s = (stream or torch.cuda.current_stream(V.device)).cuda_stream
    st = lib().chase_ph_eigval_backward_noalloc(
        m, nev, _ptr(V), _ld(V), g.ctypes.data_as(C.POINTER(C.c_double)), _ptr(GA), _ptr(GB),
        _ld(GA), C.c_void_p(s))
    if st != _lib.OK:
        raise ChasePHError(st, lib().chase_ph_last_error(None).decode())


def default_params() -> _lib.Params:
    p = _lib.Params()
    lib().chase_ph_default_params(C.byref(p))
    return p


@dataclass
class SolveInfo:
    iterations: int
    locked: int
    shifted_qr_used: int
    switch_iter: int
    mu1: float
    mu_nevex0: float
    mu_n: float
    t_lanczos: float
    t_filter: float
    t_qr: float
    t_rr: float
    t_resid: float
    t_total: float
    filter_flops: float
    rr_flops: float
    filter_flops_fp32: float
    resid_history: Optional[np.ndarray] = None
    householder_qr_used: int = 0
    backup_rr_used: int = 0
    general_rr_used: int = 0
    nex_used: int = 0
    rr_sweeps_max: int = 0
    qr_one_pass: int = 0


class PHSolver:
    """Handle over ``H = [[A, B], [-conj(B), -conj(A)]]`` (Section 1, eq. 1.1)."""

    def __init__(self, A: torch.Tensor, B: torch.Tensor, nev: int, nex: int, deg: int = 20,
                 tol: float = 1e-10, max_iter: int = 25, precision: int = _lib.FP64,
                 opt_deg: bool = False, deg_min: int = 8, deg_max: int = 20,
                 switch_tol: float = 0.0, gamma: float = 1e-3, lanczos_steps: int = 26,
                 lanczos_vecs: int = 4, rr_backup: bool = False, definite: bool = True,
                 rr_max_sweeps: int = 40):
        if A.dtype != torch.complex128 or B.dtype != torch.complex128:
            raise TypeError("A and B must be complex128")
        if not A.is_cuda or not B.is_cuda:
            raise ValueError("A and B must be device tensors")
        m = A.shape[0]
        if A.shape != (m, m) or B.shape != (m, m):
            raise ValueError("A and B must be m x m")
        self.A = A.contiguous()
        self.B = B.contiguous()
        self.m, self.n = m, 2 * m
        self.nev, self.nex = nev, nex
        self.nevex = nev + nex
        p = default_params()
        p.m, p.nev, p.nex, p.deg = m, nev, nex, deg
        p.deg_min, p.deg_max, p.opt_deg = deg_min, deg_max, int(opt_deg)
        p.max_iter, p.tol, p.precision = max_iter, tol, precision
        p.switch_tol, p.gamma = switch_tol, gamma
        p.lanczos_steps, p.lanczos_vecs = lanczos_steps, lanczos_vecs
        p.a_conj = 1          # C-contiguous Hermitian A read column-major is conj(A)
        p.rr_backup = int(rr_backup)
        p.definite = int(definite)
        p.rr_max_sweeps = rr_max_sweeps
        self.params = p
        self.device = A.device
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = lib().chase_ph_create(C.byref(p), _ptr(self.A), _ptr(self.B), m,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != _lib.OK:
            raise ChasePHError(st, "chase_ph_create failed")
        self._h = h

    # ------------------------------------------------------------------ util
    def close(self):
        if getattr(self, "_h", None):
            lib().chase_ph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != _lib.OK:
            msg = lib().chase_ph_last_error(self._h)
            raise ChasePHError(st, msg.decode() if msg else "")

    def last_timing(self):
        ms = C.c_double()
        n = C.c_int32()
        lib().chase_ph_last_timing(self._h, C.byref(ms), C.byref(n))
        return ms.value, n.value

    def profile(self, enable: bool = True):
        """Bracket every apply_h launch with HIP events (resets counters)."""
        self._check(lib().chase_ph_profile(self._h, int(enable)))

    def profile_read(self, prec: int):
        """(total_ms, flops, bytes, launches) of the recorded apply_h launches."""
        ms, fl, by, n = C.c_double(), C.c_double(), C.c_double(), C.c_int32()
        self._check(lib().chase_ph_profile_read(self._h, prec, C.byref(ms), C.byref(fl), C.byref(by),
                                                C.byref(n)))
        return ms.value, fl.value, by.value, n.value

    # ---------------------------------------------------------------- stages
    def apply_h(self, X: torch.Tensor, Y: Optional[torch.Tensor] = None, prec: int = _lib.FP64):
        """Y = H X; X is n x k (c128 for FP64, c64 for FP32)."""
        X = colmajor(X)
        k = X.shape[1]
        if Y is None:
            Y = empty_cm(self.n, k, X.dtype, X.device)
        self._check(lib().chase_ph_apply_h(self._h, k, _ptr(X), _ld(X), _ptr(Y), _ld(Y), prec))
        return Y

    def filter(self, W: torch.Tensor, mu1: float, mu_nevex: float, mu_n: float,
               degs: Optional[Sequence[int]] = None, prec: int = _lib.FP64):
        """In place W <- p(H^2) W (eq. 4.1); W column-major n x k."""
        assert W.stride(0) == 1
        k = W.shape[1]
        dp = None
        if degs is not None:
            arr = (C.c_int32 * k)(*[int(x) for x in degs])
            dp = C.cast(arr, C.POINTER(C.c_int32))
        self._check(lib().chase_ph_filter(self._h, k, _ptr(W), _ld(W), dp, mu1, mu_nevex, mu_n, prec))
        return W

    def filter_refined(self, W: torch.Tensor, R: torch.Tensor, lam, mu1: float, mu_nevex: float,
                       mu_n: float, degs: Optional[Sequence[int]] = None):
        """In place W <- p(H^2) W for unit Ritz vectors W with Ritz values lam and
        residuals R = H W - W diag(lam): c64 products, FP64 refinement."""
        assert W.stride(0) == 1
        R = colmajor(R)
        k = W.shape[1]
        lam = np.ascontiguousarray(np.asarray(lam, dtype=np.float64))
        dp = None
        if degs is not None:
            arr = (C.c_int32 * k)(*[int(x) for x in degs])
            dp = C.cast(arr, C.POINTER(C.c_int32))
        self._check(lib().chase_ph_filter_refined(
            self._h, k, _ptr(W), _ld(W), _ptr(R), _ld(R), lam.ctypes.data_as(C.POINTER(C.c_double)), dp,
            mu1, mu_nevex, mu_n))
        return W

    def qr(self, X: torch.Tensor, want_r: bool = True):
        """In place orthonormalisation of X (n x k c128, column-major): CholeskyQR2,
        shifted CholeskyQR3 or Householder QR.  Returns (R, variant) with
        variant 0, 1 or 2 respectively (truthy when a fallback ran)."""
        assert X.stride(0) == 1
        k = X.shape[1]
        R = empty_cm(k, k, torch.complex128, X.device) if want_r else None
        used = C.c_int32(0)
        self._check(lib().chase_ph_qr(self._h, k, _ptr(X), _ld(X), _ptr(R), k if want_r else 0,
                                      C.byref(used)))
        return R, int(used.value)

    def oblique_rr(self, Q: torch.Tensor):
        """Alg. 2 on orthonormal Q (n x k): returns (ritz[k/2], Zpos k x k/2, T = H Q)."""
        Q = colmajor(Q)
        k = Q.shape[1]
        ritz = np.zeros(k // 2)
        Z = empty_cm(k, k // 2, torch.complex128, Q.device)
        T = empty_cm(self.n, k, torch.complex128, Q.device)
        self._check(lib().chase_ph_oblique_rr(
            self._h, k, _ptr(Q), _ld(Q), ritz.ctypes.data_as(C.POINTER(C.c_double)),
            _ptr(Z), _ld(Z), _ptr(T), _ld(T)))
        return ritz, Z, T

    def oblique_rr_backup(self, Q: torch.Tensor):
        """Back-up quotient of Section 5.3 on orthonormal Q (n x k): returns
        (real parts of the k/2 positive Ritz values, Zpos k x k/2, T = H Q)."""
        Q = colmajor(Q)
        k = Q.shape[1]
        ritz = np.zeros(k // 2)
        Z = empty_cm(k, k // 2, torch.complex128, Q.device)
        T = empty_cm(self.n, k, torch.complex128, Q.device)
        self._check(lib().chase_ph_oblique_rr_backup(
            self._h, k, _ptr(Q), _ld(Q), ritz.ctypes.data_as(C.POINTER(C.c_double)),
            _ptr(Z), _ld(Z), _ptr(T), _ld(T)))
        return ritz, Z, T

    def oblique_rr_general(self, Q: torch.Tensor):
        """Quotient of eq. 4.7 by a general eigensolver, for any S H, on
        orthonormal Q (n x k): returns (real parts of the k/2 positive Ritz
        values, Zpos k x k/2, T = H Q)."""
        Q = colmajor(Q)
        k = Q.shape[1]
        ritz = np.zeros(k // 2)
        Z = empty_cm(k, k // 2, torch.complex128, Q.device)
        T = empty_cm(self.n, k, torch.complex128, Q.device)
        self._check(lib().chase_ph_oblique_rr_general(
            self._h, k, _ptr(Q), _ld(Q), ritz.ctypes.data_as(C.POINTER(C.c_double)),
            _ptr(Z), _ld(Z), _ptr(T), _ld(T)))
        return ritz, Z, T

    def residuals(self, Q, T, Zpos, ritz, kk: Optional[int] = None):
        """Half back-transform + residuals (Section 4.5): returns (V n x kk, resid[kk])."""
        Q, T, Zpos = colmajor(Q), colmajor(T), colmajor(Zpos)
        k = Q.shape[1]
        kk = Zpos.shape[1] if kk is None else kk
        ritz = np.ascontiguousarray(ritz[:kk], dtype=np.float64)
        V = empty_cm(self.n, kk, torch.complex128, Q.device)
        res = np.zeros(kk)
        self._check(lib().chase_ph_residuals(
            self._h, k, kk, _ptr(Q), _ld(Q), _ptr(T), _ld(T), _ptr(Zpos), _ld(Zpos),
            ritz.ctypes.data_as(C.POINTER(C.c_double)), _ptr(V), _ld(V),
            res.ctypes.data_as(C.POINTER(C.c_double))))
        return V, res

    def solve(self, W0: torch.Tensor, Lz: torch.Tensor, raise_on_noconv: bool = True):
        """Alg. 3: returns (evals[nev], V n x nev, resid[nev], SolveInfo)."""
        W0, Lz = colmajor(W0), colmajor(Lz)
        ev = np.zeros(self.nev)
        res = np.zeros(self.nev)
        V = empty_cm(self.n, self.nev, torch.complex128, W0.device)
        hist = np.zeros(self.params.max_iter * self.nevex)
        info = _lib.Info()
        info.resid_history = hist.ctypes.data_as(C.POINTER(C.c_double))
        info.resid_history_len = len(hist)
        st = lib().chase_ph_solve(self._h, _ptr(W0), _ld(W0), _ptr(Lz), _ld(Lz),
                                  ev.ctypes.data_as(C.POINTER(C.c_double)), _ptr(V), _ld(V),
                                  res.ctypes.data_as(C.POINTER(C.c_double)), C.byref(info))
        si = SolveInfo(**{f: getattr(info, f) for f, _ in _lib.Info._fields_
                          if f not in ("resid_history", "resid_history_len")})
        si.resid_history = hist
        if st == _lib.ERR_NO_CONVERGENCE and not raise_on_noconv:
            nl = si.locked
            return ev[:nl], V[:, :nl], res[:nl], si
        self._check(st)
        return ev, V, res, si

    def eigval_backward(self, V: torch.Tensor, g):
        """(G_A, G_B) for L = sum g_i lambda_i (adjoint through u = S v)."""
        V = colmajor(V)
        nev = V.shape[1]
        g = np.ascontiguousarray(np.asarray(g, dtype=np.float64))
        GA = empty_cm(self.m, self.m, torch.complex128, V.device)
        GB = empty_cm(self.m, self.m, torch.complex128, V.device)
        self._check(lib().chase_ph_eigval_backward(
            self._h, nev, _ptr(V), _ld(V), g.ctypes.data_as(C.POINTER(C.c_double)),
            _ptr(GA), _ptr(GB), self.m))
        return GA, GB


class TDASolver:
    """Handle for Hermitian ChASE on A alone (Alg. 1; the B = 0 block of
    Section 1.1): the nev smallest eigenvalues of the Hermitian A (m x m)
    and their eigenvectors, on the same H X kernels (operand D = [A, iA])."""

    def __init__(self, A: torch.Tensor, nev: int, nex: int, deg: int = 20, tol: float = 1e-10,
                 max_iter: int = 25, nex_auto: bool = False, lanczos_steps: int = 26,
                 lanczos_vecs: int = 4):
        if A.dtype != torch.complex128:
            raise TypeError("A must be complex128")
        if not A.is_cuda:
            raise ValueError("A must be a device tensor")
        m = A.shape[0]
        if A.shape != (m, m):
            raise ValueError("A must be m x m")
        self.A = A.contiguous()
        self.m = m
        self.nev, self.nex = nev, nex
        p = default_params()
        p.m, p.nev, p.nex, p.deg = m, nev, nex, deg
        p.max_iter, p.tol, p.precision = max_iter, tol, _lib.FP64
        p.lanczos_steps, p.lanczos_vecs = lanczos_steps, lanczos_vecs
        p.a_conj = 1          # C-contiguous Hermitian A read column-major is conj(A)
        p.tda, p.nex_auto = 1, int(nex_auto)
        self.params = p
        self.stream = torch.cuda.current_stream(A.device)
        h = C.c_void_p()
        st = lib().chase_ph_create(C.byref(p), _ptr(self.A), None, m,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != _lib.OK:
            raise ChasePHError(st, "chase_ph_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().chase_ph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != _lib.OK:
            msg = lib().chase_ph_last_error(self._h)
            raise ChasePHError(st, msg.decode() if msg else "")

    def apply_a(self, X: torch.Tensor, Y: Optional[torch.Tensor] = None, prec: int = _lib.FP64):
        """Y = A X; X is m x k (c128 for FP64, c64 for FP32)."""
        X = colmajor(X)
        k = X.shape[1]
        if Y is None:
            Y = empty_cm(self.m, k, X.dtype, X.device)
        self._check(lib().chase_ph_apply_h(self._h, k, _ptr(X), _ld(X), _ptr(Y), _ld(Y), prec))
        return Y

    def solve(self, W0: torch.Tensor, Lz: torch.Tensor, raise_on_noconv: bool = True):
        """Alg. 1: returns (evals[nev], X m x nev, resid[nev], SolveInfo);
        W0 is m x (nev + nex), Lz m x lanczos_vecs."""
        W0, Lz = colmajor(W0), colmajor(Lz)
        ev = np.zeros(self.nev)
        res = np.zeros(self.nev)
        V = empty_cm(self.m, self.nev, torch.complex128, W0.device)
        hist = np.zeros(self.params.max_iter * (self.nev + self.nex))
        info = _lib.Info()
        info.resid_history = hist.ctypes.data_as(C.POINTER(C.c_double))
        info.resid_history_len = len(hist)
        st = lib().chase_ph_solve(self._h, _ptr(W0), _ld(W0), _ptr(Lz), _ld(Lz),
                                  ev.ctypes.data_as(C.POINTER(C.c_double)), _ptr(V), _ld(V),
                                  res.ctypes.data_as(C.POINTER(C.c_double)), C.byref(info))
        si = SolveInfo(**{f: getattr(info, f) for f, _ in _lib.Info._fields_
                          if f not in ("resid_history", "resid_history_len")})
        si.resid_history = hist
        if st == _lib.ERR_NO_CONVERGENCE and not raise_on_noconv:
            nl = si.locked
            return ev[:nl], V[:, :nl], res[:nl], si
        self._check(st)
        return ev, V, res, si
