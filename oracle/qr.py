"""Orthonormalisation of the search block.

Section 2 orthonormalises the filtered block with a (distributed) Cholesky
QR or a Householder QR chosen by condition number.  The oracle implements
CholeskyQR2 (Cholesky QR applied twice) with the shifted CholeskyQR3 of
Fukaya, Kannan, Nakatsukasa, Yamamoto and Yanagisawa (SIAM J. Sci. Comput.
2020) as the fallback when the first Cholesky factorisation breaks down:
shift ``s = 11 (n k + k (k + 1)) u ||X||_2^2`` with ``||X||_2`` bounded by
``||X||_F`` and u the unit roundoff, then CholeskyQR2 on the result.  When
a factorisation of the shifted variant breaks down too (a numerically
rank-deficient block), ``orthonormalise`` takes the Householder QR of the
block (LAPACK's, through numpy) with the signs of R's real diagonal moved
into Q, so that R's diagonal is non-negative.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

U_ROUNDOFF = 2.0 ** -53


def _chol_upper(G: np.ndarray) -> np.ndarray:
    """Upper Cholesky factor R with G = R^H R; LinAlgError if not HPD."""
    G = 0.5 * (G + G.conj().T)
    return np.linalg.cholesky(G).conj().T


def _cholqr_once(X: np.ndarray, shift: float = 0.0):
    G = X.conj().T @ X
    if shift:
        G = G + shift * np.eye(G.shape[0])
    R = _chol_upper(G)
    Q = scipy.linalg.solve_triangular(R, X.T, trans="T", lower=False).T   # X R^{-1}
    return Q, R


def cholqr2(X: np.ndarray):
    """Return ``(Q, R, shifted)`` with ``X = Q R``, ``Q^H Q = I``, R upper
    triangular with positive real diagonal.  ``shifted`` tells whether the
    shifted first pass was needed.  Raises LinAlgError if even the shifted
    factorisation fails."""
    X = np.asarray(X, dtype=np.complex128)
    n, k = X.shape
    shifted = False
    try:
        Q1, R1 = _cholqr_once(X)
    except np.linalg.LinAlgError:
        shifted = True
        s = 11.0 * (n * k + k * (k + 1)) * U_ROUNDOFF * np.linalg.norm(X, "fro") ** 2
        Q1, R1 = _cholqr_once(X, shift=s)
        Q0, R0 = _cholqr_once(Q1)
        Q1, R1 = Q0, R0 @ R1
    Q2, R2 = _cholqr_once(Q1)
    return Q2, R2 @ R1, shifted


def householder_qr(X: np.ndarray):
    """Householder QR with a real non-negative diagonal of R: ``X = Q R``,
    ``Q^H Q = I`` for any rank (R_jj = 0 where column j depends on the
    previous ones)."""
    X = np.asarray(X, dtype=np.complex128)
    Q, R = np.linalg.qr(X)
    d = np.where(np.real(np.diag(R)) < 0, -1.0, 1.0)
    return Q * d[None, :], R * d[:, None]


def orthonormalise(X: np.ndarray):
    """``(Q, R, variant)``: CholeskyQR2 (variant 0), shifted CholeskyQR3
    (1) or, when a factorisation of both breaks down, Householder QR (2)."""
    try:
        Q, R, shifted = cholqr2(X)
        return Q, R, int(shifted)
    except np.linalg.LinAlgError:
        Q, R = householder_qr(X)
        return Q, R, 2


def kreal_qr(G: np.ndarray, lead: int = 0) -> np.ndarray:
    """Orthonormal basis of span{g_j, J g_j}, J x = K conj(x), made of
    K-real vectors ([a; conj(a)]), for the pair generators G (n x p).

    Each pair is replaced by u = (g + J g) / 2 and v = (g - J g) / (2i),
    which are K-real and span the same space; a K-real vector is described
    by the real coordinates [Re a; Im a], whose real inner products are half
    the complex ones.  The Householder QR of the coordinates [u_1..u_p,
    v_1..v_p] (ordered [u, v] of the first ``lead`` generators, then [u, v]
    of the rest, so that the first 2 lead columns span their pairs) gives an
    orthonormal basis of the K-invariant span for any rank (a dependent
    column is completed by a K-real direction), mapped back to unit K-real
    vectors.  Used by the solver when the search block is numerically rank
    deficient, so that the basis stays K-invariant."""
    G = np.asarray(G, dtype=np.complex128)
    m = G.shape[0] // 2
    g1, g2 = G[:m], G[m:]
    au = 0.5 * (g1 + g2.conj())
    av = (g1 - g2.conj()) / 2j
    A = np.concatenate([au[:, :lead], av[:, :lead], au[:, lead:], av[:, lead:]], axis=1)
    coords = np.concatenate([A.real, A.imag], axis=0)
    Qr, _ = np.linalg.qr(coords)
    a = (Qr[:m] + 1j * Qr[m:]) / np.sqrt(2.0)
    return np.concatenate([a, a.conj()], axis=0)
