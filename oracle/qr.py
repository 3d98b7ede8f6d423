"""Orthonormalisation of the search block.

Section 2 orthonormalises the filtered block with a (distributed) Cholesky
QR or a Householder QR chosen by condition number.  The oracle implements
CholeskyQR2 (Cholesky QR applied twice) with the shifted CholeskyQR3 of
Fukaya, Kannan, Nakatsukasa, Yamamoto and Yanagisawa (SIAM J. Sci. Comput.
2020) as the fallback when the first Cholesky factorisation breaks down:
shift ``s = 11 (n k + k (k + 1)) u ||X||_2^2`` with ``||X||_2`` bounded by
``||X||_F`` and u the unit roundoff, then CholeskyQR2 on the result.
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
