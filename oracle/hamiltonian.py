"""The pseudo-hermitian Hamiltonian and its structure matrices, written out
from their definitions.

* H = [[A, B], [-conj(B), -conj(A)]], A = A^H, B = B^T   (Section 1, eq. 1.1)
* S = diag(I, -I)                                       (Section 1, eq. 1.2)
* K = [[0, I], [I, 0]]                                   (Thm 3.1)
"""
from __future__ import annotations

import numpy as np


def assemble_h(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Dense n x n H from its m x m blocks (eq. 1.1)."""
    return np.block([[A, B], [-B.conj(), -A.conj()]])


def assemble_sh(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Dense SH = [[A, B], [conj(B), conj(A)]] (eq. 1.3); Hermitian, and
    positive definite in the definite case the paper treats."""
    return np.block([[A, B], [B.conj(), A.conj()]])


def apply_s(X: np.ndarray) -> np.ndarray:
    """S X: flip the sign of the lower half of the rows."""
    m = X.shape[0] // 2
    Y = X.copy()
    Y[m:] *= -1.0
    return Y


def apply_k_conj(X: np.ndarray) -> np.ndarray:
    """K conj(X): swap the two row halves of conj(X) (Thm 3.1, eq. 3.3)."""
    m = X.shape[0] // 2
    Xc = X.conj()
    return np.concatenate([Xc[m:], Xc[:m]], axis=0)


def apply_h(A: np.ndarray, B: np.ndarray, X: np.ndarray) -> np.ndarray:
    """H X by definition: assemble H densely and multiply."""
    return assemble_h(A, B) @ X
