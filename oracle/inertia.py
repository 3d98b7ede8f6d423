"""Eigenvalue count of H in (0, sigma) by Sylvester's law of inertia: a
certificate that no wanted eigenvalue was skipped, usable where a dense
eigensolver is out of reach.

H v = lambda v is S v = lambda^{-1} (S H) v (S^2 = I), and with S H
positive definite (Thm 3.2) the pencil (S, S H) is Hermitian-definite, so
its eigenvalues theta = 1 / lambda are real and, for tau > 0, the number of
them above tau is the number of positive eigenvalues of S - tau S H
(Sylvester's law of inertia for congruent matrices; Parlett, The Symmetric
Eigenvalue Problem, Section 15.2).  With tau = 1 / sigma and a positive
scaling: #{lambda in (0, sigma)} = nu_+(sigma S - S H).

The inertia comes from an LDL^H factorisation with Bunch-Kaufman pivoting
(LAPACK zhetrf through scipy): D is block diagonal with 1 x 1 and 2 x 2
Hermitian blocks and has the inertia of the matrix.  Test infrastructure
only: the library does not use it.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg.lapack as lapack


def shifted_pencil(A: np.ndarray, B: np.ndarray, sigma: float) -> np.ndarray:
    """sigma S - S H = [[sigma I - A, -B], [-conj(B), -sigma I - conj(A)]]
    (column-major, for an in-place factorisation)."""
    m = A.shape[0]
    M = np.empty((2 * m, 2 * m), dtype=np.complex128, order="F")
    M[:m, :m] = -A
    M[:m, m:] = -B
    M[m:, :m] = -np.conj(B)
    M[m:, m:] = -np.conj(A)
    idx = np.arange(m)
    M[idx, idx] += sigma
    M[m + idx, m + idx] -= sigma
    return M


def positive_inertia(M: np.ndarray) -> int:
    """Number of positive eigenvalues of the Hermitian M (lower triangle
    read; M is overwritten when it is complex128 and column-major)."""
    lu, ipiv, info = lapack.zhetrf(M, lower=1, overwrite_a=1)
    if info < 0:
        raise ValueError(f"zhetrf: argument {-info}")
    n = lu.shape[0]
    count = 0
    k = 0
    while k < n:
        if ipiv[k] > 0:                          # 1 x 1 block
            count += int(lu[k, k].real > 0)
            k += 1
        else:                                    # 2 x 2 block in rows k, k + 1
            a, c = lu[k, k].real, lu[k + 1, k + 1].real
            b = lu[k + 1, k]
            ev = np.linalg.eigvalsh(np.array([[a, np.conj(b)], [b, c]]))
            count += int(np.sum(ev > 0))
            k += 2
    return count


def count_below(A: np.ndarray, B: np.ndarray, sigma: float) -> int:
    """#{eigenvalues of H in (0, sigma)} (S H positive definite)."""
    return positive_inertia(shifted_pencil(A, B, sigma))
