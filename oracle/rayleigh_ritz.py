"""Oblique Rayleigh-Ritz without an explicit dual basis (Section 4.4).

The dual basis ``Q_L = S Q (Q^H S Q)^{-1}`` (eq. 4.6) gives the Rayleigh
quotient ``G = (Q^H S Q)^{-1} Q^H S H Q`` (eq. 4.7).  Thm 4.4: with
``Q^H S H Q = L L^H`` it is spectrally equivalent to the Hermitian matrix
``L^H (Q^H S Q)^{-1} L``, eigenvectors ``y = L^H z``.  Alg. 2 avoids the
inverse by diagonalising the inverse quotient
``L^{-1} (Q^H S Q) L^{-H}`` (eigenvalues theta = 1 / lambda~) and
back-transforming.  Steps, in Alg. 2's order:

  T = H Q;  T <- S T;  M = Q^H T;  L = chol(M);  N = I - 2 Q2^H Q2 (= Q^H S Q);
  G = L^{-1} N L^{-H};  G Y = Y Theta;  lambda~ = 1/theta,  Z = L^{-H} Y.

Reading: Alg. 2's last step prints ``L^{-1} Y``; Thm 4.4 (y = L^H z) fixes
the back-transform as ``Z = L^{-H} Y``, which is what is used.
Only the positive half of the Ritz values is returned, ascending (Thm 4.5:
the spectrum is +/- symmetric, Section 4.5: half back-transform).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .hamiltonian import apply_h, apply_s


def oblique_rr(A, B, Q, return_all: bool = False):
    """Ritz values/vectors of H on range(Q) (Q orthonormal, n x k).

    Returns ``(lam_pos, Z_pos, T)``: the k/2 positive Ritz values ascending,
    the matching k x k/2 coefficient block (Ritz vectors are ``Q Z_pos``,
    not normalised), and ``T = H Q``.  With ``return_all`` also returns all
    k Ritz values (for the +/- symmetry check).
    """
    Q = np.asarray(Q, dtype=np.complex128)
    n, k = Q.shape
    m = n // 2
    T = apply_h(A, B, Q)                                 # line 1
    TS = apply_s(T)                                      # line 2
    M = Q.conj().T @ TS                                  # line 3: Q^H S H Q
    M = 0.5 * (M + M.conj().T)
    L = np.linalg.cholesky(M)                            # line 4: M = L L^H
    Q2 = Q[m:]
    N = np.eye(k) - 2.0 * (Q2.conj().T @ Q2)            # line 5: Q^H S Q
    Gt = scipy.linalg.solve_triangular(L, N, lower=True)               # L^{-1} N
    G = scipy.linalg.solve_triangular(L, Gt.conj().T, lower=True)      # L^{-1} (L^{-1} N)^H
    G = 0.5 * (G + G.conj().T)                          # = L^{-1} N L^{-H}  (lines 6-7)
    theta, Y = np.linalg.eigh(G)                         # line 8
    Z = scipy.linalg.solve_triangular(L.conj().T, Y, lower=False)      # line 9: L^{-H} Y
    pos = theta > 0
    lam_pos = 1.0 / theta[pos]
    Z_pos = Z[:, pos]
    order = np.argsort(lam_pos)
    lam_pos = lam_pos[order]
    Z_pos = Z_pos[:, order]
    if return_all:
        return lam_pos, Z_pos, T, np.sort(1.0 / theta)
    return lam_pos, Z_pos, T
