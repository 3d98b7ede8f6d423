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
    # Theta ~ 0 belongs to a direction where Q^H S Q is singular (Section 4.4):
    # only eigenvalues resolved away from zero, theta > 1e3 u ||G||_F, count
    # as positive (fewer than k/2 of them sends the solver to the back-up).
    pos = theta > 1e3 * np.finfo(float).eps / 2 * np.linalg.norm(G)
    lam_pos = 1.0 / theta[pos]
    Z_pos = Z[:, pos]
    order = np.argsort(lam_pos)
    lam_pos = lam_pos[order]
    Z_pos = Z_pos[:, order]
    if return_all:
        return lam_pos, Z_pos, T, np.sort(1.0 / theta)
    return lam_pos, Z_pos, T


# Threshold below which a diagonal entry of Q^H S Q is replaced in the
# back-up dual basis (Section 5.3 allows replacing zero entries; any nonzero
# value keeps Q_L^H Q = I).  Reading: |d_i| < 1e-8 is taken as zero and
# replaced by 1.
BACKUP_DIAG_MIN = 1e-8


def backup_quotient(Q, T):
    """Non-hermitian back-up Rayleigh quotient of Section 5.3
    (the alternative dual basis named at the end of Section 4.4).

    With ``N = Q^H S Q`` and ``D = diag(N)`` (entries below BACKUP_DIAG_MIN in
    modulus replaced by 1), the dual basis is
    ``Q_L = [S Q - Q (N - D)] D^{-1}`` and the quotient
    ``G = D^{-1} [Q^H S H Q - (N - D) Q^H H Q]`` (``T = H Q`` given).
    Returns ``(G, d)`` with d the diagonal used.
    """
    Q = np.asarray(Q, dtype=np.complex128)
    T = np.asarray(T, dtype=np.complex128)
    N = Q.conj().T @ apply_s(Q)                          # Q^H S Q
    d = np.real(np.diag(N)).copy()
    d[np.abs(d) < BACKUP_DIAG_MIN] = 1.0
    E = N - np.diag(d)                                   # N - D
    P = Q.conj().T @ apply_s(T)                          # Q^H S H Q
    C = Q.conj().T @ T                                   # Q^H H Q
    G = (P - E @ C) / d[:, None]                         # D^{-1} [P - (N - D) C]
    return G, d


def oblique_rr_backup(A, B, Q, return_all: bool = False):
    """Rayleigh-Ritz with the back-up quotient of Section 5.3 (for a Q^H S Q
    that is singular): general eigenproblem ``G y = lambda y``, real parts
    kept.  The back-up dual basis need not be K-symmetric, so the +/- split
    of Thm 4.5 can fail (a replaced zero of diag(Q^H S Q) gives both values
    of an S-neutral pair one sign, and poorly resolved directions give
    unpaired values).  Reading: the positive half is the k/2 eigenvalues with
    the smallest positive real parts, ascending, followed, if fewer than k/2
    are positive, by the largest non-positive ones, descending (the solver
    never locks those).

    Returns ``(lam_pos, Z_pos, T)`` as ``oblique_rr``: real parts, the
    matching eigenvectors of G (Ritz vectors are ``Q Z_pos``) and ``T = H Q``;
    with ``return_all`` also the complex eigenvalues and all eigenvectors.
    """
    Q = np.asarray(Q, dtype=np.complex128)
    T = apply_h(A, B, Q)
    G, _ = backup_quotient(Q, T)
    w, Y = np.linalg.eig(G)
    lam_pos, Z_pos = select_positive_half(w, Y)
    if return_all:
        return lam_pos, Z_pos, T, w, Y
    return lam_pos, Z_pos, T


# Relative size of the smallest diagonal entry of the R factor of Q^H S Q
# (QR with a non-negative real diagonal) below which Q^H S Q counts as
# numerically singular in the general quotient (then the back-up quotient
# runs).
GENERAL_SINGULAR_REL = 1e3 * np.finfo(float).eps / 2


def qsq_singular(N) -> bool:
    """Q^H S Q numerically singular: min |R_ii| <= GENERAL_SINGULAR_REL max |R_ii|
    for N = Q_N R (Householder QR)."""
    r = np.abs(np.diag(np.linalg.qr(N, mode="r")))
    return bool(r.min() <= GENERAL_SINGULAR_REL * r.max())


def select_positive_half(w, Y):
    """The k/2 eigenvalues with the smallest positive real parts, ascending,
    then (if fewer than k/2 are positive) the largest non-positive ones,
    descending; returns (real parts, matching columns of Y)."""
    k = len(w)
    order = np.argsort(w.real, kind="stable")
    p = int(np.sum(w.real <= 0))
    npos = min(k // 2, k - p)
    sel = np.concatenate([order[p:p + npos], order[p - (k // 2 - npos):p][::-1]])
    return w[sel].real, Y[:, sel]


def oblique_rr_general(A, B, Q, return_all: bool = False):
    """Oblique Rayleigh-Ritz with the dual basis of eq. 4.6 for any S H: the
    quotient of eq. 4.7, ``G = (Q^H S Q)^{-1} Q^H S H Q``, solved by a
    general (non-hermitian) dense eigensolver.  Nothing here factors
    Q^H S H Q, so S H need not be definite (Section 5.3, last paragraph:
    a non-hermitian quotient extends the method to an indefinite S H); only
    Q^H S Q must be invertible (``qsq_singular`` is False).  The eigenvalues
    of G are the Ritz values, its eigenvectors the coefficients of the right
    Ritz vectors ``Q z``; real parts are kept and the positive half is
    selected as in ``oblique_rr_backup``.

    Returns ``(lam_pos, Z_pos, T)`` as ``oblique_rr``; with ``return_all``
    also the complex eigenvalues and all eigenvectors of G."""
    Q = np.asarray(Q, dtype=np.complex128)
    T = apply_h(A, B, Q)
    N = Q.conj().T @ apply_s(Q)                          # Q^H S Q
    P = Q.conj().T @ apply_s(T)                          # Q^H S H Q
    G = np.linalg.solve(N, P)                            # eq. 4.7
    w, Y = np.linalg.eig(G)
    lam_pos, Z_pos = select_positive_half(w, Y)
    if return_all:
        return lam_pos, Z_pos, T, w, Y
    return lam_pos, Z_pos, T
