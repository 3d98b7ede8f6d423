"""Dense structure-preserving eigensolver: the plain definition of what the
iterative method converges to.

Follows the proof of Thm 3.2 (SH Hermitian positive definite => real
spectrum): with SH = L L^H (Cholesky), H v = lambda v is equivalent to the
Hermitian problem (L^H S L) y = lambda y with y = L^H v.  This is the
reduction of Shao et al. cited in Section 1.1.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .hamiltonian import assemble_h, assemble_sh


def dense_ph_eig(A: np.ndarray, B: np.ndarray):
    """All eigenpairs of H with lambda > 0.

    Returns ``(lam, V)``: ``lam`` ascending (m values), ``V`` (n x m) with
    unit-2-norm columns, ``H V = V diag(lam)``.
    Raises ``numpy.linalg.LinAlgError`` if SH is not positive definite.
    """
    m = A.shape[0]
    sh = assemble_sh(A, B)
    L = np.linalg.cholesky(sh)                       # SH = L L^H
    s = np.concatenate([np.ones(m), -np.ones(m)])
    hh = (L.conj().T * s[None, :]) @ L               # L^H S L (Hermitian)
    hh = 0.5 * (hh + hh.conj().T)
    theta, Y = np.linalg.eigh(hh)
    V = scipy.linalg.solve_triangular(L.conj().T, Y, lower=False)   # v = L^{-H} y
    pos = theta > 0
    lam = theta[pos]
    V = V[:, pos]
    order = np.argsort(lam)
    lam = lam[order]
    V = V[:, order]
    V = V / np.linalg.norm(V, axis=0)[None, :]
    return lam, V


def smallest_positive(A: np.ndarray, B: np.ndarray, nev: int):
    """The nev smallest positive eigenvalues and unit right eigenvectors
    (the solver's output contract, Alg. 3 Input/Output)."""
    lam, V = dense_ph_eig(A, B)
    return lam[:nev], V[:, :nev]


def general_eig(A: np.ndarray, B: np.ndarray):
    """All n eigenpairs of H from the general (non-hermitian) dense
    eigensolver (LAPACK zgeev through numpy), with no use of S H: the
    reference for an indefinite S H (Section 5.3, last paragraph: the
    non-hermitian quotient does not need S H to be definite).  Returns
    ``(w, V)``: complex eigenvalues and unit-2-norm eigenvectors."""
    w, V = np.linalg.eig(assemble_h(A, B))
    V = V / np.linalg.norm(V, axis=0)[None, :]
    return w, V


def smallest_positive_real(A: np.ndarray, B: np.ndarray, nev: int, imag_tol: float = 1e-9):
    """The nev smallest positive real eigenvalues of H (ascending) and unit
    right eigenvectors, for any S H.  Reading (the paper does not treat the
    indefinite case beyond naming it): an eigenvalue counts as real when
    |Im lambda| <= imag_tol * max |lambda|; complex eigenvalues are not
    wanted (their Ritz approximations keep a residual of at least |Im lambda|
    and are never locked).  Returns ``(lam, V, n_complex)`` with n_complex
    the number of eigenvalues of H that are not real."""
    w, V = general_eig(A, B)
    real = np.abs(w.imag) <= imag_tol * np.max(np.abs(w))
    pos = real & (w.real > 0)
    lam = w.real[pos]
    V = V[:, pos]
    order = np.argsort(lam)
    return lam[order][:nev], V[:, order][:, :nev], int(np.sum(~real))
