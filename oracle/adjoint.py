"""First-order adjoint of the eigenvalues with respect to A and B.

Not in the paper; derived from its Thm 3.2 (left eigenvector u = S v) and
the bi-orthogonality D = V^H S V of eq. (3.5).  For a simple eigenvalue,
``d lambda = u^H dH v / (u^H v)`` (first-order perturbation of a simple
eigenvalue).  With ``v = [x; y]`` and
``S dH = [[dA, dB], [conj(dB), conj(dA)]]`` this gives

    d lambda = (x^H dA x + ybar^H dA ybar + 2 Re(x^H dB y)) / (x^H x - y^H y).

For ``L = sum_i g_i lambda_i`` the gradients in the convention
``grad = dL/dRe + i dL/dIm`` (so ``dL = Re <G, dX>_F``), projected onto
Hermitian dA and symmetric dB, are

    G_A = sum_i gt_i (x_i x_i^H + ybar_i ybar_i^H)
    G_B = sum_i gt_i (x_i y_i^H + ybar_i x_i^T),      gt_i = g_i / (x_i^H x_i - y_i^H y_i).
"""
from __future__ import annotations

import numpy as np


def eigval_grad(V: np.ndarray, g: np.ndarray):
    """(G_A, G_B) for right eigenvectors V (n x nev, any normalisation) and
    loss weights g (nev)."""
    m = V.shape[0] // 2
    G_A = np.zeros((m, m), dtype=np.complex128)
    G_B = np.zeros((m, m), dtype=np.complex128)
    for i in range(V.shape[1]):
        x = V[:m, i]
        y = V[m:, i]
        d = np.real(np.vdot(x, x) - np.vdot(y, y))
        gt = g[i] / d
        yb = y.conj()
        G_A += gt * (np.outer(x, x.conj()) + np.outer(yb, yb.conj()))
        G_B += gt * (np.outer(x, y.conj()) + np.outer(yb, x))
    return G_A, G_B


def eigval_grad_entries(V: np.ndarray, g: np.ndarray, rows, cols):
    """Entries (rows[i], cols[j]) of the (G_A, G_B) of eigval_grad, summed
    pair by pair without forming the m x m matrices (for sizes where they
    do not fit on the host)."""
    m = V.shape[0] // 2
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    GA = np.zeros((len(rows), len(cols)), dtype=np.complex128)
    GB = np.zeros((len(rows), len(cols)), dtype=np.complex128)
    for i in range(V.shape[1]):
        x = V[:m, i]
        y = V[m:, i]
        gt = g[i] / np.real(np.vdot(x, x) - np.vdot(y, y))
        yb = y.conj()
        GA += gt * (np.outer(x[rows], x[cols].conj()) + np.outer(yb[rows], yb[cols].conj()))
        GB += gt * (np.outer(x[rows], y[cols].conj()) + np.outer(yb[rows], x[cols]))
    return GA, GB
