"""Chebyshev filter p(H^2) W through the scaled three-term recurrence.

Section 4.2, eq. (4.1) states the recurrence
``W_{i+1} = alpha_i H^2 W_i + beta_{i-1} W_{i-1}``, i <= deg, without the
scalars.  Reading taken here (the paper defers to the ChASE/Zhou-Saad
filter): the scaled Chebyshev recurrence of Zhou and Saad (2007) on the
operator H^2, damping the interval [mu_nevex^2, mu_n^2] and normalised at
mu_1^2, so that for an eigenvector v with H v = lambda v

    p(H^2) v = T_d(t(lambda^2)) / T_d(t(mu_1^2)) v,   t(x) = (x - c) / e,
    c = (mu_n^2 + mu_nevex^2) / 2,  e = (mu_n^2 - mu_nevex^2) / 2.

The printed ``W_1 = A W_0`` inside the H^2 recurrence is read as
``W_1 = (sigma_1 / e) (H^2 - c I) W_0``.  ``deg`` counts applications of
H^2 (two products with H each).  Column j stops after its own degree d_j
(per-vector degrees, Section 6.1).
"""
from __future__ import annotations

import numpy as np

from .hamiltonian import apply_h


def filter_params(mu1: float, mu_nevex: float, mu_n: float):
    """(c, e, sigma_1) of the scaled recurrence on H^2."""
    lo, hi, a0 = mu_nevex ** 2, mu_n ** 2, mu1 ** 2
    c = 0.5 * (hi + lo)
    e = 0.5 * (hi - lo)
    sigma1 = e / (a0 - c)
    return c, e, sigma1


def chebyshev_filter(A, B, W, degs, mu1, mu_nevex, mu_n):
    """Return p_{d_j}(H^2) W[:, j] for every column j.

    ``degs`` is an int or a length-k sequence of degrees >= 1.
    """
    W = np.asarray(W, dtype=np.complex128)
    k = W.shape[1]
    degs = np.full(k, int(degs)) if np.isscalar(degs) else np.asarray(degs, dtype=int)
    c, e, sigma1 = filter_params(mu1, mu_nevex, mu_n)
    out = np.empty_like(W)
    for d in np.unique(degs):
        cols = np.nonzero(degs == d)[0]
        X0 = W[:, cols]
        h2x = apply_h(A, B, apply_h(A, B, X0))
        Y = (sigma1 / e) * (h2x - c * X0)             # first degree
        X_prev, sigma = X0, sigma1
        for _ in range(1, int(d)):
            sigma_new = 1.0 / (2.0 / sigma1 - sigma)
            h2y = apply_h(A, B, apply_h(A, B, Y))
            Y_new = (2.0 * sigma_new / e) * (h2y - c * Y) - (sigma * sigma_new) * X_prev
            X_prev, Y, sigma = Y, Y_new, sigma_new
        out[:, cols] = Y
    return out
