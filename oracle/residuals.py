"""Half back-transform and residuals (Section 4.5; Alg. 3, back-transform
and residual steps).

Ritz vectors ``V = Q Z_+`` are normalised to unit 2-norm and the residual of
pair j is the absolute ``||H v_j - lambda~_j v_j||_2`` (Section 2 defines
residuals on the unit Ritz vectors; reading: absolute, not relative).  The
oracle recomputes ``H V`` from scratch rather than reusing ``H Q``.
"""
from __future__ import annotations

import numpy as np

from .hamiltonian import apply_h


def back_transform(Q, Z_pos):
    V = Q @ Z_pos
    return V / np.linalg.norm(V, axis=0)[None, :]


def residual_norms(A, B, V, lam):
    R = apply_h(A, B, V) - V * np.asarray(lam)[None, :]
    return np.linalg.norm(R, axis=0)
