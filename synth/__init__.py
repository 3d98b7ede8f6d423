"""Seeded synthetic BSE-shaped inputs shared by the oracle and the HIP path.

This module only *draws* inputs: Hermitian resonant blocks ``A``, complex
symmetric coupling blocks ``B`` and the raw Gaussian draws the solver consumes
(initial search block, Lanczos start vectors, loss weights).  It contains none
of the eigensolver's arithmetic: the gamma scaling of the initial block, the
filter, the QR, the Rayleigh-Ritz step and the locking are implemented
separately by ``oracle/`` and by the HIP library.

The paper measures on Yambo Bethe-Salpeter Hamiltonians (Section 6), which
are not available here; these generators stand in for them with the same
structure: ``A = Q diag(d) Q^H`` with ``Q`` Haar-unitary, ``B = B^T`` complex
Gaussian rescaled to ``||B||_2 = c * min |d|`` so that, for positive d,
``SH = [[A, B], [conj(B), conj(A)]]`` is Hermitian positive definite by Weyl's
inequality (the "definite" case of Section 1, eq. (1.3)).
``indefinite_problem`` draws d of both signs: S H is then indefinite.
"""
from .problems import (  # noqa: F401
    CONFIGS,
    Problem,
    make_problem,
    config_problem,
    complex_normal,
    indefinite_problem,
)
