"""CPU FP64 oracle for pseudo-hermitian ChASE (Di Napoli, Richefort, Wu,
"Chebyshev Accelerated Subspace Eigensolver for Pseudo-hermitian
Hamiltonians", arXiv:2601.10557).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
product path (the HIP library and its Python binding) never calls into this
package and fails loudly when its own extension is missing.

The oracle is deliberately plain and slow: numpy/scipy in complex128, no
blocking, fusion or reordering beyond what the paper's definitions and
algorithms state, so that each step can be checked against the paper by eye.
It shares no code with the HIP path; the only shared module is ``synth``
(seeded input draws, no method arithmetic).

Modules
-------
hamiltonian   H from its blocks (eq. 1.1), S, K, apply_h by definition
dense         dense structure-preserving eigensolver (proof of Thm 3.2); the
              general eigensolver reference for an indefinite S H
chebyshev     scaled three-term Chebyshev recurrence on H^2 (eq. 4.1)
qr            CholeskyQR2 with a shifted-CholeskyQR3 fallback (Section 2)
rayleigh_ritz oblique Rayleigh-Ritz via the inverse Rayleigh quotient (Alg. 2),
              the back-up quotient and the general quotient of eq. 4.7
residuals     half back-transform and residual norms (Section 4.5)
lanczos       S-inner-product Lanczos spectral estimates (Section 4.1); Euclidean
              Lanczos on S H for an indefinite S H
solver        the pseudo-hermitian ChASE outer loop (Alg. 3)
adjoint       first-order eigenvalue adjoint dL/dA, dL/dB (from Thm 3.2)
tda           Hermitian ChASE on the resonant block (Alg. 1, B = 0) and the
              automatic choice of nex
"""
from . import hamiltonian, dense, chebyshev, qr, rayleigh_ritz, residuals, lanczos, solver, adjoint, tda  # noqa: F401
