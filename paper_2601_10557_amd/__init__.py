"""MI355X (gfx950) pseudo-hermitian ChASE hot path.

Chebyshev-filtered subspace iteration for the nev smallest positive
eigenpairs of ``H = [[A, B], [-conj(B), -conj(A)]]`` (arXiv:2601.10557):
scaled Chebyshev filter on H^2 applied to the positive half of the search
space, CholeskyQR2 with a shifted fallback, oblique Rayleigh-Ritz without an
explicit dual basis, residual locking, an FP32-filter / FP64-refine
precision policy and a hand-written eigenvalue adjoint.  The numerics live
in ``libchase_ph.so`` (HIP for gfx950, C ABI in ``include/chase_ph.h``);
this package only marshals arguments.
"""
from ._lib import FP32, FP64, MIXED  # noqa: F401
from .solver import ChasePHError, PHSolver, TDASolver, colmajor, empty_cm, lib  # noqa: F401
from .autograd import EigvalsPH, eigsh_ph  # noqa: F401
