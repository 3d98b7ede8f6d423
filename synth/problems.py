"""Seeded generators for the synthetic pseudo-hermitian test problems.

Draw order from ``numpy.random.default_rng(seed)`` is fixed:
``d`` -> Haar unitary ``Q`` -> coupling Gaussian ``G`` -> raw initial block
(``n x nevex``) -> raw Lanczos starts (``n x lanczos_vecs``) -> loss weights
(``nev``).  Every complex Gaussian has independent N(0, 1) real and
imaginary parts unless stated otherwise.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np
import scipy.linalg
import scipy.sparse.linalg


def complex_normal(rng: np.random.Generator, shape) -> np.ndarray:
    """Complex Gaussian with independent N(0,1) real and imaginary parts."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return re + 1j * im


def _haar_unitary(rng: np.random.Generator, m: int) -> np.ndarray:
    """Haar-distributed unitary (Mezzadri 2007): QR of a Ginibre matrix with
    the phases of diag(R) moved into Q."""
    z = complex_normal(rng, (m, m)) / math.sqrt(2.0)
    q, r = scipy.linalg.qr(z, overwrite_a=True, check_finite=False)
    ph = np.diag(r).copy()
    ph /= np.abs(ph)
    q *= ph[None, :]
    return q


def _spectral_norm(b: np.ndarray) -> float:
    """Largest singular value: dense for small blocks, Lanczos on B^H B
    (ARPACK, deterministic start) otherwise."""
    m = b.shape[0]
    if m <= 1200:
        return float(scipy.linalg.svdvals(b, check_finite=False)[0])
    bh = b.conj().T

    def mv(x):
        return bh @ (b @ x)

    op = scipy.sparse.linalg.LinearOperator((m, m), matvec=mv, dtype=np.complex128)
    v0 = np.ones(m, dtype=np.complex128)
    w = scipy.sparse.linalg.eigsh(op, k=1, which="LA", tol=1e-15, v0=v0,
                                  return_eigenvectors=False, ncv=40)
    return float(math.sqrt(w[0]))


@dataclasses.dataclass
class Problem:
    """One pseudo-hermitian test problem ``H = [[A, B], [-conj(B), -conj(A)]]``.

    ``A`` (Hermitian) and ``B`` (complex symmetric) are ``m x m`` complex128,
    C-contiguous numpy arrays.  ``w0_raw`` is the unscaled Gaussian initial
    block (``n x nevex``), ``lanczos_raw`` the unscaled Lanczos start block,
    ``loss_w`` the N(0,1) weights of a linear eigenvalue loss.
    """
    name: str
    m: int
    A: np.ndarray
    B: np.ndarray
    d: np.ndarray
    coupling: float
    nev: int
    nex: int
    deg: int
    tol: float
    deg_min: int
    deg_max: int
    w0_raw: np.ndarray
    lanczos_raw: np.ndarray
    loss_w: np.ndarray
    seed: int

    @property
    def n(self) -> int:
        return 2 * self.m

    @property
    def nevex(self) -> int:
        return self.nev + self.nex


def _uniform(lo, hi):
    def draw(rng, m):
        return rng.uniform(lo, hi, size=m)
    return draw


def _clustered(rng, m):
    """Exact counts: round(0.8 m) values in U[1, 1.2], the rest in U[1.2, 20],
    then a random permutation."""
    m1 = int(round(0.8 * m))
    d = np.concatenate([rng.uniform(1.0, 1.2, size=m1),
                        rng.uniform(1.2, 20.0, size=m - m1)])
    return d[rng.permutation(m)]


def _bands(bands):
    """Eigenvalues of A from a list of (count fraction, lo, hi) bands: exact
    counts round(fraction m) (the last band takes the rest) drawn uniformly
    in [lo, hi], then a random permutation.  Bands with hi < 0 give A
    negative eigenvalues, so that S H is indefinite."""
    def draw(rng, m):
        parts, used = [], 0
        for i, (frac, lo, hi) in enumerate(bands):
            cnt = m - used if i == len(bands) - 1 else int(round(frac * m))
            parts.append(rng.uniform(lo, hi, size=cnt))
            used += cnt
        d = np.concatenate(parts)
        return d[rng.permutation(m)]
    return draw


# An indefinite S H with a real spectrum: eigenvalues of A in bands of both
# signs, separated by gaps larger than twice ||B||_2 = 0.05 min |d|, so that
# no two eigenvalues of H of opposite S-sign meet and leave the real axis.
# The smallest positive eigenvalues of H come from the negative band
# [-1.3, -1.0] (eigenvectors mostly in the lower half, v^H S v < 0) and the
# positive band [1.5, 2.0] (v^H S v > 0).
INDEFINITE_BANDS = [(0.10, -1.3, -1.0), (0.20, 1.5, 2.0), (0.10, -2.6, -2.2), (0.60, 2.8, 6.0)]


def indefinite_problem(m: int, nev: int, nex: int, deg: int = 20, tol: float = 1e-10, seed: int = 0,
                       coupling: float = 0.05, bands=None) -> "Problem":
    """A pseudo-hermitian problem whose S H is indefinite (A has eigenvalues
    of both signs) but whose eigenvalues are real (see INDEFINITE_BANDS)."""
    return make_problem(m, _bands(bands or INDEFINITE_BANDS), coupling, nev, nex, deg, tol, seed=seed,
                        name=f"indefinite-m{m}")


def make_problem(m: int, d_draw: Callable, coupling: float, nev: int, nex: int,
                 deg: int, tol: float, seed: int = 0, name: str = "custom",
                 deg_min: Optional[int] = None, deg_max: Optional[int] = None,
                 lanczos_vecs: int = 4) -> Problem:
    """Draw one problem.  ``d_draw(rng, m)`` returns the eigenvalues of ``A``;
    ``coupling`` is c in ``||B||_2 = c * min |d|``."""
    rng = np.random.default_rng(seed)
    d = np.asarray(d_draw(rng, m), dtype=np.float64)
    q = _haar_unitary(rng, m)
    a = (q * d[None, :]) @ q.conj().T
    del q
    a = 0.5 * (a + a.conj().T)
    g = complex_normal(rng, (m, m))
    b = 0.5 * (g + g.T)
    del g
    b *= coupling * float(np.abs(d).min()) / _spectral_norm(b)
    b = 0.5 * (b + b.T)
    nevex = nev + nex
    w0 = complex_normal(rng, (2 * m, nevex))
    lz = complex_normal(rng, (2 * m, lanczos_vecs))
    lw = rng.standard_normal(nev)
    return Problem(name=name, m=m, A=np.ascontiguousarray(a), B=np.ascontiguousarray(b),
                   d=d, coupling=coupling, nev=nev, nex=nex, deg=deg, tol=tol,
                   deg_min=deg if deg_min is None else deg_min,
                   deg_max=deg if deg_max is None else deg_max,
                   w0_raw=w0, lanczos_raw=lz, loss_w=lw, seed=seed)


# The five workloads.  m, spectrum of A, coupling c, nev, nex, deg, tol.
CONFIGS = {
    0: dict(name="fp64-baseline-m500", m=500, d_draw=_uniform(1.0, 5.0), coupling=0.4,
            nev=20, nex=10, deg=20, tol=1e-10),
    1: dict(name="mixed-vs-fp64-m4000", m=4000, d_draw=_uniform(0.5, 10.0), coupling=0.3,
            nev=200, nex=60, deg=20, tol=1e-9),
    2: dict(name="clustered-m16000", m=16000, d_draw=_clustered, coupling=0.25,
            nev=1000, nex=200, deg=20, tol=1e-9, deg_min=10, deg_max=36),
    3: dict(name="adjoint-m2000", m=2000, d_draw=_uniform(1.0, 5.0), coupling=0.4,
            nev=50, nex=20, deg=20, tol=1e-12),
    4: dict(name="largest-m30000", m=30000, d_draw=_uniform(0.5, 30.0), coupling=0.3,
            nev=2000, nex=400, deg=20, tol=1e-9),
}


def config_problem(i: int, seed: int = 0, m: Optional[int] = None,
                   nev: Optional[int] = None, nex: Optional[int] = None) -> Problem:
    """Problem of workload ``i``; ``m``/``nev``/``nex`` shrink it for fast tests
    while keeping its spectrum shape and coupling."""
    c = dict(CONFIGS[i])
    name = c.pop("name")
    if m is not None:
        name = f"{name}-scaled-m{m}"
        c["m"] = m
    if nev is not None:
        c["nev"] = nev
    if nex is not None:
        c["nex"] = nex
    return make_problem(seed=seed, name=name, **c)
