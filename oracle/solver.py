"""Pseudo-hermitian ChASE outer loop, plain FP64 (Alg. 3).

Steps per outer iteration, in Alg. 3's order:
 1. filter the positive half, W_+ <- p(H^2) W_+                (Section 4.2)
 2. recover the negative half W_- = K conj(W_+)                (Thm 4.2)
 3. orthonormalise [S Y_+, S Y_-, W_+, W_-], Y_- = K conj(Y_+)  (Section 4.3, eq. 4.5)
 4. drop the 2*locked leading columns                          (Alg. 3)
 5. oblique Rayleigh-Ritz (Alg. 2)                             (Section 4.4)
 6. back-transform and residuals on the positive half only     (Section 4.5)
 7. lock converged pairs; mu_nevex <- largest positive Ritz    (Sections 2, 4.1)

Readings (the paper is silent): a contiguous prefix of the wanted pairs
with residual <= tol and a positive Ritz value is locked each iteration;
mu_1 and mu_n stay at their Lanczos values; mu_nevex follows the largest
non-converged positive Ritz value but never increases (Section 4.1: the
update gradually narrows the filtering interval), i.e.
mu_nevex <- min(mu_nevex, max lambda~); per-vector degrees follow the Chebyshev convergence-factor
bound ``d_j = ceil(ln(r_j / tol) / ln rho_j)`` clamped to [deg_min, deg_max]
with ``rho_j = |t_j| + sqrt(t_j^2 - 1)``, ``t_j = (lambda_j^2 - c) / e``
(Section 6.1 defers the rule to Winkelmann et al. 2019).
"""
from __future__ import annotations

import math

import numpy as np

from .chebyshev import chebyshev_filter, filter_params
from .hamiltonian import apply_k_conj, apply_s
from .lanczos import spectral_estimates, spectral_estimates_indefinite
from .qr import kreal_qr, orthonormalise
from .rayleigh_ritz import oblique_rr, oblique_rr_backup, oblique_rr_general, qsq_singular
from .residuals import back_transform, residual_norms


# Indefinite variant: a Ritz pair whose residual exceeds this fraction of
# |lambda~| is taken as spurious.  Reading (the paper gives no locking rule
# for an indefinite S H): without a definite S H the Ritz values of the
# quotient obey no min-max ordering, and mixtures of eigenvectors of both
# S-signs give real Ritz values anywhere in the spectrum whose residual stays
# of the order of |lambda~|; skipping them keeps one such value from
# blocking the contiguous prefix of converged pairs.
SPURIOUS_REL = 0.1


def init_block(w0_raw: np.ndarray, gamma: float) -> np.ndarray:
    """Alg. 3 first step / Section 4.6: random block with the lower half
    scaled by gamma, keeping it deep in the S-positive manifold."""
    m = w0_raw.shape[0] // 2
    W = np.array(w0_raw, dtype=np.complex128, copy=True)
    W[m:] *= gamma
    return W


def next_degrees(lam, resid, tol, mu1, mu_nevex, mu_n, deg_min, deg_max):
    c, e, _ = filter_params(mu1, mu_nevex, mu_n)
    out = np.empty(len(lam), dtype=int)
    for j, (l, r) in enumerate(zip(lam, resid)):
        t = abs((l * l - c) / e)
        if t <= 1.0 + 1e-12 or r <= tol:
            out[j] = deg_max if r > tol else deg_min
            continue
        rho = t + math.sqrt(t * t - 1.0)
        d = math.ceil(math.log(r / tol) / math.log(rho))
        out[j] = min(max(d, deg_min), deg_max)
    return out


def solve(A, B, nev, nex, deg, tol, w0_raw, lanczos_raw, max_iter=25, gamma=1e-3,
          lanczos_steps=26, deg_min=None, deg_max=None, opt_deg=False, rr_backup=0,
          definite=True):
    """Return ``(lam, V, info)``: the nev smallest positive eigenvalues found
    (ascending), unit right eigenvectors (n x nev) and an info dict.

    rr_backup: 0 uses the back-up quotient of Section 5.3 only when Q^H S Q is
    singular (fewer than k/2 positive eigenvalues of Alg. 2's quotient);
    1 uses it in every iteration.

    definite=False is the indefinite-S H variant (Section 5.3, last
    paragraph): nothing factors S H or Q^H S H Q.  The spectral estimates
    come from Lanczos on S H in the Euclidean inner product
    (lanczos.spectral_estimates_indefinite); every Rayleigh-Ritz step solves
    the quotient of eq. 4.7 with a general eigensolver
    (rayleigh_ritz.oblique_rr_general), or the back-up quotient when
    Q^H S Q is numerically singular or rr_backup is 1; spurious pairs do
    not hold a place in the locking prefix (SPURIOUS_REL).  Filter, QR and
    residuals are unchanged.  Wanted are the nev smallest positive real
    eigenvalues; the locked values are returned sorted."""
    A = np.asarray(A, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    m = A.shape[0]
    n = 2 * m
    nevex = nev + nex
    deg_min = deg if deg_min is None else deg_min
    deg_max = deg if deg_max is None else deg_max
    W = init_block(w0_raw, gamma)
    starts = init_block(lanczos_raw, gamma)
    if definite:
        mu1, mu_nevex, mu_n = spectral_estimates(A, B, starts, lanczos_steps, nevex)
    else:
        mu1, mu_nevex, mu_n = spectral_estimates_indefinite(A, B, starts, lanczos_steps, nevex)
    Yp = np.zeros((n, 0), dtype=np.complex128)
    lam_locked = []
    degs = np.full(nevex, deg, dtype=int)
    info = dict(mu1=mu1, mu_nevex0=mu_nevex, mu_n=mu_n, iterations=0,
                locked_history=[], resid_history=[], shifted_qr=[], backup_rr=[], converged=False)
    for it in range(max_iter):
        locked = Yp.shape[1]
        W = chebyshev_filter(A, B, W, degs, mu1, mu_nevex, mu_n)
        X = np.concatenate([apply_s(Yp), apply_s(apply_k_conj(Yp)), W, apply_k_conj(W)], axis=1)
        Q, _, shifted = orthonormalise(X)
        if shifted == 2:
            # rank-deficient block: K-real basis of the same K-invariant span
            # (the locked pairs' part first), completed by K-real directions
            Q = kreal_qr(np.concatenate([apply_s(Yp), W], axis=1), lead=locked)
        Q = Q[:, 2 * locked:]
        k = Q.shape[1]
        used_backup = bool(rr_backup)
        if not used_backup and definite:
            lam, Z, _ = oblique_rr(A, B, Q)
            used_backup = len(lam) != k // 2
        elif not used_backup:
            used_backup = qsq_singular(Q.conj().T @ apply_s(Q))
            if not used_backup:
                lam, Z, _ = oblique_rr_general(A, B, Q)
        if used_backup:
            lam, Z, _ = oblique_rr_backup(A, B, Q)
        V = back_transform(Q, Z)
        r = residual_norms(A, B, V, lam)
        # candidates for locking, in ascending order of the Ritz value; in the
        # indefinite variant pairs at the spurious level r > SPURIOUS_REL |lambda~|
        # do not hold a place among them
        cand = np.arange(len(lam))
        if not definite:
            cand = cand[r <= SPURIOUS_REL * np.abs(lam)]
        nlock = 0
        while nlock < min(nev - locked, len(cand)) and r[cand[nlock]] <= tol and lam[cand[nlock]] > 0:
            nlock += 1
        sel = cand[:nlock]
        rest = np.setdiff1d(np.arange(len(lam)), sel)
        Yp = np.concatenate([Yp, V[:, sel]], axis=1)
        lam_locked.extend(lam[sel].tolist())
        W = V[:, rest]
        lam_all, r_all = lam, r
        lam, r = lam[rest], r[rest]
        if np.max(lam_all) > 0:
            mu_nevex = min(mu_nevex, float(np.max(lam_all)))
        info["iterations"] = it + 1
        info["locked_history"].append(Yp.shape[1])
        info["resid_history"].append(r_all.copy())
        info["shifted_qr"].append(shifted)
        info["backup_rr"].append(used_backup)
        if Yp.shape[1] >= nev:
            info["converged"] = True
            break
        if opt_deg:
            degs = next_degrees(lam, r, tol, mu1, mu_nevex, mu_n,
                                deg_min, deg_max)
        else:
            degs = np.full(W.shape[1], deg, dtype=int)
    lam_locked = np.asarray(lam_locked)
    order = np.argsort(lam_locked, kind="stable")
    return lam_locked[order], Yp[:, order], info
