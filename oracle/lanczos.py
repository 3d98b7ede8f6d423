"""Spectral estimates mu_1, mu_nevex, mu_n from a few Lanczos steps
(Section 4.1; Alg. 3, estimation step).

Pins: the recurrence (lanczos_run) is a Gauss rule for the moments
v^H S H H^j v (j < 2 steps), and a full-dimension run reproduces the
spectrum of H.  The estimates (spectral_estimates) are pinned on starts
whose Gauss weights are set through their eigenvector components: a run
that spans the space must return the smallest |lambda|, the largest, and
the positive eigenvalue at the positive-axis weight quantile nevex / m;
on a short run, mu_n must be the largest |Ritz value| plus that Ritz
pair's residual norm, computed by Rayleigh-Ritz on the Krylov space
itself.  The estimates change how many outer iterations the solver needs,
never what it converges to.

Reading taken (the paper defers the variant to Gruning et al. 2011 and only
states that it uses S-inner products, an even step count and the
sign flip after the product): Lanczos in the inner product
``<x, y> = x^H (S H) y``.  H is self-adjoint in it (S H = H^H S) and it is
positive definite in the definite case, so the recurrence cannot break down
for a nonzero start.  Per step one product with H:

    alpha_j = w_j^H S w_j                (w_j = H v_j)
    r       = w_j - alpha_j v_j - beta_j v_{j-1}
    z       = H r,   beta_{j+1} = sqrt(r^H S z)
    v_{j+1} = r / beta_{j+1},   w_{j+1} = z / beta_{j+1}

From the Ritz values theta and weights tau = |first eigenvector entry|^2 of
the tridiagonal T (Section 2, ChASE spectral density):
mu_1 = min |theta|; mu_n = max |theta| plus the Lanczos residual bound of
the extreme Ritz value (Zhou 2011 style upper bound); mu_nevex = the
positive theta at which the accumulated positive-axis weight reaches
nevex / m (Section 4.1: density integrated over the positive axis only).
"""
from __future__ import annotations

import numpy as np

from .hamiltonian import apply_h


def _sdot(x, y):
    """x^H S y."""
    m = x.shape[0] // 2
    return np.vdot(x[:m], y[:m]) - np.vdot(x[m:], y[m:])


def lanczos_run(A, B, v0, steps):
    """One S H - inner-product Lanczos run; returns (alpha, beta) with
    ``len(alpha) == steps`` and ``beta[j]`` the coupling after step j."""
    v = np.asarray(v0, dtype=np.complex128)
    w = apply_h(A, B, v)
    nrm = np.sqrt(np.real(_sdot(v, w)))
    v, w = v / nrm, w / nrm
    v_prev = np.zeros_like(v)
    beta_prev = 0.0
    alpha = np.zeros(steps)
    beta = np.zeros(steps)
    for j in range(steps):
        a = np.real(_sdot(w, w))
        r = w - a * v - beta_prev * v_prev
        z = apply_h(A, B, r)
        b = np.sqrt(max(np.real(_sdot(r, z)), 0.0))
        alpha[j], beta[j] = a, b
        if b == 0.0:
            return alpha[: j + 1], beta[: j + 1]
        v_prev, v, w, beta_prev = v, r / b, z / b, b
    return alpha, beta


def spectral_estimates(A, B, starts, steps, nevex):
    """(mu_1, mu_nevex, mu_n) from len(starts[0]) Lanczos runs."""
    m = A.shape[0]
    thetas, weights = [], []
    mu1 = np.inf
    mu_n = 0.0
    nruns = starts.shape[1]
    for i in range(nruns):
        a, b = lanczos_run(A, B, starts[:, i], steps)
        T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
        th, Y = np.linalg.eigh(T)
        tau = np.abs(Y[0, :]) ** 2
        mu1 = min(mu1, float(np.min(np.abs(th))))
        imax = int(np.argmax(np.abs(th)))
        mu_n = max(mu_n, float(abs(th[imax]) + abs(b[-1] * Y[-1, imax])))
        thetas.append(th)
        weights.append(tau / nruns)
    th = np.concatenate(thetas)
    tau = np.concatenate(weights)
    pos = th > 0
    th, tau = th[pos], tau[pos]
    order = np.argsort(th)
    th, tau = th[order], tau[order]
    cum = np.cumsum(tau) / np.sum(tau)
    idx = int(np.searchsorted(cum, nevex / m))
    idx = min(idx, len(th) - 1)
    mu_nevex = float(th[idx])
    if mu_nevex <= mu1:
        above = th[th > mu1 * (1.0 + 1e-8)]
        mu_nevex = float(above[0]) if len(above) else 0.5 * (mu1 + mu_n)
    mu_nevex = min(mu_nevex, 0.99 * mu_n)
    return mu1, mu_nevex, mu_n


# ---------------------------------------------------------------------------
# Indefinite S H.  The S H inner product above is then not an inner product
# (r^H S H r can be negative) and the recurrence breaks down.  Reading (the
# paper names the indefinite case for the non-hermitian quotient only): the
# estimates come from Lanczos on the Hermitian S H in the Euclidean inner
# product.  Its eigenvalues theta give the singular values |theta| of H
# (H^H H = (S H)^2, S unitary), so that
#   mu_n = max |theta| + residual bound  >=  ||H||_2  >=  |lambda| for every eigenvalue,
#   mu_1 = min |theta|, and
#   mu_nevex = the |theta| at which the Gauss weight accumulated on the folded
#              axis reaches nevex / m (the 2 nevex eigenvalues +-lambda_1..nevex
#              of the n are a fraction nevex / m of the spectrum).
# For B = 0 the |theta| are exactly the |lambda| (S H = diag(A, conj(A)),
# H = diag(A, -conj(A))); with coupling they differ, and only the number of
# outer iterations depends on them.


def lanczos_run_euclid(A, B, v0, steps):
    """Hermitian Lanczos on S H, Euclidean inner product, one product with H
    (and a sign flip of the lower half) per step; returns (alpha, beta)."""
    v = np.asarray(v0, dtype=np.complex128)
    v = v / np.linalg.norm(v)
    v_prev = np.zeros_like(v)
    beta_prev = 0.0
    alpha = np.zeros(steps)
    beta = np.zeros(steps)
    m = v.shape[0] // 2
    for j in range(steps):
        w = apply_h(A, B, v)
        w[m:] *= -1.0                                   # S H v
        a = float(np.real(np.vdot(v, w)))
        r = w - a * v - beta_prev * v_prev
        b = float(np.linalg.norm(r))
        alpha[j], beta[j] = a, b
        if b == 0.0:
            return alpha[: j + 1], beta[: j + 1]
        v_prev, v, beta_prev = v, r / b, b
    return alpha, beta


def spectral_estimates_indefinite(A, B, starts, steps, nevex):
    """(mu_1, mu_nevex, mu_n) for an indefinite S H from len(starts[0])
    Euclidean Lanczos runs on S H (see the reading above)."""
    m = A.shape[0]
    absth, weights = [], []
    mu1 = np.inf
    mu_n = 0.0
    nruns = starts.shape[1]
    for i in range(nruns):
        a, b = lanczos_run_euclid(A, B, starts[:, i], steps)
        T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
        th, Y = np.linalg.eigh(T)
        tau = np.abs(Y[0, :]) ** 2
        mu1 = min(mu1, float(np.min(np.abs(th))))
        imax = int(np.argmax(np.abs(th)))
        mu_n = max(mu_n, float(abs(th[imax]) + abs(b[-1] * Y[-1, imax])))
        absth.append(np.abs(th))
        weights.append(tau / nruns)
    th = np.concatenate(absth)
    tau = np.concatenate(weights)
    order = np.argsort(th)
    th, tau = th[order], tau[order]
    cum = np.cumsum(tau) / np.sum(tau)
    idx = min(int(np.searchsorted(cum, nevex / m)), len(th) - 1)
    mu_nevex = float(th[idx])
    if mu_nevex <= mu1:
        above = th[th > mu1 * (1.0 + 1e-8)]
        mu_nevex = float(above[0]) if len(above) else 0.5 * (mu1 + mu_n)
    mu_nevex = min(mu_nevex, 0.99 * mu_n)
    return mu1, mu_nevex, mu_n
