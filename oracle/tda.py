"""Hermitian ChASE on the resonant block alone (Alg. 1; the TDA case B = 0
of Section 1.1), plain FP64, and the automatic choice of nex.

Alg. 1 computes the nev smallest eigenpairs of the Hermitian A (m x m).
Steps per outer iteration, in Alg. 1's order:
 1. filter W <- p(A) W (eq. 2.1);
 2. orthonormalise [Y, W] (Section 2: Cholesky QR), Y the locked vectors;
 3. keep the non-locked columns;
 4. Rayleigh quotient G = Q^H A Q (the Galerkin condition eq. 2.2);
 5. G Z = Z Omega (Hermitian eigensolver), W = Q Z;
 6. residuals ||A w - omega w|| on unit w;
 7. lock the converged pairs.

Readings (as for the pseudo-hermitian solver): the scalars of eq. 2.1 are
those of the Zhou-Saad scaled Chebyshev recurrence on A over the damped
interval [mu_nevex, mu_m], normalised at mu_1; the spectral estimates come
from Lanczos on A (Section 2): mu_1 the smallest Ritz value, mu_m the
largest plus the residual bound, mu_nevex the Ritz value at which the Gauss
weight accumulated from the left end reaches nevex / m; locking takes the
contiguous prefix of the first nev - locked pairs with residual <= tol.

Automatic nex (named as future work at the end of Section 6.1): from the
same Lanczos density, for each candidate nex the nev-th and (nev+nex)-th
eigenvalues are read off as density quantiles, the filter's convergence
factor of the nev-th pair per outer iteration is 1 / |T_deg(t(omega_nev))|
on the damped interval [omega_nevex, mu_m], and the number of iterations
to shrink a residual of size mu_m - mu_1 to tol follows; the chosen nex
minimises iterations x (nev + nex), the filter work.
"""
from __future__ import annotations

import math

import numpy as np

from .qr import cholqr2


def lanczos_run(A, v0, steps):
    """Hermitian Lanczos on A from v0; returns (alpha, beta)."""
    v = np.asarray(v0, dtype=np.complex128)
    v = v / np.linalg.norm(v)
    v_prev = np.zeros_like(v)
    beta_prev = 0.0
    alpha = np.zeros(steps)
    beta = np.zeros(steps)
    for j in range(steps):
        w = A @ v
        a = float(np.real(np.vdot(v, w)))
        r = w - a * v - beta_prev * v_prev
        b = float(np.linalg.norm(r))
        alpha[j], beta[j] = a, b
        if b == 0.0:
            return alpha[: j + 1], beta[: j + 1]
        v_prev, v, beta_prev = v, r / b, b
    return alpha, beta


def lanczos_density(A, starts, steps):
    """Ritz values and Gauss weights of len(starts[0]) Lanczos runs (weights
    of one run sum to 1 / runs), plus the upper bound mu_m."""
    th_all, w_all = [], []
    mu_m = -np.inf
    runs = starts.shape[1]
    for i in range(runs):
        a, b = lanczos_run(A, starts[:, i], steps)
        T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
        th, Y = np.linalg.eigh(T)
        imax = int(np.argmax(th))
        mu_m = max(mu_m, float(th[imax] + abs(b[-1] * Y[-1, imax])))
        th_all.append(th)
        w_all.append(np.abs(Y[0, :]) ** 2 / runs)
    th = np.concatenate(th_all)
    w = np.concatenate(w_all)
    order = np.argsort(th, kind="stable")
    return th[order], w[order], mu_m


def density_quantile(th, w, frac):
    """Smallest Ritz value at which the weight accumulated from the left end
    reaches frac (of the total)."""
    cum = np.cumsum(w) / np.sum(w)
    idx = min(int(np.searchsorted(cum, frac)), len(th) - 1)
    return float(th[idx])


def spectral_estimates(A, starts, steps, nevex):
    """(mu_1, mu_nevex, mu_m) for Alg. 1."""
    m = A.shape[0]
    th, w, mu_m = lanczos_density(A, starts, steps)
    mu1 = float(th[0])
    mu_nevex = density_quantile(th, w, nevex / m)
    if mu_nevex <= mu1:
        above = th[th > mu1 + 1e-8 * max(1.0, abs(mu1))]
        mu_nevex = float(above[0]) if len(above) else 0.5 * (mu1 + mu_m)
    mu_nevex = min(mu_nevex, mu_m - 0.01 * (mu_m - mu1))
    return mu1, mu_nevex, mu_m


def filter_params(mu1, mu_nevex, mu_m):
    c = 0.5 * (mu_m + mu_nevex)
    e = 0.5 * (mu_m - mu_nevex)
    return c, e, e / (mu1 - c)


def chebyshev_filter(A, W, degs, mu1, mu_nevex, mu_m):
    """W <- p_d(A) W column by column (eq. 2.1 with the Zhou-Saad scalars):
    W_1 = (sigma_1 / e)(A - c) W_0,
    W_{s+1} = (2 sigma_{s+1} / e)(A - c) W_s - sigma_s sigma_{s+1} W_{s-1};
    column j stops at degree degs[j]."""
    c, e, s1 = filter_params(mu1, mu_nevex, mu_m)
    W = np.array(W, dtype=np.complex128, copy=True)
    degs = np.broadcast_to(np.asarray(degs, dtype=int), (W.shape[1],))
    out = np.empty_like(W)
    for j in range(W.shape[1]):
        w0 = W[:, j]
        w1 = (s1 / e) * (A @ w0 - c * w0)
        sig = s1
        for _ in range(1, degs[j]):
            sn = 1.0 / (2.0 / s1 - sig)
            w2 = (2.0 * sn / e) * (A @ w1 - c * w1) - sig * sn * w0
            w0, w1, sig = w1, w2, sn
        out[:, j] = w1 if degs[j] >= 1 else W[:, j]
    return out


def rayleigh_ritz(A, Q):
    """Ritz values (ascending) and vectors of A on range(Q) (Q orthonormal)."""
    G = Q.conj().T @ (A @ Q)
    G = 0.5 * (G + G.conj().T)
    om, Z = np.linalg.eigh(G)
    return om, Q @ Z


def auto_nex(th, w, mu1, mu_m, m, nev, deg, tol, candidates):
    """nex among candidates minimising iterations x (nev + nex) (see the
    module docstring); returns (nex, table of (nex, factor, iterations,
    cost))."""
    best, table = None, []
    for nex in candidates:
        om_nev = density_quantile(th, w, nev / m)
        om_nevex = density_quantile(th, w, (nev + nex) / m)
        if om_nevex <= om_nev or om_nevex >= mu_m:
            table.append((nex, 1.0, math.inf, math.inf))
            continue
        c = 0.5 * (mu_m + om_nevex)
        e = 0.5 * (mu_m - om_nevex)
        t = abs((om_nev - c) / e)
        rho = t + math.sqrt(t * t - 1.0)                 # |T_d(t)| ~ rho^d / 2
        factor = 2.0 / (rho ** deg + rho ** (-deg))      # 1 / |T_deg(t)|
        its = math.ceil(math.log(tol / (mu_m - mu1)) / math.log(factor))
        cost = its * (nev + nex)
        table.append((nex, factor, its, cost))
        if best is None or cost < best[1]:
            best = (nex, cost)
    return (best[0] if best else candidates[-1]), table


def solve(A, nev, nex, deg, tol, w0_raw, lanczos_raw, max_iter=25, lanczos_steps=26):
    """Alg. 1: returns (omega, X, info): the nev smallest eigenvalues of A
    found (ascending), unit eigenvectors (m x nev), info dict."""
    A = np.asarray(A, dtype=np.complex128)
    m = A.shape[0]
    nevex = nev + nex
    W = np.array(w0_raw[:, :nevex], dtype=np.complex128, copy=True)
    mu1, mu_nevex, mu_m = spectral_estimates(A, lanczos_raw, lanczos_steps, nevex)
    Y = np.zeros((m, 0), dtype=np.complex128)
    om_locked = []
    info = dict(mu1=mu1, mu_nevex0=mu_nevex, mu_m=mu_m, iterations=0, locked_history=[], converged=False)
    for it in range(max_iter):
        locked = Y.shape[1]
        W = chebyshev_filter(A, W, deg, mu1, mu_nevex, mu_m)
        Q, _, _ = cholqr2(np.concatenate([Y, W], axis=1))
        Q = Q[:, locked:]
        om, V = rayleigh_ritz(A, Q)
        V = V / np.linalg.norm(V, axis=0)[None, :]
        r = np.linalg.norm(A @ V - V * om[None, :], axis=0)
        nlock = 0
        while nlock < nev - locked and r[nlock] <= tol:
            nlock += 1
        Y = np.concatenate([Y, V[:, :nlock]], axis=1)
        om_locked.extend(om[:nlock].tolist())
        W = V[:, nlock:]
        mu_nevex = min(mu_nevex, float(np.max(om)))
        info["iterations"] = it + 1
        info["locked_history"].append(Y.shape[1])
        if Y.shape[1] >= nev:
            info["converged"] = True
            break
    return np.asarray(om_locked), Y, info
