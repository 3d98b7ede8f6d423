"""Pins of the CPU oracle against facts that do not come from the oracle
itself: a general (non-structured) eigensolver, 50-digit brute force,
closed forms, invariants the paper proves, special cases that reduce to a
textbook problem.  CPU only.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.linalg

from oracle import adjoint, chebyshev, dense, hamiltonian as ham, lanczos, qr, rayleigh_ritz, residuals, solver
from synth import make_problem, config_problem, complex_normal
from cases import decoupled_singular_case


def small_problem(m, seed=0, coupling=0.4, lo=1.0, hi=5.0, nev=4, nex=3, deg=10, tol=1e-10):
    return make_problem(m, lambda rng, mm: rng.uniform(lo, hi, size=mm), coupling,
                        nev, nex, deg, tol, seed=seed)


# ----------------------------------------------------------------- generator
@pytest.mark.parametrize("cfg,m", [(0, 40), (1, 40), (2, 50), (3, 30), (4, 30)])
def test_generator_structure(cfg, m):
    p = config_problem(cfg, m=m)
    assert np.allclose(p.A, p.A.conj().T, atol=0)
    assert np.allclose(p.B, p.B.T, atol=0)
    assert np.allclose(np.sort(np.linalg.eigvalsh(p.A)), np.sort(p.d), atol=1e-12 * p.d.max())
    nb = scipy.linalg.svdvals(p.B)[0]
    assert abs(nb - p.coupling * p.d.min()) <= 1e-12 * nb
    # Weyl: lambda_min(SH) >= (1 - c) min d  (definite case, eq. 1.3)
    lmin = np.linalg.eigvalsh(ham.assemble_sh(p.A, p.B))[0]
    assert lmin >= (1 - p.coupling) * p.d.min() - 1e-12


def test_generator_clustered_counts():
    p = config_problem(2, m=100)
    assert np.sum((p.d >= 1.0) & (p.d <= 1.2)) == 80
    assert np.sum(p.d > 1.2) == 20


def test_generator_large_norm_path():
    # the Lanczos path of ||B||_2 must agree with dense svd
    p = make_problem(1300, lambda rng, m: rng.uniform(1, 2, m), 0.3, 2, 2, 4, 1e-8)
    assert abs(scipy.linalg.svdvals(p.B)[0] - 0.3 * p.d.min()) < 1e-11


# ------------------------------------------------ H structure (eq 1.1-1.3)
def test_pseudo_hermitian_relation():
    p = small_problem(12)
    H = ham.assemble_h(p.A, p.B)
    s = np.concatenate([np.ones(12), -np.ones(12)])
    SH = s[:, None] * H
    assert np.allclose(SH, H.conj().T * s[None, :], atol=1e-14)       # S H = H^H S
    assert np.allclose(SH, ham.assemble_sh(p.A, p.B), atol=0)


def test_apply_h_kconj_symmetry():
    # Thm 3.1 / eq. 3.3: H v = lambda v  <=>  H K conj(v) = -lambda K conj(v)
    p = small_problem(10)
    lam, V = dense.dense_ph_eig(p.A, p.B)
    W = ham.apply_k_conj(V)
    assert np.allclose(ham.apply_h(p.A, p.B, W), -W * lam[None, :], atol=1e-12)


# --------------------------------------------------------- dense oracle
@pytest.mark.parametrize("m,seed", [(4, 0), (8, 1), (16, 2), (32, 3)])
def test_dense_vs_general_eig(m, seed):
    p = small_problem(m, seed=seed)
    lam, V = dense.dense_ph_eig(p.A, p.B)
    w = np.linalg.eigvals(ham.assemble_h(p.A, p.B))
    assert np.max(np.abs(w.imag)) < 1e-10                 # Thm 3.2: real spectrum
    wr = np.sort(w.real)
    assert np.allclose(wr[m:], lam, rtol=1e-11, atol=0)  # positive half
    assert np.allclose(wr[:m], -lam[::-1], rtol=1e-11)    # +/- pairs (Thm 3.1)
    H = ham.assemble_h(p.A, p.B)
    assert np.max(np.abs(H @ V - V * lam[None, :])) < 1e-12 * np.abs(lam).max()
    assert np.allclose(np.linalg.norm(V, axis=0), 1.0)


@pytest.mark.parametrize("m", [4, 8])
def test_dense_vs_mpmath_bruteforce(m):
    p = small_problem(m, seed=7)
    lam, _ = dense.dense_ph_eig(p.A, p.B)
    mpmath.mp.dps = 50
    H = ham.assemble_h(p.A, p.B)
    Hm = mpmath.matrix([[mpmath.mpc(complex(H[i, j])) for j in range(2 * m)] for i in range(2 * m)])
    ev = mpmath.eig(Hm, left=False, right=False)
    ev = sorted(float(mpmath.re(e)) for e in ev)
    assert max(abs(float(mpmath.im(e))) for e in mpmath.eig(Hm, left=False, right=False)) < 1e-30
    assert np.allclose(np.array(ev[m:]), lam, rtol=1e-13, atol=0)


def test_b_zero_reduces_to_tda():
    # Section 1.1: B = 0 gives the Hermitian problem A X = X Omega;
    # spectrum is +/- eig(A), vectors [x; 0].
    p = small_problem(12)
    lam, V = dense.dense_ph_eig(p.A, np.zeros_like(p.B))
    assert np.allclose(lam, np.sort(p.d), rtol=1e-12)
    assert np.max(np.abs(V[12:])) < 1e-12


def test_interval_and_upper_bound():
    # Lemma 3.3 (|lambda| <= rho(A)) and the Shao bound lambda_i <= omega_i(A)
    p = small_problem(20, coupling=0.6)
    lam, _ = dense.dense_ph_eig(p.A, p.B)
    om = np.sort(p.d)
    assert np.all(lam <= om + 1e-12)
    assert lam.max() <= om.max() + 1e-12


def test_bi_orthogonality():
    # eq. 3.5-3.6: D = V^H S V diagonal, D_- = -D_+, V_+^H S V_- = 0
    p = small_problem(10)
    lam, Vp = dense.dense_ph_eig(p.A, p.B)
    Vm = ham.apply_k_conj(Vp)
    V = np.concatenate([Vp, Vm], axis=1)
    D = V.conj().T @ ham.apply_s(V)
    off = D - np.diag(np.diag(D))
    assert np.max(np.abs(off)) < 1e-12
    dp = np.real(np.diag(D)[:10])
    dm = np.real(np.diag(D)[10:])
    assert np.all(dp > 0) and np.allclose(dm, -dp)


def test_condition_numbers_equal():
    # Thm 3.4: cond(SH) = cond(H)
    p = small_problem(10)
    H = ham.assemble_h(p.A, p.B)
    c1 = np.linalg.cond(H)
    c2 = np.linalg.cond(ham.assemble_sh(p.A, p.B))
    assert abs(c1 - c2) < 1e-10 * c1


def test_inertia_count_matches():
    # Hv = lambda v <=> S v = lambda^{-1} (SH) v, a definite pencil, so the
    # positive inertia of sigma S - SH counts the eigenvalues in (0, sigma).
    p = small_problem(16)
    lam, _ = dense.dense_ph_eig(p.A, p.B)
    s = np.concatenate([np.ones(16), -np.ones(16)])
    for sigma in [0.5 * (lam[3] + lam[4]), 0.5 * (lam[9] + lam[10])]:
        M = sigma * np.diag(s) - ham.assemble_sh(p.A, p.B)
        npos = int(np.sum(np.linalg.eigvalsh(M) > 0))
        assert npos == int(np.sum((lam > 0) & (lam < sigma)))


# ------------------------------------------------------- Chebyshev filter
def _cheb_T(d, t):
    """T_d(t) from its trigonometric/hyperbolic closed form."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    a = np.abs(t) <= 1
    out[a] = np.cos(d * np.arccos(t[a]))
    b = t > 1
    out[b] = np.cosh(d * np.arccosh(t[b]))
    c = t < -1
    out[c] = (-1) ** d * np.cosh(d * np.arccosh(-t[c]))
    return out


@pytest.mark.parametrize("deg", [1, 2, 5, 12])
def test_filter_closed_form_on_eigenvectors(deg):
    p = small_problem(20)
    lam, Vp = dense.dense_ph_eig(p.A, p.B)
    mu1, mu_nevex, mu_n = 0.9 * lam[0], lam[6], 1.05 * lam[-1]
    V = np.concatenate([Vp[:, :8], ham.apply_k_conj(Vp[:, :3]), Vp[:, -2:]], axis=1)
    lv = np.concatenate([lam[:8], -lam[:3], lam[-2:]])
    c = 0.5 * (mu_n ** 2 + mu_nevex ** 2)
    e = 0.5 * (mu_n ** 2 - mu_nevex ** 2)
    ratio = _cheb_T(deg, (lv ** 2 - c) / e) / _cheb_T(deg, np.array([(mu1 ** 2 - c) / e]))[0]
    out = chebyshev.chebyshev_filter(p.A, p.B, V, deg, mu1, mu_nevex, mu_n)
    expect = V * ratio[None, :]
    scale = np.maximum(np.abs(ratio), 1.0)
    assert np.max(np.abs(out - expect) / scale[None, :]) < 1e-10


def test_filter_per_column_degrees_closed_form():
    p = small_problem(16)
    lam, Vp = dense.dense_ph_eig(p.A, p.B)
    mu1, mu_nevex, mu_n = lam[0], lam[5], lam[-1]
    degs = np.array([3, 3, 7, 10, 1, 7])
    V = Vp[:, :6]
    out = chebyshev.chebyshev_filter(p.A, p.B, V, degs, mu1, mu_nevex, mu_n)
    c = 0.5 * (mu_n ** 2 + mu_nevex ** 2)
    e = 0.5 * (mu_n ** 2 - mu_nevex ** 2)
    for j in range(6):
        r = _cheb_T(degs[j], np.array([(lam[j] ** 2 - c) / e]))[0] / \
            _cheb_T(degs[j], np.array([(mu1 ** 2 - c) / e]))[0]
        assert np.allclose(out[:, j], r * V[:, j], rtol=0, atol=1e-10 * max(1, abs(r)))


def test_filter_kconj_equivariance():
    # Thm 4.2: p(H^2) K conj(W) = K conj(p(H^2) W)
    p = small_problem(14)
    rng = np.random.default_rng(3)
    W = complex_normal(rng, (28, 5))
    f = lambda X: chebyshev.chebyshev_filter(p.A, p.B, X, 6, 1.0, 2.0, 5.5)
    a = f(ham.apply_k_conj(W))
    b = ham.apply_k_conj(f(W))
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))


# ------------------------------------------------------------------ QR
def _phase_normalised_qr(X):
    Qn, Rn = np.linalg.qr(X)
    ph = np.diag(Rn) / np.abs(np.diag(Rn))
    return Qn * ph[None, :], Rn * ph.conj()[:, None]


def test_cholqr2_matches_householder():
    rng = np.random.default_rng(0)
    X = complex_normal(rng, (200, 30))
    Q, R, shifted = qr.cholqr2(X)
    assert not shifted
    Qr, Rr = _phase_normalised_qr(X)
    assert np.allclose(Q, Qr, atol=1e-12)
    assert np.allclose(R, Rr, atol=1e-11)
    assert np.allclose(np.diag(R).imag, 0) and np.all(np.diag(R).real > 0)
    assert np.allclose(np.triu(R), R)


def test_cholqr_shifted_fallback_ill_conditioned():
    rng = np.random.default_rng(1)
    n, k = 300, 20
    U, _ = np.linalg.qr(complex_normal(rng, (n, k)))
    Vh, _ = np.linalg.qr(complex_normal(rng, (k, k)))
    s = np.logspace(0, -13, k)
    X = (U * s[None, :]) @ Vh.conj().T
    Q, R, shifted = qr.cholqr2(X)
    assert shifted
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(k))) < 1e-12
    assert np.max(np.abs(Q @ R - X)) < 1e-13 * np.linalg.norm(X, 2) * 10


# -------------------------------------------------------- oblique RR
def _search_basis(p, k_half, seed=0, gamma=1e-3):
    rng = np.random.default_rng(seed)
    W = solver.init_block(complex_normal(rng, (2 * p.m, k_half)), gamma)
    W = chebyshev.chebyshev_filter(p.A, p.B, W, 4, 0.8, 2.0, 5.5)
    X = np.concatenate([W, ham.apply_k_conj(W)], axis=1)
    Q, _, _ = qr.cholqr2(X)
    return Q


def test_rr_matches_explicit_nonhermitian_quotient():
    p = small_problem(30)
    Q = _search_basis(p, 6)
    lam, Z, T = rayleigh_ritz.oblique_rr(p.A, p.B, Q)
    QSQ = Q.conj().T @ ham.apply_s(Q)
    QSHQ = Q.conj().T @ ham.apply_s(ham.apply_h(p.A, p.B, Q))
    G = np.linalg.solve(QSQ, QSHQ)                        # eq. 4.7
    w, Zg = np.linalg.eig(G)
    assert np.max(np.abs(w.imag)) < 1e-9
    wp = np.sort(w.real[w.real > 0])
    assert np.allclose(lam, wp, rtol=1e-10)
    assert np.allclose(G @ Z, Z * lam[None, :], atol=1e-9 * np.abs(Z).max())
    assert np.allclose(T, ham.apply_h(p.A, p.B, Q))


def test_rr_plus_minus_symmetry():
    # Thm 4.5: Ritz values +/- symmetric; Q Z_- = K conj(Q Z_+)
    p = small_problem(30)
    Q = _search_basis(p, 5, seed=2)
    lam, Z, _, allv = rayleigh_ritz.oblique_rr(p.A, p.B, Q, return_all=True)
    assert np.allclose(np.sort(allv), np.sort(-allv), rtol=1e-10)
    QSQ = Q.conj().T @ ham.apply_s(Q)
    QSHQ = Q.conj().T @ ham.apply_s(ham.apply_h(p.A, p.B, Q))
    w, Zg = np.linalg.eig(np.linalg.solve(QSQ, QSHQ))
    for j in range(len(lam)):
        i = int(np.argmin(np.abs(w - (-lam[j]))))
        vm = Q @ Zg[:, i]
        vp = ham.apply_k_conj(Q @ Z[:, j])
        # equal up to a complex scalar
        c = np.vdot(vp, vm) / np.vdot(vp, vp)
        assert np.linalg.norm(vm - c * vp) < 1e-8 * np.linalg.norm(vm)


def test_rr_exact_invariant_subspace():
    p = small_problem(24)
    lam, Vp = dense.dense_ph_eig(p.A, p.B)
    X = np.concatenate([Vp[:, :5], ham.apply_k_conj(Vp[:, :5])], axis=1)
    Q, _, _ = qr.cholqr2(X)
    lr, Z, _ = rayleigh_ritz.oblique_rr(p.A, p.B, Q)
    assert np.allclose(lr, lam[:5], rtol=1e-12)
    V = residuals.back_transform(Q, Z)
    assert np.max(residuals.residual_norms(p.A, p.B, V, lr)) < 1e-12


def test_rr_quadratic_convergence():
    # Lemma 5.5: |lambda - lambda~| = O(sigma_v^2)
    p = small_problem(30)
    lam, Vp = dense.dense_ph_eig(p.A, p.B)
    rng = np.random.default_rng(5)
    E = complex_normal(rng, (60, 4))
    errs = []
    epss = [1e-2, 1e-3, 1e-4]
    for eps in epss:
        Wp = Vp[:, :4] + eps * E
        X = np.concatenate([Wp, ham.apply_k_conj(Wp)], axis=1)
        Q, _, _ = qr.cholqr2(X)
        lr, _, _ = rayleigh_ritz.oblique_rr(p.A, p.B, Q)
        errs.append(np.max(np.abs(lr - lam[:4])))
    slopes = np.diff(np.log10(errs)) / np.diff(np.log10(epss))
    assert np.all(slopes > 1.8), slopes


def test_rr_ritz_values_in_field_of_values_interval():
    # Thm 5.6
    p = small_problem(30)
    Q = _search_basis(p, 6, seed=4)
    _, _, _, allv = rayleigh_ritz.oblique_rr(p.A, p.B, Q, return_all=True)
    QSQ = Q.conj().T @ ham.apply_s(Q)
    lmin = np.min(np.abs(np.linalg.eigvalsh(0.5 * (QSQ + QSQ.conj().T))))
    rho = np.max(np.abs(np.linalg.eigvalsh(ham.assemble_sh(p.A, p.B))))
    assert np.all(np.abs(allv) <= rho / lmin * (1 + 1e-12))
    assert lmin <= 1.0 + 1e-12


def _backup_dual_basis(Q):
    # Q_L = [S Q - Q (Q^H S Q - D)] D^{-1}, D = diag(Q^H S Q) (Sections 4.4, 5.3),
    # written from the dual-basis equation, not from the quotient
    N = Q.conj().T @ ham.apply_s(Q)
    d = np.real(np.diag(N)).copy()
    d[np.abs(d) < rayleigh_ritz.BACKUP_DIAG_MIN] = 1.0
    return (ham.apply_s(Q) - Q @ (N - np.diag(d))) / d[None, :]


def test_backup_quotient_is_dual_projection():
    # the quotient equation of Section 5.3 equals Q_L^H H Q for the dual basis
    # equation, and Q_L^H Q = I
    p = small_problem(30)
    Q = _search_basis(p, 6, seed=7)
    H = ham.assemble_h(p.A, p.B)
    G, _ = rayleigh_ritz.backup_quotient(Q, H @ Q)
    QL = _backup_dual_basis(Q)
    assert np.abs(QL.conj().T @ Q - np.eye(12)).max() < 1e-12
    assert np.abs(G - QL.conj().T @ H @ Q).max() < 1e-12 * np.abs(G).max()


def test_backup_petrov_galerkin_residuals():
    # every eigenpair of the back-up quotient leaves a residual orthogonal to
    # range(Q_L) (the oblique projection condition), complex values included
    p = small_problem(30)
    Q = _search_basis(p, 5, seed=8)
    _, _, T, w, Y = rayleigh_ritz.oblique_rr_backup(p.A, p.B, Q, return_all=True)
    QL = _backup_dual_basis(Q)
    R = T @ Y - (Q @ Y) * w[None, :]
    assert np.abs(QL.conj().T @ R).max() < 1e-11 * np.abs(T).max()
    # a filtered basis: real parts split +/- and the positive half lies
    # near the Alg. 2 values
    lam_rr, _, _ = rayleigh_ritz.oblique_rr(p.A, p.B, Q)
    lam_bk, _, _ = rayleigh_ritz.oblique_rr_backup(p.A, p.B, Q)
    assert np.all(lam_bk > 0) and np.sum(w.real < 0) == 5
    assert np.allclose(lam_bk, lam_rr, rtol=1e-2)


def test_backup_exact_invariant_subspace():
    p = small_problem(24)
    lam, Vp = dense.dense_ph_eig(p.A, p.B)
    X = np.concatenate([Vp[:, :5], ham.apply_k_conj(Vp[:, :5])], axis=1)
    Q, _, _ = qr.cholqr2(X)
    lr, Z, _, w, _ = rayleigh_ritz.oblique_rr_backup(p.A, p.B, Q, return_all=True)
    assert np.allclose(lr, lam[:5], rtol=1e-11)
    assert np.max(np.abs(w.imag)) < 1e-11 * np.max(np.abs(w))
    V = residuals.back_transform(Q, Z)
    assert np.max(residuals.residual_norms(p.A, p.B, V, lr)) < 1e-11


def test_backup_recovers_pairs_when_qsq_singular():
    # range(Q) = an exact +/- eigenpair of the trailing block plus the two
    # S-neutral, mutually S-orthogonal vectors [e0; e1], [e1; e0]: Q^H S Q has
    # a 2 x 2 zero block, Alg. 2 resolves one positive value only, the
    # back-up quotient (zero diagonal entries replaced) gives both, and the
    # exact pair among them
    A, B, Q, lam_exact = decoupled_singular_case()
    N = Q.conj().T @ ham.apply_s(Q)
    assert np.linalg.matrix_rank(N, tol=1e-10) == 2
    lam_rr, _, _ = rayleigh_ritz.oblique_rr(A, B, Q)
    assert len(lam_rr) == 1
    lam_bk, Z, _ = rayleigh_ritz.oblique_rr_backup(A, B, Q)
    assert len(lam_bk) == 2
    i = int(np.argmin(np.abs(lam_bk - lam_exact)))
    assert abs(lam_bk[i] - lam_exact) < 1e-12 * lam_exact
    Vb = residuals.back_transform(Q, Z[:, i:i + 1])
    assert residuals.residual_norms(A, B, Vb, lam_bk[i:i + 1])[0] < 1e-12


# ------------------------------------------------------------- solver
def test_init_block_is_s_positive():
    # Section 4.6: the start block must lie in the S-positive manifold; the
    # lower half of the Gaussian block is scaled by gamma (Alg. 3, first
    # step), so the coupling ratio ||y|| / ||x|| of every column is gamma
    # times the raw one and W^H S W is positive definite, while the raw
    # block is S-indefinite
    rng = np.random.default_rng(2)
    m, k, gamma = 50, 12, 1e-3
    raw = complex_normal(rng, (2 * m, k))
    W = solver.init_block(raw, gamma)
    assert np.array_equal(W[:m], raw[:m])
    ratio = np.linalg.norm(W[m:], axis=0) / np.linalg.norm(W[:m], axis=0)
    raw_ratio = np.linalg.norm(raw[m:], axis=0) / np.linalg.norm(raw[:m], axis=0)
    assert np.allclose(ratio, gamma * raw_ratio, rtol=1e-14)
    assert np.linalg.eigvalsh(W.conj().T @ ham.apply_s(W))[0] > 0
    ev_raw = np.linalg.eigvalsh(raw.conj().T @ ham.apply_s(raw))
    assert ev_raw[0] < 0 < ev_raw[-1]


def test_back_transform_unit_columns():
    # Section 4.5 / Alg. 3: the back-transformed Ritz vectors Q Z_+ are the
    # eigenvector estimates whose residuals are measured, on unit vectors
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(complex_normal(rng, (40, 10)))
    Z = 3.0 * complex_normal(rng, (10, 5))
    V = residuals.back_transform(Q, Z)
    assert np.allclose(np.linalg.norm(V, axis=0), 1.0, rtol=0, atol=1e-14)
    QZ = Q @ Z
    cos = np.abs(np.einsum("ij,ij->j", V.conj(), QZ)) / np.linalg.norm(QZ, axis=0)
    assert np.allclose(cos, 1.0, rtol=0, atol=1e-14)


def test_solver_matches_dense():
    p = small_problem(60, nev=6, nex=4, deg=10, tol=1e-10)
    lam, V, info = solver.solve(p.A, p.B, p.nev, p.nex, p.deg, p.tol, p.w0_raw, p.lanczos_raw)
    ref, _ = dense.smallest_positive(p.A, p.B, p.nev)
    assert info["converged"]
    assert np.allclose(lam, ref, rtol=1e-10, atol=0)
    r = residuals.residual_norms(p.A, p.B, V, lam)
    assert np.all(r <= p.tol)
    D = V.conj().T @ ham.apply_s(V)                    # S-orthogonality (eq. 3.5)
    assert np.max(np.abs(D - np.diag(np.diag(D)))) < 1e-9
    assert np.all(np.real(np.diag(D)) > 0)


def test_solver_zero_start_column_uses_kreal_qr():
    # a zero start column keeps the first search block rank deficient; the
    # K-real Householder basis keeps the span K-invariant and the iteration
    # still reaches the dense eigenvalues
    p = small_problem(60, nev=6, nex=4, deg=10, tol=1e-10)
    w0 = np.array(p.w0_raw, copy=True)
    w0[:, 2] = 0
    lam, V, info = solver.solve(p.A, p.B, p.nev, p.nex, p.deg, p.tol, w0, p.lanczos_raw)
    assert info["shifted_qr"][0] == 2
    ref, _ = dense.smallest_positive(p.A, p.B, p.nev)
    assert info["converged"]
    assert np.allclose(lam, ref, rtol=1e-10, atol=0)


def test_solver_b_zero_case():
    p = small_problem(50, nev=5, nex=4, deg=10, tol=1e-10)
    lam, V, info = solver.solve(p.A, np.zeros_like(p.B), p.nev, p.nex, p.deg, p.tol,
                                p.w0_raw, p.lanczos_raw)
    assert np.allclose(lam, np.sort(p.d)[:5], rtol=1e-10)
    assert np.max(np.abs(V[50:])) < 1e-8


def test_solver_per_vector_degrees():
    p = small_problem(60, nev=6, nex=4, deg=12, tol=1e-10)
    lam, V, info = solver.solve(p.A, p.B, p.nev, p.nex, p.deg, p.tol, p.w0_raw,
                                p.lanczos_raw, deg_min=4, deg_max=16, opt_deg=True)
    ref, _ = dense.smallest_positive(p.A, p.B, p.nev)
    assert np.allclose(lam, ref, rtol=1e-10)


def test_solver_backup_rr_every_iteration():
    # the back-up quotient of Section 5.3 in every iteration still converges to
    # the dense eigenvalues (no quadratic convergence, so more iterations)
    p = small_problem(40, nev=4, nex=4)
    rng = np.random.default_rng(0)
    lam, V, info = solver.solve(p.A, p.B, p.nev, p.nex, 12, 1e-9, complex_normal(rng, (80, 8)),
                                complex_normal(rng, (80, 4)), max_iter=40, rr_backup=1)
    assert info["converged"] and all(info["backup_rr"])
    exact, _ = dense.smallest_positive(p.A, p.B, p.nev)
    assert np.allclose(lam, exact, rtol=1e-9)


def test_solver_max_iter_partial():
    p = small_problem(60, nev=6, nex=4, deg=2, tol=1e-14)
    lam, V, info = solver.solve(p.A, p.B, p.nev, p.nex, p.deg, p.tol, p.w0_raw,
                                p.lanczos_raw, max_iter=1)
    assert not info["converged"] and info["iterations"] == 1


@pytest.mark.parametrize("steps", [3, 5, 6])
def test_lanczos_gauss_quadrature_moments(steps):
    # s steps of Lanczos in the S H inner product form a Gauss rule: the
    # nodes theta (eigenvalues of T) and weights tau (squared first
    # components of its eigenvectors) reproduce the moments
    # v^H S H H^j v / v^H S H v for j < 2 s, and miss the one at j = 2 s
    p = small_problem(6, seed=1)
    H = ham.assemble_h(p.A, p.B)
    SH = ham.assemble_sh(p.A, p.B)
    v = complex_normal(np.random.default_rng(3), (12,))
    a, b = lanczos.lanczos_run(p.A, p.B, v, steps)
    T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    th, Y = np.linalg.eigh(T)
    tau = np.abs(Y[0]) ** 2
    nrm = np.real(np.vdot(v, SH @ v))
    mom = [np.real(np.vdot(v, SH @ np.linalg.matrix_power(H, j) @ v)) / nrm for j in range(2 * steps + 1)]
    for j in range(2 * steps):
        assert abs(np.sum(tau * th ** j) - mom[j]) <= 1e-11 * max(1.0, abs(mom[j]))
    assert abs(np.sum(tau * th ** (2 * steps)) - mom[2 * steps]) > 1e-8 * abs(mom[2 * steps])


def test_lanczos_full_dimension_reproduces_spectrum():
    # n steps span the whole space: the eigenvalues of T are those of H
    p = small_problem(6, seed=1)
    v = complex_normal(np.random.default_rng(4), (12,))
    a, b = lanczos.lanczos_run(p.A, p.B, v, 12)
    T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    lam = np.sort(np.linalg.eigvals(ham.assemble_h(p.A, p.B)).real)
    assert np.allclose(np.sort(np.linalg.eigvalsh(T)), lam, rtol=1e-10, atol=0)


def test_next_degrees_is_the_smallest_sufficient_degree():
    # per-vector degrees: the smallest d in [deg_min, deg_max] with
    # r rho^-d <= tol, rho the growth rate of T_d at t = (lambda^2 - c) / e,
    # taken here from the Chebyshev recurrence itself (T_{d+1} / T_d at
    # d = 60) on the interval [mu_nevex^2, mu_n^2] of the filter on H^2
    mu1, mu_nevex, mu_n = 1.0, 1.6, 5.0
    c = 0.5 * (mu_n ** 2 + mu_nevex ** 2)
    e = 0.5 * (mu_n ** 2 - mu_nevex ** 2)

    def rho_of(lam):
        t = abs(lam * lam - c) / e
        tm, tc = 1.0, t
        for _ in range(60):
            tm, tc = tc, 2.0 * t * tc - tm
        return tc / tm

    lam = np.array([1.0, 1.05, 1.2, 1.4, 1.55, 1.59, 2.0, 3.0, 1.3])
    res = np.array([1e-2, 1e-4, 1e-6, 1e-3, 1e-1, 1e-2, 1e-2, 1e-3, 1e-12])
    tol, dmin, dmax = 1e-10, 4, 40
    got = solver.next_degrees(lam, res, tol, mu1, mu_nevex, mu_n, dmin, dmax)
    for l, r, d in zip(lam, res, got):
        if r <= tol:
            assert d == dmin                        # converged: the smallest degree
            continue
        if l * l >= mu_nevex ** 2:
            assert d == dmax                        # inside the damped interval: no gain rate
            continue
        rho = rho_of(l)
        want = next(dd for dd in range(1, 10 ** 4) if r * rho ** (-dd) <= tol)
        assert d == min(max(want, dmin), dmax), (l, r, d, want)


def _all_eigenpairs(p):
    """Every eigenpair of H from the dense definite solver: the positive
    half and its K-conj partners (Thm 3.1: H K conj(v) = -lambda K conj(v))."""
    lam, V = dense.dense_ph_eig(p.A, p.B)
    return np.concatenate([lam, -lam]), np.concatenate([V, ham.apply_k_conj(V)], axis=1), lam


@pytest.mark.parametrize("m,J,seed", [(8, 3, 0), (8, 5, 1), (10, 4, 2)])
def test_lanczos_estimates_full_dimension_weighted_start(m, J, seed):
    # A start v0 = sum_i c_i v_i over all 2m eigenvectors carries, in the
    # S H inner product, the Gauss weight |c_i|^2 lambda_i v_i^H S v_i on
    # eigenvalue lambda_i (the eigenvectors are S H-orthogonal, eq. 3.5;
    # lambda_i v_i^H S v_i > 0 for both signs since S H is positive definite).
    # The c_i are chosen for weight 1 on every eigenvalue except 2 on the
    # J-th positive one and m on -lambda_1.  A run of n = 2m steps spans the
    # whole space, so its Ritz values are the spectrum and its weights are
    # these, and Section 4.1 then fixes all three estimates: mu_1 the
    # smallest |lambda|, mu_n the largest, and mu_nevex the positive
    # eigenvalue where the weight accumulated over the positive axis alone
    # (total m + 1) first reaches nevex / m; with nevex = J that is lambda_J
    # (J - 1 < J (m + 1) / m <= J + 1).  Weights of the negative axis, from
    # the wrong row of the eigenvectors of T, or a shifted quantile all
    # land elsewhere.
    p = small_problem(m, seed=seed)
    alll, allv, lam = _all_eigenpairs(p)
    sn = np.real(np.einsum("ij,ij->j", allv.conj(), ham.apply_s(allv)))
    w = np.ones(2 * m)
    w[J - 1] = 2.0
    w[m] = float(m)                                  # the partner -lambda_1
    phase = np.exp(2j * np.pi * np.random.default_rng(seed + 7).random(2 * m))
    v0 = allv @ (np.sqrt(w / (alll * sn)) * phase)
    mu1, mu_nevex, mu_n = lanczos.spectral_estimates(p.A, p.B, v0[:, None], 2 * m, J)
    assert abs(mu1 - lam[0]) <= 1e-10 * lam[0]
    assert abs(mu_nevex - lam[J - 1]) <= 1e-10 * lam[J - 1]
    assert abs(mu_n - lam[-1]) <= 1e-10 * lam[-1]


@pytest.mark.parametrize("m,J,seed", [(8, 3, 0), (10, 4, 1)])
def test_lanczos_estimates_start_without_lambda1(m, J, seed):
    # the same construction with no component on lambda_1 (weight 1
    # elsewhere): 2m - 1 steps span the invariant subspace of the other
    # eigenvalues, so mu_1 = min |theta| comes from -lambda_1 alone, and the
    # positive-axis quantile nevex / m of the m - 1 equal weights lands on
    # lambda_(J+1) (J - 1 < J (m - 1) / m <= J)
    p = small_problem(m, seed=seed)
    alll, allv, lam = _all_eigenpairs(p)
    sn = np.real(np.einsum("ij,ij->j", allv.conj(), ham.apply_s(allv)))
    w = np.ones(2 * m)
    w[0] = 0.0
    phase = np.exp(2j * np.pi * np.random.default_rng(seed + 9).random(2 * m))
    v0 = allv @ (np.sqrt(w / (alll * sn)) * phase)
    mu1, mu_nevex, mu_n = lanczos.spectral_estimates(p.A, p.B, v0[:, None], 2 * m - 1, J)
    assert abs(mu1 - lam[0]) <= 1e-10 * lam[0]
    assert abs(mu_nevex - lam[J]) <= 1e-10 * lam[J]
    assert abs(mu_n - lam[-1]) <= 1e-10 * lam[-1]


@pytest.mark.parametrize("steps,seed", [(4, 0), (5, 1), (6, 2)])
def test_lanczos_upper_estimate_is_ritz_value_plus_residual(steps, seed):
    # mu_n = max |theta| plus the S H-norm of the residual of that Ritz
    # pair.  Computed here without the recurrence: Rayleigh-Ritz in the S H
    # inner product on the Krylov space span{v, H v, ..., H^(s-1) v}, with
    # an S H-orthonormal basis from the Cholesky factor of its Gram matrix.
    # H is self-adjoint in that inner product, so an eigenvalue of H lies
    # within the residual of the Ritz value (Krylov-Weinberger bound).
    p = small_problem(8, seed=seed)
    H = ham.assemble_h(p.A, p.B)
    SH = ham.assemble_sh(p.A, p.B)
    v = complex_normal(np.random.default_rng(seed + 11), (16,))
    Kr = np.stack([np.linalg.matrix_power(H, j) @ v for j in range(steps)], axis=1)
    L = np.linalg.cholesky(Kr.conj().T @ SH @ Kr)
    U = scipy.linalg.solve_triangular(L.conj(), Kr.T, lower=True).T      # U = Kr L^-H
    Tr = U.conj().T @ SH @ H @ U
    th, Y = np.linalg.eigh(0.5 * (Tr + Tr.conj().T))
    i = int(np.argmax(np.abs(th)))
    x = U @ Y[:, i]
    r = H @ x - th[i] * x
    delta = math.sqrt(np.real(np.vdot(r, SH @ r)))
    _, mu_nevex, mu_n = lanczos.spectral_estimates(p.A, p.B, v[:, None], steps, 2)
    assert abs(mu_n - (abs(th[i]) + delta)) <= 1e-9 * mu_n
    alll, _, _ = _all_eigenpairs(p)
    assert np.min(np.abs(alll - th[i])) <= delta * (1 + 1e-9)


def test_lanczos_estimates_bounds():
    # on a short run (26 steps, n = 160) the estimates are only bounded
    p = small_problem(80)
    lam, _ = dense.dense_ph_eig(p.A, p.B)
    mu1, mu_nevex, mu_n = lanczos.spectral_estimates(
        p.A, p.B, solver.init_block(p.lanczos_raw, 1e-3), 26, p.nevex)
    assert mu_n >= lam[-1] * (1 - 1e-10)
    assert mu1 <= 1.2 * lam[0]
    assert mu1 < mu_nevex < mu_n


# ------------------------------------------------------------ adjoint
def test_adjoint_central_fd():
    p = small_problem(20)
    nev = 5
    rng = np.random.default_rng(11)
    g = rng.standard_normal(nev)
    lam, V = dense.smallest_positive(p.A, p.B, nev)
    GA, GB = adjoint.eigval_grad(V, g)
    assert np.allclose(GA, GA.conj().T) and np.allclose(GB, GB.T)
    h = 1e-6
    for _ in range(4):
        EA = complex_normal(rng, (20, 20))
        EA = 0.5 * (EA + EA.conj().T)
        EB = complex_normal(rng, (20, 20))
        EB = 0.5 * (EB + EB.T)
        lp, _ = dense.smallest_positive(p.A + h * EA, p.B + h * EB, nev)
        lm, _ = dense.smallest_positive(p.A - h * EA, p.B - h * EB, nev)
        fd = (g @ lp - g @ lm) / (2 * h)
        an = np.real(np.vdot(GA, EA)) + np.real(np.vdot(GB, EB))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_adjoint_scale_invariance():
    # the formula is homogeneous of degree 0 in each eigenvector
    p = small_problem(12)
    lam, V = dense.smallest_positive(p.A, p.B, 3)
    g = np.array([1.0, -2.0, 0.5])
    a1 = adjoint.eigval_grad(V, g)
    a2 = adjoint.eigval_grad(V * np.array([2.0, 1j, -0.3])[None, :], g)
    assert np.allclose(a1[0], a2[0]) and np.allclose(a1[1], a2[1])


def test_adjoint_sampled_entries_match_full_gradient():
    # the entrywise sum (used at sizes where G_A, G_B do not fit on the host)
    # equals the full gradient, which is pinned by finite differences above
    p = small_problem(12)
    lam, V = dense.smallest_positive(p.A, p.B, 4)
    g = np.array([0.7, -1.1, 2.0, 0.3])
    GA, GB = adjoint.eigval_grad(V, g)
    rows, cols = [0, 5, 11], [2, 5, 7, 11]
    ga, gb = adjoint.eigval_grad_entries(V, g, rows, cols)
    assert np.allclose(ga, GA[np.ix_(rows, cols)], rtol=1e-13, atol=1e-15)
    assert np.allclose(gb, GB[np.ix_(rows, cols)], rtol=1e-13, atol=1e-15)


def test_householder_qr_matches_unique_qr():
    # full column rank: the QR with a positive real diagonal is unique, so
    # the Householder route and CholeskyQR2 must agree
    rng = np.random.default_rng(21)
    X = complex_normal(rng, (60, 12))
    Qh, Rh = qr.householder_qr(X)
    Qc, Rc, shifted = qr.cholqr2(X)
    assert not shifted
    assert np.max(np.abs(Qh - Qc)) < 1e-12
    assert np.max(np.abs(Rh - Rc)) < 1e-12 * np.max(np.abs(Rc))
    assert np.allclose(np.diag(Rh).imag, 0) and np.all(np.diag(Rh).real > 0)


def test_orthonormalise_rank_deficient_block():
    # a zero column and a repeated column: both Cholesky variants break down
    # and the Householder QR still returns an orthonormal Q with X = Q R
    rng = np.random.default_rng(22)
    X = complex_normal(rng, (50, 10))
    X[:, 3] = 0
    X[:, 7] = X[:, 2]
    with pytest.raises(np.linalg.LinAlgError):
        qr.cholqr2(X)
    Q, R, variant = qr.orthonormalise(X)
    assert variant == 2
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(10))) < 1e-13
    assert np.max(np.abs(Q @ R - X)) < 1e-13 * np.max(np.abs(X))
    assert np.max(np.abs(np.tril(R, -1))) < 1e-13 * np.max(np.abs(X))
    d = np.diag(R)
    assert np.allclose(d.imag, 0) and np.all(d.real >= 0)
    assert d[3] == 0 and abs(d[7]) < 1e-13 * np.max(np.abs(X))
    # leading columns before the first dependent one: the unique QR
    Qu, Ru = qr.householder_qr(X[:, :3])
    assert np.max(np.abs(Q[:, :3] - Qu)) < 1e-13


def _j(X):
    """J X = K conj(X): swap the halves of the rows and conjugate."""
    m = X.shape[0] // 2
    return np.concatenate([X[m:], X[:m]], axis=0).conj()


def test_kreal_qr_basis():
    rng = np.random.default_rng(23)
    G = complex_normal(rng, (40, 7))
    Q = qr.kreal_qr(G, lead=3)
    assert Q.shape == (40, 14)
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(14))) < 1e-13
    assert np.max(np.abs(_j(Q) - Q)) < 1e-15                       # every column K-real
    span = np.concatenate([G, _j(G)], axis=1)
    assert np.max(np.abs(Q @ (Q.conj().T @ span) - span)) < 1e-13 * np.max(np.abs(span))
    lead = np.concatenate([G[:, :3], _j(G[:, :3])], axis=1)        # first 6 columns: the lead pairs
    Q6 = Q[:, :6]
    assert np.max(np.abs(Q6 @ (Q6.conj().T @ lead) - lead)) < 1e-13 * np.max(np.abs(lead))


def test_kreal_qr_rank_deficient_keeps_pm_pairs():
    # a zero generator: the completed basis is still orthonormal, K-real and
    # K-invariant, so the oblique Rayleigh-Ritz values stay in +/- pairs
    # (Thm 4.5) with a balanced count
    p = small_problem(10)
    rng = np.random.default_rng(24)
    G = complex_normal(rng, (p.n, 4))
    G[:, 1] = 0
    Q = qr.kreal_qr(G)
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(8))) < 1e-13
    assert np.max(np.abs(_j(Q) - Q)) < 1e-15
    span = np.concatenate([G, _j(G)], axis=1)
    assert np.max(np.abs(Q @ (Q.conj().T @ span) - span)) < 1e-13 * np.max(np.abs(span))
    H = ham.assemble_h(p.A, p.B)
    S = np.diag(np.r_[np.ones(p.m), -np.ones(p.m)])
    ev = np.linalg.eigvals(np.linalg.solve(Q.conj().T @ S @ Q, Q.conj().T @ S @ H @ Q))
    assert np.max(np.abs(ev.imag)) < 1e-8
    ev = np.sort(ev.real)
    assert np.sum(ev > 0) == 4
    assert np.max(np.abs(ev + ev[::-1])) < 1e-9 * np.max(np.abs(ev))


# ------------------------------------------------ indefinite S H (Section 5.3)
# The variant for an indefinite S H: dense reference from the general
# eigensolver, Lanczos on S H in the Euclidean inner product for the
# estimates, the quotient of eq. 4.7 solved by a general eigensolver.
def _indefinite_small(m=8, seed=0, coupling=0.05):
    from synth import indefinite_problem
    return indefinite_problem(m, 2, 2, seed=seed, coupling=coupling)


def test_indefinite_generator_is_indefinite_with_real_spectrum():
    from synth import indefinite_problem
    p = indefinite_problem(120, 16, 10)
    assert np.linalg.eigvalsh(ham.assemble_sh(p.A, p.B))[0] < -0.5      # S H indefinite
    w = np.linalg.eigvals(ham.assemble_h(p.A, p.B))
    assert np.max(np.abs(w.imag)) <= 1e-12 * np.max(np.abs(w))
    lam, V, nc = dense.smallest_positive_real(p.A, p.B, p.nev)
    sn = np.real(np.einsum("ij,ij->j", V.conj(), ham.apply_s(V)))
    assert nc == 0 and np.any(sn < 0) and np.any(sn > 0)                 # both S-signs wanted
    with pytest.raises(np.linalg.LinAlgError):
        dense.dense_ph_eig(p.A, p.B)                                     # Thm 3.2's reduction needs S H > 0


def test_general_eig_b_zero_indefinite():
    # B = 0: H = diag(A, -conj(A)), so the positive eigenvalues are the
    # positive d (vectors [x; 0], S-sign +1) and -d for the negative d
    # (vectors [0; conj(x)], S-sign -1)
    p = _indefinite_small(12)
    lam, V, nc = dense.smallest_positive_real(p.A, np.zeros_like(p.B), 12)
    assert nc == 0
    assert np.allclose(lam, np.sort(np.abs(p.d)), rtol=1e-12, atol=0)
    sn = np.real(np.einsum("ij,ij->j", V.conj(), ham.apply_s(V)))
    d_of = np.sort(np.abs(p.d))
    sign_ref = np.array([1.0 if np.any(np.isclose(p.d, x)) else -1.0 for x in d_of])
    assert np.allclose(sn, sign_ref, atol=1e-12)


@pytest.mark.parametrize("m", [4, 8])
def test_general_eig_vs_mpmath_bruteforce_indefinite(m):
    p = _indefinite_small(m, seed=3, coupling=0.3)
    lam, _, nc = dense.smallest_positive_real(p.A, p.B, m)
    mpmath.mp.dps = 50
    H = ham.assemble_h(p.A, p.B)
    Hm = mpmath.matrix([[mpmath.mpc(complex(H[i, j])) for j in range(2 * m)] for i in range(2 * m)])
    ev = mpmath.eig(Hm, left=False, right=False)
    real_pos = sorted(float(mpmath.re(e)) for e in ev
                      if abs(mpmath.im(e)) < 1e-30 and mpmath.re(e) > 0)
    assert nc == sum(1 for e in ev if abs(mpmath.im(e)) >= 1e-30)
    assert np.allclose(np.array(real_pos[:len(lam)]), lam, rtol=1e-13, atol=0)


@pytest.mark.parametrize("m,seed", [(4, 2), (6, 1)])
def test_general_eig_vs_mpmath_with_complex_eigenvalues(m, seed):
    # strong coupling (||B||_2 = 2 min d) puts eigenvalues of H off the real
    # axis: only the real positive ones are returned, the others counted
    p = make_problem(m, lambda rng, mm: rng.uniform(1.0, 2.0, mm), 2.0, 2, 2, 4, 1e-8, seed=seed)
    lam, V, nc = dense.smallest_positive_real(p.A, p.B, 2 * m)
    mpmath.mp.dps = 50
    H = ham.assemble_h(p.A, p.B)
    Hm = mpmath.matrix([[mpmath.mpc(complex(H[i, j])) for j in range(2 * m)] for i in range(2 * m)])
    ev = mpmath.eig(Hm, left=False, right=False)
    cplx = [e for e in ev if abs(mpmath.im(e)) > 1e-20]
    real_pos = sorted(float(mpmath.re(e)) for e in ev if abs(mpmath.im(e)) <= 1e-20 and mpmath.re(e) > 0)
    assert len(cplx) > 0 and nc == len(cplx)
    assert len(lam) == len(real_pos)
    assert np.allclose(lam, np.array(real_pos), rtol=1e-12, atol=0)
    assert np.max(np.linalg.norm(H @ V - V * lam[None, :], axis=0)) < 1e-12 * np.max(np.abs(lam))


def test_general_eig_matches_structured_dense_in_definite_case():
    p = small_problem(30, seed=2)
    lam, _ = dense.smallest_positive(p.A, p.B, 10)
    lam_g, V, nc = dense.smallest_positive_real(p.A, p.B, 10)
    assert nc == 0
    assert np.allclose(lam_g, lam, rtol=1e-12, atol=0)
    H = ham.assemble_h(p.A, p.B)
    assert np.max(np.linalg.norm(H @ V - V * lam_g[None, :], axis=0)) < 1e-12 * np.max(np.abs(lam_g))


@pytest.mark.parametrize("steps", [3, 5, 6])
def test_euclid_lanczos_gauss_quadrature_moments(steps):
    # Hermitian Lanczos on S H: nodes and weights of T reproduce the
    # moments v^H (S H)^j v / v^H v for j < 2 s and miss j = 2 s
    p = _indefinite_small(6, seed=1)
    SH = ham.assemble_sh(p.A, p.B)
    v = complex_normal(np.random.default_rng(3), (12,))
    a, b = lanczos.lanczos_run_euclid(p.A, p.B, v, steps)
    T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    th, Y = np.linalg.eigh(T)
    tau = np.abs(Y[0]) ** 2
    mom = [np.real(np.vdot(v, np.linalg.matrix_power(SH, j) @ v)) / np.real(np.vdot(v, v))
           for j in range(2 * steps + 1)]
    for j in range(2 * steps):
        assert abs(np.sum(tau * th ** j) - mom[j]) <= 1e-11 * max(1.0, abs(mom[j]))
    assert abs(np.sum(tau * th ** (2 * steps)) - mom[2 * steps]) > 1e-8 * abs(mom[2 * steps])


@pytest.mark.parametrize("m,nevex,seed", [(8, 3, 0), (8, 2, 1), (10, 4, 2)])
def test_indefinite_estimates_full_dimension_weighted_start(m, nevex, seed):
    # Start v0 = sum_i c_i u_i over the 2m unit eigenvectors u_i of the
    # Hermitian S H: its Gauss weights are |c_i|^2.  Weight 1 on every
    # eigenvalue except 2 on the one of rank 2 nevex in |theta|.  A run of
    # n steps spans the space, so mu_1 = min |theta|, mu_n = max |theta|
    # (= ||H||_2), and the weight accumulated over |theta| (total n + 1)
    # first reaches nevex / m = 2 nevex / n at rank 2 nevex
    # ((2 nevex - 1)/(n + 1) < 2 nevex / n <= (2 nevex + 1)/(n + 1)).
    p = _indefinite_small(m, seed=seed, coupling=0.3)
    th, U = np.linalg.eigh(ham.assemble_sh(p.A, p.B))
    assert th[0] < 0
    rank = np.argsort(np.abs(th))
    w = np.ones(2 * m)
    w[rank[2 * nevex - 1]] = 2.0
    phase = np.exp(2j * np.pi * np.random.default_rng(seed + 5).random(2 * m))
    v0 = U @ (np.sqrt(w) * phase)
    mu1, mu_nevex, mu_n = lanczos.spectral_estimates_indefinite(p.A, p.B, v0[:, None], 2 * m, nevex)
    a = np.sort(np.abs(th))
    assert abs(mu1 - a[0]) <= 1e-10 * a[-1]
    assert abs(mu_nevex - a[2 * nevex - 1]) <= 1e-10 * a[-1]
    assert abs(mu_n - a[-1]) <= 1e-10 * a[-1]
    assert abs(a[-1] - np.linalg.norm(ham.assemble_h(p.A, p.B), 2)) <= 1e-12 * a[-1]


def test_indefinite_estimates_bound_the_spectrum():
    from synth import indefinite_problem
    p = indefinite_problem(80, 8, 6)
    starts = solver.init_block(p.lanczos_raw, 1e-3)
    mu1, mu_nevex, mu_n = lanczos.spectral_estimates_indefinite(p.A, p.B, starts, 26, p.nevex)
    w = np.linalg.eigvals(ham.assemble_h(p.A, p.B))
    assert mu_n >= np.max(np.abs(w))
    assert 0 < mu1 < mu_nevex < mu_n


def test_general_rr_matches_alg2_in_definite_case():
    # independent routes to the same Ritz values: Cholesky + Hermitian
    # eigensolver of the inverse quotient (Alg. 2) and LU + general
    # eigensolver of eq. 4.7
    p = small_problem(40, seed=4)
    X = complex_normal(np.random.default_rng(5), (80, 6))
    Q, _ = np.linalg.qr(np.concatenate([X, ham.apply_k_conj(X)], axis=1))
    lam1, Z1, _ = rayleigh_ritz.oblique_rr(p.A, p.B, Q)
    lam2, Z2, _ = rayleigh_ritz.oblique_rr_general(p.A, p.B, Q)
    assert np.allclose(lam2, lam1, rtol=1e-11, atol=0)
    for j in range(6):
        v1, v2 = Q @ Z1[:, j], Q @ Z2[:, j]
        assert abs(abs(np.vdot(v1, v2)) - np.linalg.norm(v1) * np.linalg.norm(v2)) < 1e-9 * np.linalg.norm(v1) * np.linalg.norm(v2)


def _kinv_basis(X):
    Q, _ = np.linalg.qr(np.concatenate([X, ham.apply_k_conj(X)], axis=1))
    return Q


def test_general_rr_indefinite_exact_invariant_subspace():
    from synth import indefinite_problem
    p = indefinite_problem(40, 6, 2)
    lam, V, _ = dense.smallest_positive_real(p.A, p.B, 6)
    Q = _kinv_basis(V)
    lam_r, _, _, w, _ = rayleigh_ritz.oblique_rr_general(p.A, p.B, Q, return_all=True)
    assert np.allclose(lam_r, lam, rtol=1e-11, atol=0)
    assert np.allclose(np.sort(w.real), np.sort(np.concatenate([lam, -lam])), rtol=1e-11, atol=0)


def test_general_rr_indefinite_petrov_galerkin_and_pm_pairs():
    # dual basis S Q (Q^H S Q)^{-1} (eq. 4.6): every Ritz pair leaves a
    # residual S-orthogonal to range(Q); on a K-invariant Q the Ritz values
    # come in +/- pairs (Thm 4.5)
    from synth import indefinite_problem
    p = indefinite_problem(40, 6, 2, coupling=0.3)
    X = complex_normal(np.random.default_rng(6), (80, 5))
    Q = _kinv_basis(X)
    lam, Z, T, w, Y = rayleigh_ritz.oblique_rr_general(p.A, p.B, Q, return_all=True)
    for j in range(10):
        v = Q @ Y[:, j]
        r = ham.apply_h(p.A, p.B, v[:, None])[:, 0] - w[j] * v
        assert np.linalg.norm(Q.conj().T @ ham.apply_s(r[:, None])) <= 1e-10 * np.linalg.norm(v) * abs(w[j])
    ws = np.sort_complex(w)
    assert np.allclose(np.sort_complex(-w), ws, atol=1e-10 * np.max(np.abs(w)))


def test_qsq_singular_detects_zero_block():
    A, B, Q, _ = decoupled_singular_case()
    assert rayleigh_ritz.qsq_singular(Q.conj().T @ ham.apply_s(Q))
    Qr = _kinv_basis(complex_normal(np.random.default_rng(1), (20, 3)))
    assert not rayleigh_ritz.qsq_singular(Qr.conj().T @ ham.apply_s(Qr))


@pytest.mark.parametrize("m,nev,nex,seed", [(120, 16, 10, 0), (200, 30, 14, 2)])
def test_solver_indefinite_matches_general_dense(m, nev, nex, seed):
    from synth import indefinite_problem
    p = indefinite_problem(m, nev, nex, tol=1e-10, seed=seed)
    lam_ref, _, _ = dense.smallest_positive_real(p.A, p.B, nev)
    lam, V, info = solver.solve(p.A, p.B, nev, nex, p.deg, p.tol, p.w0_raw, p.lanczos_raw,
                                max_iter=30, definite=False)
    assert info["converged"]
    assert np.allclose(lam, lam_ref, rtol=1e-10, atol=0)
    assert np.all(residuals.residual_norms(p.A, p.B, V, lam) <= p.tol)
    sn = np.real(np.einsum("ij,ij->j", V.conj(), ham.apply_s(V)))
    assert np.any(sn < 0) and np.any(sn > 0)


def test_solver_indefinite_skips_spurious_pairs():
    # With the back-up quotient in every iteration, this problem produces a
    # spurious Ritz value (residual of the order of |lambda~|) ahead of the
    # wanted pairs; it must not hold a place in the locking prefix.
    from synth import indefinite_problem
    p = indefinite_problem(120, 16, 10, tol=1e-10, seed=0)
    lam_ref, _, _ = dense.smallest_positive_real(p.A, p.B, p.nev)
    lam, V, info = solver.solve(p.A, p.B, p.nev, p.nex, p.deg, p.tol, p.w0_raw, p.lanczos_raw,
                                max_iter=30, definite=False, rr_backup=1)
    assert info["converged"] and info["iterations"] <= 10
    assert np.allclose(lam, lam_ref, rtol=1e-10, atol=0)


# ------------------------------------------------ Hermitian ChASE (Alg. 1)
def _tda_problem(m=60, seed=0, nev=6, nex=4):
    return small_problem(m, seed=seed, nev=nev, nex=nex)


@pytest.mark.parametrize("deg", [1, 2, 7])
def test_tda_filter_closed_form_on_eigenvectors(deg):
    # p_d(A) x_i = T_d(t(omega_i)) / T_d(t(mu_1)) x_i, t(w) = (w - c) / e,
    # T_d by cos / cosh (the scaled recurrence equals this ratio exactly)
    from oracle import tda
    p = _tda_problem()
    om, X = np.linalg.eigh(p.A)
    mu1, mu_nevex, mu_m = 0.97 * om[0], om[9], 1.01 * om[-1]
    c, e, _ = tda.filter_params(mu1, mu_nevex, mu_m)

    def T(d, t):
        return math.cos(d * math.acos(t)) if abs(t) <= 1 else (np.sign(t) ** d) * math.cosh(d * math.acosh(abs(t)))

    out = tda.chebyshev_filter(p.A, X, deg, mu1, mu_nevex, mu_m)
    scale = np.array([T(deg, (w - c) / e) / T(deg, (mu1 - c) / e) for w in om])
    assert np.max(np.abs(out - X * scale[None, :])) <= 1e-11 * max(1.0, np.max(np.abs(scale)))


@pytest.mark.parametrize("steps", [3, 6])
def test_tda_lanczos_gauss_quadrature_moments(steps):
    from oracle import tda
    p = _tda_problem(12)
    v = complex_normal(np.random.default_rng(5), (12,))
    a, b = tda.lanczos_run(p.A, v, steps)
    T = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    th, Y = np.linalg.eigh(T)
    tau = np.abs(Y[0]) ** 2
    mom = [np.real(np.vdot(v, np.linalg.matrix_power(p.A, j) @ v)) / np.real(np.vdot(v, v)) for j in range(2 * steps + 1)]
    for j in range(2 * steps):
        assert abs(np.sum(tau * th ** j) - mom[j]) <= 1e-11 * max(1.0, abs(mom[j]))
    assert abs(np.sum(tau * th ** (2 * steps)) - mom[2 * steps]) > 1e-8 * abs(mom[2 * steps])


@pytest.mark.parametrize("m,J,seed", [(10, 3, 0), (12, 5, 1)])
def test_tda_estimates_full_dimension_weighted_start(m, J, seed):
    # weight 1 on every eigenvector of A but 2 on the J-th: a run of m steps
    # gives mu_1 = omega_1, mu_m = omega_m and the left-end quantile
    # nevex / m with nevex = J at omega_J ((J - 1)/(m + 1) < J/m <= (J + 1)/(m + 1))
    from oracle import tda
    p = _tda_problem(m, seed=seed)
    om, X = np.linalg.eigh(p.A)
    w = np.ones(m)
    w[J - 1] = 2.0
    phase = np.exp(2j * np.pi * np.random.default_rng(seed + 3).random(m))
    v0 = X @ (np.sqrt(w) * phase)
    mu1, mu_nevex, mu_m = tda.spectral_estimates(p.A, v0[:, None], m, J)
    assert abs(mu1 - om[0]) <= 1e-10 * om[-1]
    assert abs(mu_nevex - om[J - 1]) <= 1e-10 * om[-1]
    assert abs(mu_m - om[-1]) <= 1e-10 * om[-1]


def test_tda_rayleigh_ritz_exact_and_interlacing():
    from oracle import tda
    p = _tda_problem()
    om, X = np.linalg.eigh(p.A)
    Q, _ = np.linalg.qr(X[:, :5] @ np.linalg.qr(complex_normal(np.random.default_rng(1), (5, 5)))[0])
    om_r, V = tda.rayleigh_ritz(p.A, Q)
    assert np.allclose(om_r, om[:5], rtol=1e-12, atol=0)
    Q, _ = np.linalg.qr(complex_normal(np.random.default_rng(2), (60, 8)))
    om_r, _ = tda.rayleigh_ritz(p.A, Q)
    assert np.all(om_r >= om[:8] - 1e-12) and np.all(om_r <= om[-8:] + 1e-12)   # Cauchy interlacing


@pytest.mark.parametrize("m,nev,nex,seed", [(120, 10, 6, 0), (200, 16, 8, 1)])
def test_tda_solve_matches_the_spectrum_of_a(m, nev, nex, seed):
    # the generator builds A = Q diag(d) Q^H: the nev smallest d are the answer
    from oracle import tda
    p = make_problem(m, lambda rng, mm: rng.uniform(1.0, 5.0, mm), 0.4, nev, nex, 20, 1e-10, seed=seed)
    om, X, info = tda.solve(p.A, nev, nex, 20, 1e-10, p.w0_raw[:m], p.lanczos_raw[:m])
    assert info["converged"]
    assert np.allclose(om, np.sort(p.d)[:nev], rtol=1e-10, atol=0)
    assert np.max(np.linalg.norm(p.A @ X - X * om[None, :], axis=0)) <= 1e-10
    assert np.allclose(X.conj().T @ X, np.eye(nev), atol=1e-10)


def test_auto_nex_minimises_the_estimated_filter_work():
    # uniform density on [1, 5] with 1000 equal weights: the quantiles are
    # known, and the factor of each candidate is 1 / cosh(deg arccosh |t|)
    from oracle import tda
    m, nev, deg, tol = 1000, 20, 12, 1e-9
    th = np.linspace(1.0, 5.0, m)
    w = np.ones(m)
    cands = [2, 5, 10, 20, 40, 80]
    nex, table = tda.auto_nex(th, w, 1.0, 5.0, m, nev, deg, tol, cands)
    costs = []
    for (nx, factor, its, cost) in table:
        om_nev = th[nev - 1]
        om_nevex = th[nev + nx - 1]
        c, e = 0.5 * (5.0 + om_nevex), 0.5 * (5.0 - om_nevex)
        ref = 1.0 / math.cosh(deg * math.acosh(abs((om_nev - c) / e)))
        assert abs(factor - ref) <= 1e-12 * ref
        assert its == math.ceil(math.log(tol / 4.0) / math.log(ref))
        costs.append(its * (nev + nx))
    assert nex == cands[int(np.argmin(costs))]


@pytest.mark.parametrize("m,coupling,seed", [(16, 0.4, 0), (40, 0.9, 1), (64, 0.3, 2)])
def test_inertia_certificate_counts_eigenvalues(m, coupling, seed):
    # the LDL^H (Bunch-Kaufman) count of nu_+(sigma S - S H) against the
    # eigenvalues of the dense solver and the eigenvalues of the shifted
    # matrix itself, at shifts between every few consecutive eigenvalues
    from oracle import inertia
    p = small_problem(m, coupling=coupling, seed=seed)
    lam, _ = dense.dense_ph_eig(p.A, p.B)
    for j in range(0, m - 1, 5):
        sigma = 0.5 * (lam[j] + lam[j + 1])
        M = inertia.shifted_pencil(p.A, p.B, sigma)
        npos_eig = int(np.sum(np.linalg.eigvalsh(np.array(M)) > 0))
        assert inertia.count_below(p.A, p.B, sigma) == j + 1 == npos_eig
    assert inertia.count_below(p.A, p.B, 0.5 * lam[0]) == 0
    assert inertia.count_below(p.A, p.B, 2 * lam[-1]) == m


def test_inertia_count_uses_two_by_two_pivots():
    # an S-indefinite shift makes Bunch-Kaufman take 2 x 2 pivots; the count
    # must still match the eigenvalues of the matrix
    from oracle import inertia
    import scipy.linalg.lapack as lapack
    p = small_problem(40, coupling=0.9, seed=4)
    lam, _ = dense.dense_ph_eig(p.A, p.B)
    sigma = 0.5 * (lam[20] + lam[21])
    M = inertia.shifted_pencil(p.A, p.B, sigma)
    _, ipiv, _ = lapack.zhetrf(np.array(M), lower=1)
    assert np.any(ipiv < 0)
    assert inertia.positive_inertia(M) == 21
