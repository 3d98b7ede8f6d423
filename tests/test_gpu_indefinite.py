"""Parity of the indefinite-S H variant (Section 5.3, last paragraph: a
non-hermitian quotient does not need S H to be definite) against the
oracle: Euclidean Lanczos estimates on S H, the quotient of eq. 4.7 by a
general eigensolver (chase_ph_oblique_rr_general) and the whole solve with
definite = 0, in both precisions.  Bar: eigenvalues within 1e-10 relative
of the general dense reference (FP64 path) and 1e-9 (mixed path); every
returned pair has residual <= tol."""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from cases import decoupled_singular_case
from gpu_helpers import align_columns, dev_blocks, print_case, to_dev, to_host
from oracle import dense, hamiltonian as ham, lanczos, rayleigh_ritz, residuals as ores
from oracle import solver as osolver
from paper_2601_10557_amd import FP64, MIXED, ChasePHError, PHSolver
from paper_2601_10557_amd import _lib
from synth import complex_normal, config_problem, indefinite_problem, make_problem


@pytest.fixture(scope="module")
def ind():
    # m = 300: the 64-row tiles of the H X kernels end on a ragged 44 rows
    p = indefinite_problem(300, 40, 20, tol=1e-10, seed=4)
    lam, V, nc = dense.smallest_positive_real(p.A, p.B, p.nev + p.nex)
    assert nc == 0
    return p, lam, V


def _solver(p, **kw):
    A, B = dev_blocks(p)
    return PHSolver(A, B, p.nev, p.nex, deg=p.deg, tol=kw.pop("tol", p.tol), definite=False, **kw)


def _kinv_basis(X):
    Q, _ = np.linalg.qr(np.concatenate([X, ham.apply_k_conj(X)], axis=1))
    return Q


def _unit_ritz(Q, Z):
    V = Q @ Z
    return V / np.linalg.norm(V, axis=0)[None, :]


def test_lanczos_indefinite_estimates_match_oracle(ind):
    p, _, _ = ind
    print_case("lanczos_indefinite", m=p.m)
    s = _solver(p, max_iter=1)
    _, _, _, info = s.solve(to_dev(p.w0_raw), to_dev(p.lanczos_raw), raise_on_noconv=False)
    s.close()
    ref = lanczos.spectral_estimates_indefinite(p.A, p.B, osolver.init_block(p.lanczos_raw, 1e-3), 26, p.nevex)
    assert np.allclose([info.mu1, info.mu_nevex0, info.mu_n], ref, rtol=1e-9, atol=0)


@pytest.mark.parametrize("kh,noise", [(1, 1e-2), (6, 1e-2), (30, 1e-3), (60, 1e-3)])
def test_oblique_rr_general_matches_oracle(ind, kh, noise):
    # K-invariant block near the wanted eigenvectors (both S-signs among
    # them) plus noise: k = 2 .. 120 (Householder QR of Q^H S Q over up to
    # four panels, Hessenberg reduction and QR iteration)
    p, lam, V = ind
    print_case("oblique_rr_general", m=p.m, k=2 * kh)
    X = V[:, :kh] + noise * complex_normal(np.random.default_rng(kh), (p.n, kh))
    Q = _kinv_basis(X)
    lam_ref, Z_ref, T_ref = rayleigh_ritz.oblique_rr_general(p.A, p.B, Q)
    s = _solver(p)
    Qd = to_dev(Q)
    ritz, Z, T = s.oblique_rr_general(Qd)
    assert np.allclose(ritz, lam_ref, rtol=1e-10, atol=0)
    assert np.max(np.abs(to_host(T) - T_ref)) < 1e-12 * np.max(np.abs(T_ref))
    Vref = _unit_ritz(Q, Z_ref)
    Vg = align_columns(_unit_ritz(Q, to_host(Z)), Vref)
    assert np.max(np.abs(Vg - Vref)) < 1e-8
    Vr, res = s.residuals(Qd, T, Z, ritz)
    rref = ores.residual_norms(p.A, p.B, ores.back_transform(Q, Z_ref), lam_ref)
    assert np.allclose(res, rref, rtol=1e-6, atol=1e-12)
    s.close()


def test_oblique_rr_general_exact_invariant_subspace(ind):
    p, lam, V = ind
    print_case("oblique_rr_general_exact", m=p.m, k=16)
    s = _solver(p)
    ritz, _, _ = s.oblique_rr_general(to_dev(_kinv_basis(V[:, :8])))
    assert np.allclose(ritz, lam[:8], rtol=1e-11, atol=0)
    s.close()


def test_oblique_rr_general_equals_alg2_in_definite_case():
    p = config_problem(0, m=300, nev=10, nex=6)
    print_case("oblique_rr_general_definite", m=p.m, k=20)
    lam, V = dense.smallest_positive(p.A, p.B, 10)
    Q = _kinv_basis(V + 1e-2 * complex_normal(np.random.default_rng(3), V.shape))
    lam_ref, _, _ = rayleigh_ritz.oblique_rr(p.A, p.B, Q)
    A, B = dev_blocks(p)
    s = PHSolver(A, B, p.nev, p.nex)
    ritz, _, _ = s.oblique_rr_general(to_dev(Q))
    assert np.allclose(ritz, lam_ref, rtol=1e-10, atol=0)
    s.close()


def test_oblique_rr_general_reports_singular_qsq():
    A, B, Q, _ = decoupled_singular_case()
    print_case("oblique_rr_general_singular", m=A.shape[0], k=4)
    p = make_problem(A.shape[0], lambda rng, mm: rng.uniform(1.0, 2.0, mm), 0.1, 1, 1, 4, 1e-8)
    p.A, p.B = A, B
    Ad, Bd = dev_blocks(p)
    s = PHSolver(Ad, Bd, 1, 1)
    with pytest.raises(ChasePHError) as e:
        s.oblique_rr_general(to_dev(Q))
    assert e.value.status == _lib.ERR_SINGULAR_QSQ
    s.close()


def _check(p, lam, ev, V, res, rtol):
    assert len(ev) == p.nev and np.all(np.diff(ev) > 0)
    assert np.max(np.abs(ev - lam[: p.nev]) / lam[: p.nev]) <= rtol
    Vh = to_host(V)
    r = ores.residual_norms(p.A, p.B, Vh, ev)
    assert np.all(r <= 1.5 * p.tol) and np.all(res <= p.tol)
    sn = np.real(np.einsum("ij,ij->j", Vh.conj(), ham.apply_s(Vh)))
    assert np.any(sn < 0) and np.any(sn > 0)      # wanted pairs of both S-signs


def test_solve_indefinite_fp64(ind):
    p, lam, _ = ind
    print_case("solve_indefinite_fp64", m=p.m, nev=p.nev)
    s = _solver(p, precision=FP64)
    ev, V, res, info = s.solve(to_dev(p.w0_raw), to_dev(p.lanczos_raw))
    _check(p, lam, ev, V, res, 1e-10)
    assert info.general_rr_used == info.iterations - info.backup_rr_used
    s.close()


def test_solve_indefinite_mixed(ind):
    p, lam, _ = ind
    print_case("solve_indefinite_mixed", m=p.m, nev=p.nev)
    s = _solver(p, precision=MIXED, tol=1e-9)
    ev, V, res, info = s.solve(to_dev(p.w0_raw), to_dev(p.lanczos_raw))
    _check(dataclasses.replace(p, tol=1e-9), lam, ev, V, res, 1e-9)
    s.close()


def test_solve_indefinite_variant_on_a_definite_problem():
    # definite = 0 must also reach the answer when S H happens to be definite
    p = config_problem(0)
    print_case("solve_indefinite_variant_definite", m=p.m)
    lam, _ = dense.dense_ph_eig(p.A, p.B)
    s = _solver(p, precision=FP64)
    ev, V, res, info = s.solve(to_dev(p.w0_raw), to_dev(p.lanczos_raw))
    assert np.max(np.abs(ev - lam[: p.nev]) / lam[: p.nev]) <= 1e-10
    assert np.all(ores.residual_norms(p.A, p.B, to_host(V), ev) <= 1.5 * p.tol)
    s.close()


def test_definite_path_rejects_indefinite_problem(ind):
    # Alg. 2 and the S H inner product need S H > 0: the definite path stops
    # with CHASE_PH_ERR_NOT_DEFINITE on the indefinite problem
    p, _, _ = ind
    print_case("definite_path_on_indefinite", m=p.m)
    A, B = dev_blocks(p)
    s = PHSolver(A, B, p.nev, p.nex, deg=p.deg, tol=p.tol)
    with pytest.raises(ChasePHError) as e:
        s.solve(to_dev(p.w0_raw), to_dev(p.lanczos_raw))
    assert e.value.status == _lib.ERR_NOT_DEFINITE
    s.close()
