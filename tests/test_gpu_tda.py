"""Parity of Hermitian ChASE on A alone (Alg. 1; the B = 0 block of
Section 1.1) against the oracle: the TDA mode of the H X kernels (A X on
D = [A, iA]), the Lanczos estimates on A, the whole solve (eq. 2.1 filter,
Cholesky QR, Rayleigh-Ritz of eq. 2.2, residual locking) and the automatic
nex.  Bar: A X within 1e-13 (FP64) and 1e-5 (FP32) of the norm-scaled
product; eigenvalues within 1e-10 relative of numpy's eigh of A; every
returned pair has residual <= tol; the automatic nex equals the oracle's
choice on the oracle's own Lanczos density."""
import ctypes as C
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_helpers import print_case, to_dev, to_host
from oracle import tda
from paper_2601_10557_amd import FP32, FP64, ChasePHError, PHSolver, TDASolver, lib
from paper_2601_10557_amd import _lib
from synth import complex_normal, make_problem


def _problem(m, nev, nex, lo=1.0, hi=5.0, seed=0, tol=1e-10):
    return make_problem(m, lambda rng, mm: rng.uniform(lo, hi, mm), 0.3, nev, nex, 20, tol, seed=seed)


def _dev_a(p):
    return torch.from_numpy(np.ascontiguousarray(p.A)).cuda()


@pytest.mark.parametrize("m,k", [(300, 1), (300, 37), (300, 130), (257, 64), (64, 5)])
def test_apply_a_matches_the_product(m, k):
    # m = 300: the 2m = 600 real rows end on a ragged tile; k = 130 puts the
    # real columns past one 128-wide tile
    print_case("tda_apply_a", m=m, k=k)
    p = _problem(m, 4, 2, seed=m + k)
    X = complex_normal(np.random.default_rng(k), (m, k))
    ref = p.A @ X
    s = TDASolver(_dev_a(p), 4, 2)
    Y = to_host(s.apply_a(to_dev(X)))
    scale = np.linalg.norm(p.A, 2) * np.max(np.linalg.norm(X, axis=0))
    assert np.max(np.abs(Y - ref)) <= 1e-13 * scale
    Y32 = to_host(s.apply_a(to_dev(X, torch.complex64), prec=FP32)).astype(np.complex128)
    assert np.max(np.abs(Y32 - ref)) <= 1e-5 * scale
    s.close()


def test_tda_lanczos_estimates_match_oracle():
    p = _problem(300, 20, 10, seed=3)
    print_case("tda_lanczos", m=p.m)
    s = TDASolver(_dev_a(p), p.nev, p.nex, max_iter=1)
    _, _, _, info = s.solve(to_dev(p.w0_raw[: p.m]), to_dev(p.lanczos_raw[: p.m]), raise_on_noconv=False)
    s.close()
    ref = tda.spectral_estimates(p.A, p.lanczos_raw[: p.m], 26, p.nev + p.nex)
    assert np.allclose([info.mu1, info.mu_nevex0, info.mu_n], ref, rtol=1e-9, atol=0)


def _check_solution(p, ev, V, res, nev, tol):
    om = np.linalg.eigvalsh(p.A)
    assert len(ev) == nev
    assert np.max(np.abs(ev - om[:nev]) / np.maximum(1.0, np.abs(om[:nev]))) <= 1e-10
    X = to_host(V)
    r = np.linalg.norm(p.A @ X - X * ev[None, :], axis=0)
    assert np.all(r <= 1.5 * tol) and np.all(res <= tol)
    assert np.max(np.abs(X.conj().T @ X - np.eye(nev))) <= 1e-10


@pytest.mark.parametrize("m,nev,nex,lo,hi,seed", [(300, 20, 10, 1.0, 5.0, 0), (257, 12, 8, -2.0, 3.0, 1),
                                                  (130, 1, 4, 0.5, 9.0, 2)])
def test_tda_solve_matches_oracle_and_eigh(m, nev, nex, lo, hi, seed):
    # (257, -2 .. 3): an indefinite A (Alg. 1 takes the smallest eigenvalues);
    # nev = 1: a single wanted pair
    p = _problem(m, nev, nex, lo, hi, seed)
    print_case("tda_solve", m=m, nev=nev, nex=nex, seed=seed)
    s = TDASolver(_dev_a(p), nev, nex, tol=p.tol)
    ev, V, res, info = s.solve(to_dev(p.w0_raw[:m]), to_dev(p.lanczos_raw[:m]))
    s.close()
    _check_solution(p, ev, V, res, nev, p.tol)
    om_ref, X_ref, inf_ref = tda.solve(p.A, nev, nex, 20, p.tol, p.w0_raw[:m], p.lanczos_raw[:m])
    assert inf_ref["converged"]
    assert np.allclose(ev, om_ref, rtol=1e-11, atol=1e-11)
    # same iteration, up to a locking decision taken on a residual within
    # rounding of tol
    assert abs(info.iterations - inf_ref["iterations"]) <= 1
    assert info.nex_used == nex


def test_tda_equals_the_pseudo_hermitian_solver_at_b_zero():
    # Section 1.1: with B = 0 the positive eigenpairs of H are those of A,
    # with vectors [x; 0]
    p = _problem(300, 16, 8, seed=5)
    print_case("tda_vs_ph_b0", m=p.m)
    s = TDASolver(_dev_a(p), p.nev, p.nex, tol=p.tol)
    ev_t, V_t, _, _ = s.solve(to_dev(p.w0_raw[: p.m]), to_dev(p.lanczos_raw[: p.m]))
    s.close()
    A = _dev_a(p)
    ph = PHSolver(A, torch.zeros_like(A), p.nev, p.nex, tol=p.tol)
    ev_h, V_h, _, _ = ph.solve(to_dev(p.w0_raw), to_dev(p.lanczos_raw))
    ph.close()
    assert np.allclose(ev_t, ev_h, rtol=1e-11, atol=0)
    Vh = to_host(V_h)
    assert np.max(np.abs(Vh[p.m:])) <= 1e-10
    Vt = to_host(V_t)
    ov = np.abs(np.sum(Vt.conj() * Vh[: p.m], axis=0))   # |<x_tda, x_ph>| = 1 for simple eigenvalues
    assert np.all(ov >= 1 - 1e-9)


def test_tda_nex_auto_matches_oracle_choice():
    p = _problem(400, 20, 40, seed=7)
    print_case("tda_nex_auto", m=p.m)
    s = TDASolver(_dev_a(p), p.nev, p.nex, tol=p.tol, nex_auto=True)
    ev, V, res, info = s.solve(to_dev(p.w0_raw[: p.m]), to_dev(p.lanczos_raw[: p.m]))
    s.close()
    th, w, mu_m = tda.lanczos_density(p.A, p.lanczos_raw[: p.m], 26)
    cands = sorted({math.ceil(j * p.nex / 8) for j in range(1, 9)})
    nex_ref, _ = tda.auto_nex(th, w, float(th[0]), mu_m, p.m, p.nev, 20, p.tol, cands)
    assert info.nex_used == nex_ref
    _check_solution(p, ev, V, res, p.nev, p.tol)


def test_pseudo_hermitian_stage_calls_refuse_a_tda_handle():
    p = _problem(64, 4, 2, seed=9)
    print_case("tda_stage_refusal", m=p.m)
    s = TDASolver(_dev_a(p), 4, 2)
    W = to_dev(complex_normal(np.random.default_rng(0), (2 * p.m, 6)))
    st = lib().chase_ph_filter(s._h, 6, C.c_void_p(W.data_ptr()), 2 * p.m, None, 1.0, 2.0, 5.0, FP64)
    assert st == _lib.ERR_ARG
    with pytest.raises(ChasePHError):
        s.apply_a(to_dev(np.zeros((p.m, 2))), prec=_lib.FP64_KREAL)
    s.close()
