"""GPU parity of each stage of the C ABI against the CPU oracle.

Sizes span several kernel tiles with ragged tails (m = 300: 128-row tiles
end at 44 rows; 2k = 74 output columns end mid-tile).  Tolerances:
FP64 stages ~1e-12 relative (rounding of an O(n) inner product), c64
stages 1e-5 relative (unit roundoff 6e-8 times the inner-product length).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from oracle import chebyshev, dense, hamiltonian as ham, qr as oqr, rayleigh_ritz, residuals as ores, solver as osolver
from paper_2601_10557_amd import FP32, FP64, ChasePHError, PHSolver, empty_cm
from paper_2601_10557_amd import _lib
from synth import make_problem, complex_normal
from gpu_helpers import align_columns, dev_blocks, print_case, to_dev, to_host
from cases import decoupled_singular_case


def problem(m=300, seed=0, coupling=0.4, nev=12, nex=8):
    return make_problem(m, lambda rng, mm: rng.uniform(1.0, 5.0, mm), coupling, nev, nex, 10, 1e-10, seed=seed)


@pytest.fixture(scope="module")
def prob():
    return problem()


@pytest.fixture(scope="module")
def solver(prob):
    A, B = dev_blocks(prob)
    return PHSolver(A, B, prob.nev, prob.nex)


@pytest.mark.parametrize("k", [1, 5, 37])
def test_apply_h_fp64(prob, solver, k):
    print_case("apply_h_fp64", m=prob.m, k=k)
    rng = np.random.default_rng(k)
    X = complex_normal(rng, (prob.n, k))
    Y = to_host(solver.apply_h(to_dev(X)))
    ref = ham.apply_h(prob.A, prob.B, X)
    assert np.max(np.abs(Y - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_apply_h_empty(solver):
    X = empty_cm(solver.n, 0)
    Y = solver.apply_h(X)
    assert Y.shape == (solver.n, 0)


@pytest.mark.parametrize("k", [3, 37])
def test_apply_h_fp32(prob, solver, k):
    print_case("apply_h_fp32", m=prob.m, k=k)
    rng = np.random.default_rng(100 + k)
    X = complex_normal(rng, (prob.n, k))
    Y = to_host(solver.apply_h(to_dev(X, torch.complex64), prec=FP32)).astype(np.complex128)
    ref = ham.apply_h(prob.A, prob.B, X.astype(np.complex64).astype(np.complex128))
    assert np.max(np.abs(Y - ref)) <= 1e-5 * np.max(np.abs(ref))


# every c64 tile shape of the real H X GEMM (0: 256 x 128, 1: 256 x 64 on
# the 32x32x2 MFMA, 2: 256 x 32 on the 16x16x4 MFMA), with and without the
# split-K reduction; "cfg,splits" forces the plan of each launch
@pytest.mark.parametrize("plan", ["0,1", "0,4", "0,9", "1,1", "1,5", "2,1", "2,3", "2,8"])
@pytest.mark.parametrize("k", [37, 61])
def test_apply_h_fp32_every_tile_plan(prob, solver, plan, k, monkeypatch):
    print_case("apply_h_fp32_plan", m=prob.m, k=k, plan=plan)
    monkeypatch.setenv("CHASE_PH_APPLY_PLAN", plan)
    rng = np.random.default_rng(200 + k)
    X = complex_normal(rng, (prob.n, k))
    Y = to_host(solver.apply_h(to_dev(X, torch.complex64), prec=FP32)).astype(np.complex128)
    ref = ham.apply_h(prob.A, prob.B, X.astype(np.complex64).astype(np.complex128))
    assert np.max(np.abs(Y - ref)) <= 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("k", [1, 37, 70])
def test_apply_h_fp64_kreal(prob, solver80, k):
    # K-real columns x = [a; conj(a)]: H x = [t; -conj(t)] from half the
    # products, against the oracle's H X and the general c128 mode
    print_case("apply_h_fp64_kreal", m=prob.m, k=k)
    rng = np.random.default_rng(500 + k)
    a = complex_normal(rng, (prob.m, k))
    X = np.concatenate([a, a.conj()], axis=0)
    Y = to_host(solver80.apply_h(to_dev(X), prec=_lib.FP64_KREAL))
    ref = ham.apply_h(prob.A, prob.B, X)
    assert np.max(np.abs(Y - ref)) <= 1e-12 * np.max(np.abs(ref))
    Yg = to_host(solver80.apply_h(to_dev(X), prec=FP64))
    assert np.max(np.abs(Y - Yg)) <= 1e-13 * np.max(np.abs(ref))


# every c128 tile shape (0: 128 x 128, 1: 128 x 64, 2: 128 x 32, all on
# the f64 16x16x4 MFMA)
@pytest.mark.parametrize("plan", ["0,1", "0,3", "1,1", "1,4", "2,1", "2,6"])
@pytest.mark.parametrize("k", [37, 61])
def test_apply_h_fp64_every_tile_plan(prob, solver, plan, k, monkeypatch):
    print_case("apply_h_fp64_plan", m=prob.m, k=k, plan=plan)
    monkeypatch.setenv("CHASE_PH_APPLY_PLAN", plan)
    rng = np.random.default_rng(300 + k)
    X = complex_normal(rng, (prob.n, k))
    Y = to_host(solver.apply_h(to_dev(X)))
    ref = ham.apply_h(prob.A, prob.B, X)
    assert np.max(np.abs(Y - ref)) <= 1e-12 * np.max(np.abs(ref))


# 2k a few columns past a multiple of 128 (k % 64 <= 20; k >= 64): the
# library splits the launch by columns, in one launch (c64 with 64 < k <= 80:
# one column of wide tiles instead)
@pytest.mark.parametrize("k", [73, 84, 132, 145, 260])
def test_apply_h_column_split(prob, solver, k):
    print_case("apply_h_column_split", m=prob.m, k=k)
    rng = np.random.default_rng(400 + k)
    X = complex_normal(rng, (prob.n, k))
    Y64 = to_host(solver.apply_h(to_dev(X)))
    ref = ham.apply_h(prob.A, prob.B, X)
    assert np.max(np.abs(Y64 - ref)) <= 1e-12 * np.max(np.abs(ref))
    Y32 = to_host(solver.apply_h(to_dev(X, torch.complex64), prec=FP32)).astype(np.complex128)
    ref32 = ham.apply_h(prob.A, prob.B, X.astype(np.complex64).astype(np.complex128))
    assert np.max(np.abs(Y32 - ref32)) <= 1e-5 * np.max(np.abs(ref32))


# c64 products with 64 < k <= 80 on one column of wide tiles (256 x 160): 2k
# up to exactly the tile width (k = 80) and ragged (k = 65, 73); k = 81 and
# k = 132 take the split launch beside them
@pytest.mark.parametrize("k", [65, 73, 80, 81, 132])
def test_apply_h_fp32_wide_last_column(prob, solver, k):
    print_case("apply_h_fp32_wide", m=prob.m, k=k)
    rng = np.random.default_rng(450 + k)
    X = complex_normal(rng, (prob.n, k))
    Y32 = to_host(solver.apply_h(to_dev(X, torch.complex64), prec=FP32)).astype(np.complex128)
    ref32 = ham.apply_h(prob.A, prob.B, X.astype(np.complex64).astype(np.complex128))
    assert np.max(np.abs(Y32 - ref32)) <= 1e-5 * np.max(np.abs(ref32))


# the split launch with every main tile shape (the remainder keeps the
# narrow one): one pair kernel per main shape, or two plain launches when
# the main part is on the narrow shape too
@pytest.mark.parametrize("plan", ["0,1", "0,3", "1,2", "2,4"])
@pytest.mark.parametrize("k", [73, 145])
def test_apply_h_column_split_every_main_plan(prob, solver, plan, k, monkeypatch):
    print_case("apply_h_column_split_plan", m=prob.m, k=k, plan=plan)
    monkeypatch.setenv("CHASE_PH_APPLY_PLAN", plan)
    rng = np.random.default_rng(500 + k)
    X = complex_normal(rng, (prob.n, k))
    Y64 = to_host(solver.apply_h(to_dev(X)))
    ref = ham.apply_h(prob.A, prob.B, X)
    assert np.max(np.abs(Y64 - ref)) <= 1e-12 * np.max(np.abs(ref))
    Y32 = to_host(solver.apply_h(to_dev(X, torch.complex64), prec=FP32)).astype(np.complex128)
    ref32 = ham.apply_h(prob.A, prob.B, X.astype(np.complex64).astype(np.complex128))
    assert np.max(np.abs(Y32 - ref32)) <= 1e-5 * np.max(np.abs(ref32))


def test_apply_h_more_columns_than_the_packed_buffer(prob, solver):
    # the packed operand holds 512 columns: k = 530 runs as 512 + 18
    print_case("apply_h_chunks", m=prob.m, k=530)
    rng = np.random.default_rng(530)
    X = complex_normal(rng, (prob.n, 530))
    Y = to_host(solver.apply_h(to_dev(X)))
    ref = ham.apply_h(prob.A, prob.B, X)
    assert np.max(np.abs(Y - ref)) <= 1e-12 * np.max(np.abs(ref))


def _mus(prob):
    lam, _ = dense.dense_ph_eig(prob.A, prob.B)
    return 0.95 * lam[0], lam[prob.nevex - 1], 1.02 * lam[-1]


@pytest.mark.parametrize("degs", [[1] * 6, [4] * 7, [7] * 5, [1, 2, 2, 3, 7, 7, 10, 11]])
def test_filter_fp64(prob, solver, degs):
    print_case("filter_fp64", m=prob.m, degs=degs)
    mu1, mu_nevex, mu_n = _mus(prob)
    rng = np.random.default_rng(len(degs) + sum(degs))
    W = osolver.init_block(complex_normal(rng, (prob.n, len(degs))), 1e-3)
    Wd = to_dev(W)
    solver.filter(Wd, mu1, mu_nevex, mu_n, degs=degs, prec=FP64)
    ref = chebyshev.chebyshev_filter(prob.A, prob.B, W, np.array(degs), mu1, mu_nevex, mu_n)
    got = to_host(Wd)
    err = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert np.max(err) < 1e-11, err


def test_filter_fp64_column_split(prob):
    # 132 columns: every product of the recurrence takes the column split
    print_case("filter_fp64_column_split", m=prob.m, k=132)
    A, B = dev_blocks(prob)
    wide = PHSolver(A, B, 100, 40)
    mu1, mu_nevex, mu_n = _mus(prob)
    rng = np.random.default_rng(7)
    W = osolver.init_block(complex_normal(rng, (prob.n, 132)), 1e-3)
    Wd = to_dev(W)
    degs = [3] * 132
    wide.filter(Wd, mu1, mu_nevex, mu_n, degs=degs, prec=FP64)
    wide.close()
    ref = chebyshev.chebyshev_filter(prob.A, prob.B, W, np.array(degs), mu1, mu_nevex, mu_n)
    err = np.linalg.norm(to_host(Wd) - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert np.max(err) < 1e-11, err


def test_filter_fp32(prob, solver):
    print_case("filter_fp32", m=prob.m)
    mu1, mu_nevex, mu_n = _mus(prob)
    rng = np.random.default_rng(7)
    degs = [2, 5, 5, 9, 12]
    W = osolver.init_block(complex_normal(rng, (prob.n, len(degs))), 1e-3)
    Wd = to_dev(W, torch.complex64)
    solver.filter(Wd, mu1, mu_nevex, mu_n, degs=degs, prec=FP32)
    ref = chebyshev.chebyshev_filter(prob.A, prob.B, W, np.array(degs), mu1, mu_nevex, mu_n)
    got = to_host(Wd).astype(np.complex128)
    err = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert np.max(err) < 1e-4, err


@pytest.mark.parametrize("eps", [1e-2, 1e-5, 1e-8])
def test_filter_refined_accuracy_tracks_the_residual(prob, solver, eps):
    # c64 products + FP64 refinement: the error is relative to the
    # correction term, so near-eigenvectors are filtered to FP64 accuracy
    # while the plain c64 filter stays at ~1e-6 relative.
    print_case("filter_refined", m=prob.m, eps=eps)
    lam, Vp = dense.dense_ph_eig(prob.A, prob.B)
    mu1, mu_nevex, mu_n = _mus(prob)
    rng = np.random.default_rng(11)
    k = 6
    V = Vp[:, :k] + eps * complex_normal(rng, (prob.n, k))
    V = V / np.linalg.norm(V, axis=0)[None, :]
    HV = ham.apply_h(prob.A, prob.B, V)
    lr = np.real(np.einsum("ij,ij->j", V.conj(), HV))
    R = HV - V * lr[None, :]
    degs = [2, 5, 5, 8, 12, 12]
    ref = chebyshev.chebyshev_filter(prob.A, prob.B, V, np.array(degs), mu1, mu_nevex, mu_n)
    Wd = to_dev(V)
    solver.filter_refined(Wd, to_dev(R), lr, mu1, mu_nevex, mu_n, degs=degs)
    got = to_host(Wd)
    err = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert np.max(err) < 1e-3 * eps + 1e-12, err


def test_filter_kconj_equivariance(prob, solver):
    # Thm 4.2 on the device path
    mu1, mu_nevex, mu_n = _mus(prob)
    rng = np.random.default_rng(3)
    W = complex_normal(rng, (prob.n, 4))
    a = to_dev(W)
    b = to_dev(ham.apply_k_conj(W))
    solver.filter(a, mu1, mu_nevex, mu_n, degs=[6] * 4)
    solver.filter(b, mu1, mu_nevex, mu_n, degs=[6] * 4)
    x, y = to_host(a), to_host(b)
    assert np.max(np.abs(ham.apply_k_conj(x) - y)) <= 1e-11 * np.max(np.abs(y))


def _search_block(prob, kh, seed=0):
    rng = np.random.default_rng(seed)
    mu1, mu_nevex, mu_n = _mus(prob)
    W = osolver.init_block(complex_normal(rng, (prob.n, kh)), 1e-3)
    W = chebyshev.chebyshev_filter(prob.A, prob.B, W, 6, mu1, mu_nevex, mu_n)
    return np.concatenate([W, ham.apply_k_conj(W)], axis=1)


@pytest.mark.parametrize("kh", [3, 20])
def test_qr(prob, solver, kh):
    print_case("qr", m=prob.m, k=2 * kh)
    X = _search_block(prob, kh)
    Xd = to_dev(X)
    R, shifted = solver.qr(Xd)
    Q, R = to_host(Xd), to_host(R)
    Qr, Rr, sh = oqr.cholqr2(X)
    assert not shifted and not sh
    k = X.shape[1]
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(k))) < 1e-12
    assert np.max(np.abs(Q @ R - X)) < 1e-12 * np.max(np.abs(X))
    assert np.max(np.abs(np.tril(R, -1))) == 0.0
    assert np.allclose(np.diag(R).imag, 0) and np.all(np.diag(R).real > 0)
    assert np.max(np.abs(Q - Qr)) < 1e-9
    assert np.max(np.abs(R - Rr)) < 1e-9 * np.max(np.abs(Rr))


def test_qr_shifted_fallback(solver, prob):
    print_case("qr_shifted", m=prob.m)
    rng = np.random.default_rng(1)
    n, k = prob.n, 24
    U, _ = np.linalg.qr(complex_normal(rng, (n, k)))
    Vh, _ = np.linalg.qr(complex_normal(rng, (k, k)))
    X = (U * np.logspace(0, -13, k)[None, :]) @ Vh.conj().T
    Xd = to_dev(X)
    R, shifted = solver.qr(Xd)
    Q, R = to_host(Xd), to_host(R)
    assert shifted == 1
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(k))) < 1e-12
    assert np.max(np.abs(Q @ R - X)) < 1e-12


@pytest.fixture(scope="module")
def solver80(prob):
    """Handle with nevex = 40: QR blocks of up to 80 columns."""
    A, B = dev_blocks(prob)
    return PHSolver(A, B, 20, 20)


def test_qr_householder_fallback_unique_part(solver80, prob):
    # zero last column: both Cholesky variants break down, and the leading
    # 69 columns of the Householder QR are the unique QR (three panels, the
    # last one ragged)
    print_case("qr_householder_unique", m=prob.m, k=70)
    rng = np.random.default_rng(31)
    X = complex_normal(rng, (prob.n, 70))
    X[:, 69] = 0
    Xd = to_dev(X)
    R, variant = solver80.qr(Xd)
    Q, R = to_host(Xd), to_host(R)
    Qo, Ro, vo = oqr.orthonormalise(X)
    assert variant == 2 and vo == 2
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(70))) < 1e-12
    assert np.max(np.abs(Q @ R - X)) < 1e-12 * np.max(np.abs(X))
    assert np.max(np.abs(np.tril(R, -1))) == 0.0
    d = np.diag(R)
    assert np.all(d.imag == 0) and np.all(d.real >= 0)
    assert d[69] == 0
    assert np.max(np.abs(Q[:, :69] - Qo[:, :69])) < 1e-11
    assert np.max(np.abs(R[:69, :] - Ro[:69, :])) < 1e-11 * np.max(np.abs(Ro))


def test_qr_householder_fallback_rank_deficient(solver80, prob):
    # a zero column in the first panel and a repeated one in the second
    # (k = 45: a full panel of 32 and a ragged one of 13)
    print_case("qr_householder_deficient", m=prob.m, k=45)
    rng = np.random.default_rng(32)
    X = complex_normal(rng, (prob.n, 45))
    X[:, 3] = 0
    X[:, 40] = X[:, 7]
    Xd = to_dev(X)
    R, variant = solver80.qr(Xd)
    Q, R = to_host(Xd), to_host(R)
    Qo, _, vo = oqr.orthonormalise(X)
    assert variant == 2 and vo == 2
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(45))) < 1e-12
    assert np.max(np.abs(Q @ R - X)) < 1e-12 * np.max(np.abs(X))
    d = np.diag(R)
    assert np.all(d.imag == 0) and np.all(d.real >= 0)
    assert d[3] == 0 and abs(d[40]) < 1e-12 * np.max(np.abs(X))
    assert np.all(np.delete(d.real, [3, 40]) > 1e-3 * np.max(np.abs(X)))
    assert np.max(np.abs(Q[:, :3] - Qo[:, :3])) < 1e-12


def test_qr_many_cholesky_blocks(prob, solver260):
    # k = 260: the Gram matrix is padded to 320, five 64-column blocks of the
    # blocked Cholesky (diagonal-block factor and inverse, panel, update) and
    # of the blocked inverse; Q and R are unique, so they match the oracle's
    print_case("qr_many_blocks", m=prob.m, k=260)
    rng = np.random.default_rng(41)
    X = complex_normal(rng, (prob.n, 260))
    Xd = to_dev(X)
    R, shifted = solver260.qr(Xd)
    Q, R = to_host(Xd), to_host(R)
    Qr, Rr, sh = oqr.cholqr2(X)
    assert not shifted and not sh
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(260))) < 1e-12
    assert np.max(np.abs(Q @ R - X)) < 1e-12 * np.max(np.abs(X))
    assert np.max(np.abs(np.tril(R, -1))) == 0.0
    assert np.allclose(np.diag(R).imag, 0) and np.all(np.diag(R).real > 0)
    assert np.max(np.abs(Q - Qr)) < 1e-10
    assert np.max(np.abs(R - Rr)) < 1e-10 * np.max(np.abs(Rr))


@pytest.mark.parametrize("kh", [2, 20])
def test_oblique_rr_and_residuals(prob, solver, kh):
    print_case("oblique_rr", m=prob.m, k=2 * kh)
    X = _search_block(prob, kh, seed=5)
    Q, _, _ = oqr.cholqr2(X)
    lam_ref, Z_ref, T_ref = rayleigh_ritz.oblique_rr(prob.A, prob.B, Q)
    Qd = to_dev(Q)
    ritz, Z, T = solver.oblique_rr(Qd)
    assert np.allclose(ritz, lam_ref, rtol=1e-11, atol=0)
    assert np.max(np.abs(to_host(T) - T_ref)) < 1e-12 * np.max(np.abs(T_ref))
    Vref = ores.back_transform(Q, Z_ref)
    rref = ores.residual_norms(prob.A, prob.B, Vref, lam_ref)
    V, res = solver.residuals(Qd, T, Z, ritz)
    V = align_columns(to_host(V), Vref)
    assert np.max(np.abs(V - Vref)) < 1e-8
    assert np.allclose(res, rref, rtol=1e-6, atol=1e-12)
    # Thm 4.5 consequence: the positive Ritz pairs satisfy the Galerkin
    # condition with the dual basis S Q
    Vh = to_host(solver.residuals(Qd, T, Z, ritz)[0])
    R = ham.apply_h(prob.A, prob.B, Vh) - Vh * ritz[None, :]
    assert np.max(np.abs(Q.conj().T @ ham.apply_s(R))) < 1e-11


def test_rr_exact_invariant_subspace(prob, solver):
    lam, Vp = dense.dense_ph_eig(prob.A, prob.B)
    X = np.concatenate([Vp[:, :6], ham.apply_k_conj(Vp[:, :6])], axis=1)
    Q, _, _ = oqr.cholqr2(X)
    ritz, Z, T = solver.oblique_rr(to_dev(Q))
    assert np.allclose(ritz, lam[:6], rtol=1e-12)


def test_rr_reports_an_unconverged_jacobi_eigensolver(prob):
    # one sweep cannot diagonalise the quotient of a random block:
    # CHASE_PH_ERR_EIG, not a silently inaccurate result; with the default
    # limit the same call succeeds
    print_case("rr_jacobi_sweep_limit", m=prob.m, k=40)
    X = _search_block(prob, 20, seed=11)
    Q, _, _ = oqr.cholqr2(X)
    A, B = dev_blocks(prob)
    s1 = PHSolver(A, B, prob.nev, prob.nex, rr_max_sweeps=1)
    with pytest.raises(ChasePHError) as e:
        s1.oblique_rr(to_dev(Q))
    assert e.value.status == _lib.ERR_EIG
    s1.close()
    s40 = PHSolver(A, B, prob.nev, prob.nex)
    ritz, _, _ = s40.oblique_rr(to_dev(Q))
    lam_ref, _, _ = rayleigh_ritz.oblique_rr(prob.A, prob.B, Q)
    assert np.allclose(ritz, lam_ref, rtol=1e-11, atol=0)
    s40.close()


def _unit_ritz(Q, Z):
    V = Q @ Z
    return V / np.linalg.norm(V, axis=0)[None, :]


@pytest.fixture(scope="module")
def solver260(prob):
    """Handle with nevex = 130: Rayleigh-Ritz blocks of up to 260 columns."""
    A, B = dev_blocks(prob)
    s = PHSolver(A, B, 100, 30)
    yield s
    s.close()


@pytest.mark.parametrize("kh", [1, 2, 20, 40, 130])
def test_oblique_rr_backup_matches_oracle(prob, solver, solver80, solver260, kh):
    # Section 5.3 back-up quotient on a filtered search block; k = 2 .. 260
    # (Hessenberg reduction over ragged 64-row groups, QR iteration, back-
    # substitution over up to five 64-thread groups)
    s = solver if kh <= 20 else (solver80 if kh <= 40 else solver260)
    print_case("oblique_rr_backup", m=prob.m, k=2 * kh)
    X = _search_block(prob, kh, seed=6)
    Q, _, _ = oqr.cholqr2(X)
    lam_ref, Z_ref, T_ref = rayleigh_ritz.oblique_rr_backup(prob.A, prob.B, Q)
    Qd = to_dev(Q)
    ritz, Z, T = s.oblique_rr_backup(Qd)
    assert np.allclose(ritz, lam_ref, rtol=1e-10, atol=0)
    assert np.max(np.abs(to_host(T) - T_ref)) < 1e-12 * np.max(np.abs(T_ref))
    Vref = _unit_ritz(Q, Z_ref)
    V = align_columns(_unit_ritz(Q, to_host(Z)), Vref)
    assert np.max(np.abs(V - Vref)) < 1e-8
    Vr, res = s.residuals(Qd, T, Z, ritz)
    rref = ores.residual_norms(prob.A, prob.B, ores.back_transform(Q, Z_ref), lam_ref)
    assert np.allclose(res, rref, rtol=1e-6, atol=1e-12)


def test_oblique_rr_backup_exact_invariant_subspace(prob, solver):
    lam, Vp = dense.dense_ph_eig(prob.A, prob.B)
    X = np.concatenate([Vp[:, :6], ham.apply_k_conj(Vp[:, :6])], axis=1)
    Q, _, _ = oqr.cholqr2(X)
    ritz, Z, T = solver.oblique_rr_backup(to_dev(Q))
    assert np.allclose(ritz, lam[:6], rtol=1e-11)


def test_oblique_rr_backup_recovers_exact_pair_when_qsq_singular():
    # Q^H S Q with a 2 x 2 zero block: Alg. 2 reports the singularity, the
    # back-up quotient returns the exact pair in range(Q)
    A, B, Q, lam_exact = decoupled_singular_case()
    print_case("oblique_rr_backup_singular", m=A.shape[0], k=4)
    p = make_problem(A.shape[0], lambda rng, mm: rng.uniform(1.0, 2.0, mm), 0.1, 1, 1, 4, 1e-8)
    p.A, p.B = A, B
    Ad, Bd = dev_blocks(p)
    s = PHSolver(Ad, Bd, 1, 1)
    with pytest.raises(ChasePHError) as e:
        s.oblique_rr(to_dev(Q))
    assert e.value.status == _lib.ERR_SINGULAR_QSQ
    lam_ref, Z_ref, _ = rayleigh_ritz.oblique_rr_backup(A, B, Q)
    ritz, Z, T = s.oblique_rr_backup(to_dev(Q))
    assert np.allclose(ritz, lam_ref, rtol=1e-12)
    assert np.min(np.abs(ritz - lam_exact)) < 1e-12 * lam_exact


def test_oblique_rr_backup_on_s_neutral_basis(prob, solver):
    # Q^H S Q = 0: every diagonal entry is replaced by 1
    m, k = prob.m, 4
    Q = np.zeros((prob.n, k), dtype=np.complex128)
    for j in range(k):
        Q[j, j] = Q[m + j, j] = 1 / np.sqrt(2)
    lam_ref, _, _ = rayleigh_ritz.oblique_rr_backup(prob.A, prob.B, Q)
    ritz, _, _ = solver.oblique_rr_backup(to_dev(Q))
    assert np.allclose(ritz, lam_ref, rtol=1e-12)


def test_backward_matches_oracle(prob, solver):
    from oracle import adjoint
    lam, V = dense.smallest_positive(prob.A, prob.B, 7)
    g = np.random.default_rng(2).standard_normal(7)
    GA_ref, GB_ref = adjoint.eigval_grad(V, g)
    GA, GB = solver.eigval_backward(to_dev(V), g)
    GA, GB = to_host(GA), to_host(GB)
    assert np.max(np.abs(GA - GA_ref)) < 1e-12 * np.max(np.abs(GA_ref))
    assert np.max(np.abs(GB - GB_ref)) < 1e-12 * np.max(np.abs(GB_ref))


# ------------------------------------------------------------ error paths
def test_argument_errors(solver, prob):
    X = to_dev(np.zeros((prob.n, 3)))
    with pytest.raises(ChasePHError) as e:
        solver.oblique_rr(X)          # odd k
    assert e.value.status == _lib.ERR_ARG
    W = to_dev(np.ones((prob.n, 3)))
    with pytest.raises(ChasePHError) as e:
        solver.filter(W, 1.0, 2.0, 5.0, degs=[3, 2, 4])   # not sorted
    assert e.value.status == _lib.ERR_ARG
    with pytest.raises(ChasePHError) as e:
        solver.filter(W, 2.0, 1.0, 5.0)                   # mu order
    assert e.value.status == _lib.ERR_ARG


def test_not_definite_detected():
    # SH indefinite: ||B||_2 = 2 min d.  A block containing an eigenvector of
    # SH with a negative eigenvalue makes Q^H S H Q indefinite.
    p = make_problem(64, lambda rng, mm: rng.uniform(1.0, 2.0, mm), 2.0, 2, 2, 4, 1e-8)
    SH = ham.assemble_sh(p.A, p.B)
    w, U = np.linalg.eigh(SH)
    assert w[0] < 0
    X = np.concatenate([U[:, :1], ham.apply_k_conj(U[:, :1])], axis=1)
    Q, _, _ = oqr.cholqr2(X)
    A, B = dev_blocks(p)
    s = PHSolver(A, B, 2, 2)
    with pytest.raises(ChasePHError) as e:
        s.oblique_rr(to_dev(Q))
    assert e.value.status == _lib.ERR_NOT_DEFINITE


def test_singular_qsq_detected(prob, solver):
    # S-neutral basis (Section 4.6): Q^H S Q = 0
    m, k = prob.m, 4
    Q = np.zeros((prob.n, k), dtype=np.complex128)
    for j in range(k):
        Q[j, j] = Q[m + j, j] = 1 / np.sqrt(2)
    with pytest.raises(ChasePHError) as e:
        solver.oblique_rr(to_dev(Q))
    assert e.value.status == _lib.ERR_SINGULAR_QSQ
