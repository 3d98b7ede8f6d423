"""Full-size GPU checks of the larger workloads.

* adjoint workload (m = 2000): gradient of L = sum_i w_i lambda_i against the
  dense FP64 oracle gradient and against central finite differences
  (h = 1e-6) on 32 random unit-Frobenius Hermitian/symmetric directions;
* clustered (m = 16000) and largest (m = 30000) workloads, at full size:
  - H X in c64 and c128 on sampled rows recomputed on the host from rows of
    A and B, and Thm 4.2 (K-conj equivariance of the filter);
  - one pass of the stage chain (c64 filter with per-vector degrees, QR,
    oblique Rayleigh-Ritz, residuals, eigenvalue adjoint) checked on sampled
    columns against host recomputation and the oracle's formulas.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from oracle import adjoint, dense
from oracle.hamiltonian import apply_s
from paper_2601_10557_amd import FP32, FP64, PHSolver, colmajor, eigsh_ph
from synth import config_problem
from synth.gpu import config_problem_device
from gpu_helpers import print_case, to_dev, to_host


def test_adjoint_workload_fd_and_dense_gradient():
    p = config_problem(3)
    print_case("adjoint_m2000", m=p.m, nev=p.nev)
    A = torch.from_numpy(p.A).cuda()
    B = torch.from_numpy(p.B).cuda()
    W0, Lz = to_dev(p.w0_raw), to_dev(p.lanczos_raw)
    kw = dict(deg=p.deg, tol=p.tol, max_iter=40)
    Ag = A.clone().requires_grad_(True)
    Bg = B.clone().requires_grad_(True)
    lam = eigsh_ph(Ag, Bg, p.nev, p.nex, W0, Lz, **kw)
    w = torch.from_numpy(p.loss_w).cuda()
    (lam * w).sum().backward()
    GA, GB = to_host(Ag.grad), to_host(Bg.grad)
    # dense FP64 reference gradient from the oracle's eigenvectors
    lam_ref, Vref = dense.smallest_positive(p.A, p.B, p.nev)
    assert np.max(np.abs(to_host(lam) - lam_ref) / lam_ref) < 1e-11
    GA_ref, GB_ref = adjoint.eigval_grad(Vref, p.loss_w)
    assert np.max(np.abs(GA - GA_ref)) < 1e-8 * np.max(np.abs(GA_ref))
    assert np.max(np.abs(GB - GB_ref)) < 1e-8 * np.max(np.abs(GB_ref))
    # central finite differences through the GPU solver
    rng = np.random.default_rng(123)
    h = 1e-6
    worst = 0.0
    for t in range(32):
        EA = rng.standard_normal((p.m, p.m)) + 1j * rng.standard_normal((p.m, p.m))
        EA = 0.5 * (EA + EA.conj().T)
        EA /= np.linalg.norm(EA)
        EB = rng.standard_normal((p.m, p.m)) + 1j * rng.standard_normal((p.m, p.m))
        EB = 0.5 * (EB + EB.T)
        EB /= np.linalg.norm(EB)
        EAd, EBd = torch.from_numpy(EA).cuda(), torch.from_numpy(EB).cuda()
        vals = []
        for sgn in (1.0, -1.0):
            s = PHSolver(A + sgn * h * EAd, B + sgn * h * EBd, p.nev, p.nex, **kw)
            ev, _, _, _ = s.solve(W0, Lz)
            s.close()
            vals.append(float(p.loss_w @ ev))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = float(np.real(np.vdot(GA, EA)) + np.real(np.vdot(GB, EB)))
        rel = abs(fd - an) / max(1.0, abs(an))
        worst = max(worst, rel)
    print_case("adjoint_fd", worst_rel=worst)
    assert worst <= 1e-6


def _sampled_rows_check(p, k, prec):
    m = p.m
    s = PHSolver(p.A, p.B, 8, 8)
    dt = torch.complex64 if prec == FP32 else torch.complex128
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    X = torch.complex(torch.randn(2 * m, k, dtype=torch.float64, device="cuda", generator=g),
                      torch.randn(2 * m, k, dtype=torch.float64, device="cuda", generator=g)).to(dt)
    X = colmajor(X)
    Y = s.apply_h(X, prec=prec)
    rows = np.r_[0, 1, m // 3, m - 1]
    Xh = X.cpu().numpy().astype(np.complex128)
    Ah = p.A[rows].cpu().numpy()
    Bh = p.B[rows].cpu().numpy()
    if prec == FP32:
        Ah = Ah.astype(np.complex64).astype(np.complex128)
        Bh = Bh.astype(np.complex64).astype(np.complex128)
    X1, X2 = Xh[:m], Xh[m:]
    top = Ah @ X1 + Bh @ X2                      # rows of A X1 + B X2
    bot = -(Bh.conj() @ X1 + Ah.conj() @ X2)     # rows of -(conj(B) X1 + conj(A) X2)
    Yh = Y.cpu().numpy().astype(np.complex128)
    err_t = np.max(np.abs(Yh[rows] - top)) / np.max(np.abs(top))
    err_b = np.max(np.abs(Yh[m + rows] - bot)) / np.max(np.abs(bot))
    s.close()
    return max(err_t, err_b)


U32 = 2.0 ** -24  # unit roundoff of binary32


def _c64_apply_tol(m):
    """Bound on max |error| / max |exact| of one c64 product with H.

    The test rounds A, B and X to c64 on both sides, so only the FP32
    accumulation over the inner dimension n = 2m differs.  Its error grows
    like u sqrt(n) relative to the result (probabilistic rounding-error
    analysis of inner products); the factor 4 covers the complex products
    (four real products per term) and the max over sampled entries.
    """
    return 4.0 * U32 * np.sqrt(2.0 * m)


@pytest.fixture(scope="module", params=[2, 4])
def big(request):
    """Full-size clustered (m = 16000) and largest (m = 30000) workloads,
    drawn on the device; pytest runs every test of one before the next."""
    p = config_problem_device(request.param)
    yield request.param, p
    del p
    torch.cuda.empty_cache()


def test_apply_h_full_size_sampled_rows(big):
    cfg, p = big
    print_case("apply_h_full", cfg=cfg, m=p.m)
    assert _sampled_rows_check(p, 64, FP64) < 1e-12
    e32 = _sampled_rows_check(p, 64, FP32)
    print_case("apply_h_full_c64", cfg=cfg, err=e32, tol=_c64_apply_tol(p.m))
    assert e32 < _c64_apply_tol(p.m)
    # Thm 4.2 at full size: p(H^2) K conj(W) = K conj(p(H^2) W) (c64 filter)
    s = PHSolver(p.A, p.B, 8, 8)
    m = p.m
    W = p.w0_raw[:, :4].clone()
    KW = torch.cat([W[m:], W[:m]], dim=0).conj()
    a = colmajor(W.to(torch.complex64))
    b = colmajor(KW.to(torch.complex64))
    mu1, mu_nevex, mu_n = 0.9 * p.d.min() * (1 - p.coupling), 0.5 * (p.d.min() + p.d.max()) * 0.3, 1.1 * p.d.max() * (1 + p.coupling)
    s.filter(a, mu1, mu_nevex, mu_n, degs=[3] * 4, prec=FP32)
    s.filter(b, mu1, mu_nevex, mu_n, degs=[3] * 4, prec=FP32)
    x = a.cpu().numpy()
    y = b.cpu().numpy()
    kx = np.concatenate([x[m:], x[:m]], axis=0).conj()
    # both sides carry the rounding of 2 * deg c64 products
    assert np.max(np.abs(kx - y)) <= 2 * 3 * _c64_apply_tol(m) * np.max(np.abs(y))
    s.close()


def test_stage_chain_full_size(big):
    """One pass of filter -> QR -> Rayleigh-Ritz -> residuals -> adjoint at
    full size, in the launch configuration of the solver, on sampled columns.

    The filter interval comes from bounds that hold for every definite
    problem: |lambda| <= rho(A) = max d (Section 3) and lambda >= (1 - c) min d
    (Weyl: SH >= (1 - c) min d I).  The clustered workload runs per-vector
    degrees spread over [10, 36]; the largest one degree 3 (time)."""
    cfg, p = big
    m, n, nevex, nev = p.m, p.n, p.nevex, p.nev
    k = 2 * nevex
    lo = (1.0 - p.coupling) * float(p.d.min())
    mu1, mu_nevex, mu_n = 0.95 * lo, float(np.sort(p.d)[nevex]), 1.01 * float(p.d.max())
    if p.deg_min != p.deg_max:
        degs = np.round(np.linspace(p.deg_min, p.deg_max, nevex)).astype(int)
    else:
        degs = np.full(nevex, 3)
    print_case("stage_chain_full", cfg=cfg, m=m, nevex=nevex, deg_lo=int(degs[0]), deg_hi=int(degs[-1]))
    s = PHSolver(p.A, p.B, nev, p.nex, tol=p.tol)
    W = p.w0_raw.clone()
    W[m:] *= 1e-3                                    # Section 4.6
    W32 = colmajor(W.to(torch.complex64))
    del W
    s.filter(W32, mu1, mu_nevex, mu_n, degs=degs.tolist(), prec=FP32)
    W = W32.to(torch.complex128)
    del W32
    X = colmajor(torch.cat([W, torch.cat([W[m:], W[:m]]).conj()], dim=1))   # [W+, K conj(W+)]
    del W
    X0 = X.cpu().numpy()
    R, shifted = s.qr(X)
    ritz, Z, T = s.oblique_rr(X)
    V, res = s.residuals(X, T, Z, ritz)
    g = np.random.default_rng(11).standard_normal(nev)
    GA, GB = s.eigval_backward(V[:, :nev], g)
    rows, gcols = np.r_[0, m // 2, m - 1], np.r_[0, 7, m // 3, m - 1]
    ga = GA[rows][:, gcols].cpu().numpy()
    gb = GB[rows][:, gcols].cpu().numpy()
    del GA, GB
    torch.cuda.synchronize()
    print_case("stage_chain_full_done", cfg=cfg, shifted_qr=shifted, ritz0=float(ritz[0]), ritz_last=float(ritz[-1]))
    Qh, Th, Zh, Vh, Rh = (t.cpu().numpy() for t in (X, T, Z, V, R))
    del X, T, Z, V, R
    s.close()
    rng = np.random.default_rng(5)
    cols = np.unique(np.r_[0, 1, nevex - 1, nevex, k - 1, rng.choice(k, 11, replace=False)])
    # QR: orthonormal sampled columns; X = Q R column by column, R upper
    # triangular with a positive real diagonal
    Gs = Qh[:, cols].conj().T @ Qh[:, cols]
    assert np.max(np.abs(Gs - np.eye(len(cols)))) < 1e-12
    assert np.all(np.abs(np.tril(Rh, -1)) == 0)
    dR = np.diag(Rh)
    assert np.all(dR.real > 0) and np.allclose(dR.imag, 0)
    xs = np.max(np.linalg.norm(X0, axis=0))
    for j in cols:
        rec = Qh[:, :j + 1] @ Rh[:j + 1, j]
        assert np.linalg.norm(rec - X0[:, j]) <= 1e-12 * xs
    del X0
    # T = H Q on sampled columns, from the host copies of A and B
    Ah, Bh = p.A.cpu().numpy(), p.B.cpu().numpy()

    def h_apply(Y):
        y1, y2 = Y[:m], Y[m:]
        return np.concatenate([Ah @ y1 + Bh @ y2, -np.conj(Bh @ y1.conj() + Ah @ y2.conj())])

    tc = cols[:4]
    HQ = h_apply(Qh[:, tc])
    assert np.max(np.abs(Th[:, tc] - HQ)) <= 1e-12 * np.max(np.abs(HQ))
    # Ritz values: ascending, positive, above the definiteness bound
    assert np.all(np.diff(ritz) >= 0) and ritz[0] >= lo * (1 - 1e-12)
    # Petrov-Galerkin condition, back-transform and residuals of sampled pairs
    jj = np.r_[0, nevex // 2, nevex - 1]
    Vs = Qh @ Zh[:, jj]
    Vs /= np.linalg.norm(Vs, axis=0)
    HV = h_apply(Vs)
    for t, j in enumerate(jj):
        z = Zh[:, j]
        r = Th @ z - ritz[j] * (Qh @ z)
        pg = Qh.conj().T @ apply_s(r[:, None])[:, 0]
        assert np.linalg.norm(pg) <= 1e-10 * np.linalg.norm(Th @ z)
        v = Vh[:, j]
        ph = np.vdot(Vs[:, t], v)
        assert abs(abs(ph) - 1) < 1e-12
        assert np.linalg.norm(v - Vs[:, t] * ph) < 1e-12
        rh = np.linalg.norm(HV[:, t] - ritz[j] * Vs[:, t])
        assert abs(res[j] - rh) <= 1e-8 * rh + 1e-12 * mu_n
    # eigenvalue adjoint on the positive Ritz pairs, sampled entries
    ga_ref, gb_ref = adjoint.eigval_grad_entries(Vh[:, :nev], g, rows, gcols)
    assert np.max(np.abs(ga - ga_ref)) <= 1e-11 * np.max(np.abs(ga_ref))
    assert np.max(np.abs(gb - gb_ref)) <= 1e-11 * np.max(np.abs(gb_ref))
