"""Full-size GPU checks of the larger workloads.

* adjoint workload (m = 2000): gradient of L = sum_i w_i lambda_i against the
  dense FP64 oracle gradient and against central finite differences
  (h = 1e-6) on 32 random unit-Frobenius Hermitian/symmetric directions;
* clustered (m = 16000) and largest (m = 30000) workloads: H X in c64 and
  c128 on sampled rows recomputed on the host from rows of A and B, and
  Thm 4.2 (K-conj equivariance of the filter) at full size.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from oracle import adjoint, dense
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


@pytest.mark.parametrize("cfg", [2, 4])
def test_apply_h_full_size_sampled_rows(cfg):
    p = config_problem_device(cfg)
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
