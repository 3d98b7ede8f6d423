// Host side of libchase_ph: handle, workspace, stage entry points and the
// outer loop of the pseudo-hermitian ChASE solver (Alg. 3).  Every numerical
// step is a kernel of this library; the host only sequences launches, keeps
// O(k) scalars (Ritz values, residuals, degrees, spectral estimates) and
// diagonalises the tiny Lanczos tridiagonals.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "common.h"
#include "dense.h"
#include "geev.h"
#include "vec.h"

using namespace chase;

struct chase_ph_s {
  chase_ph_params p{};
  const c128* A = nullptr;
  const c128* B = nullptr;
  int64_t ld = 0;
  hipStream_t st = nullptr;
  int64_t m = 0, n = 0;
  int nevex = 0, kmax = 0, kp = 0;
  // D = [A + B, i (A - B)] column-interleaved (m x 2m, ldd): the real
  // operand of every H X product, in c128 (D64) and, for the mixed / FP32
  // filter, in c64 (D32)
  c128* D64 = nullptr;
  c64* D32 = nullptr;
  int64_t ldd = 0;
  bool d64_ready = false;
  bool shadow_ready = false;
  // packed real coordinates of the H X operand (k-pair layout: yrows row
  // pairs of ldyr reals, in doubles; the c64 path uses it as floats)
  double* Yr = nullptr;
  int64_t ldyr = 0;
  int kcap = 0;    // columns the packed buffer holds (calls with more run in chunks)
  int64_t yrows = 0;
  // filter work buffers (n x nevex)
  c128* F1 = nullptr;
  c128* FT = nullptr;
  c64* W32 = nullptr;
  c64* F1_32 = nullptr;
  c64* FT_32 = nullptr;
  // residual-correction filter (mixed path)
  c128* Rv = nullptr;     // n x nevex unit-Ritz-vector residuals from the last RR
  c128* Rk = nullptr;     // same, in the column order of Wk
  c64* S32 = nullptr;     // n x nevex source (H + lambda) r
  c64* R32 = nullptr;     // n x nevex residuals in c64
  float* dcoef = nullptr; // per-step per-column source coefficients
  double* dpw = nullptr;  // per-column p_d(lambda^2)
  int coef_cap = 0;
  // QR / RR (n x kmax)
  c128* Xs = nullptr;
  c128* Xt = nullptr;
  c128* Tq = nullptr;
  c128* Vt = nullptr;
  c128* TZ = nullptr;
  // small padded (kp x kp)
  c128* G = nullptr;
  c128* L1 = nullptr;
  c128* L2 = nullptr;
  c128* L3 = nullptr;
  c128* Li = nullptr;
  c128* Nb = nullptr;
  c128* Tk = nullptr;
  c128* Ev = nullptr;
  c128* Ys = nullptr;
  c128* Zp = nullptr;  // kmax x kmax/2
  HouseholderWs hhw;   // Householder QR (last-resort orthonormalisation); Q in Xt
  GeevWs gw;           // general eigenproblem of the back-up Rayleigh quotient
  c128* Wev = nullptr; // kmax complex Ritz values of the back-up quotient
  // solver state
  c128* Ylock = nullptr;  // n x nev
  c128* Wk = nullptr;     // n x nevex
  double* dlam = nullptr;
  double* dres = nullptr;
  int* dperm = nullptr;
  // Lanczos (n x lanczos_vecs each)
  c128 *lv = nullptr, *lvp = nullptr, *lw = nullptr, *lr = nullptr, *lz = nullptr;
  double* dab = nullptr;  // 2 * steps * vecs
  void* ws = nullptr;
  size_t ws_bytes = 0;
  DenseWs dws;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double last_ms = 0;
  int last_launches = 0;
  int last_sweeps = 0;  // Jacobi sweeps of the last Alg. 2 Rayleigh-Ritz step
  bool qr_one_pass = false;  // the last qr_impl stopped after one Cholesky QR pass
  std::string err;
  bool dead = false;
  std::vector<void*> allocs;
  // apply_h launch profiling (chase_ph_profile)
  bool prof = false;
  std::vector<hipEvent_t> evpool;
  struct Launch {
    int prec, k;
    double flops, bytes;
  };
  std::vector<Launch> launches;
};

namespace {

constexpr double U_ROUND = 1.1102230246251565e-16;
// Largest deviation of Q^H Q from I after one Cholesky QR pass at which the
// solver skips the second pass (the Rayleigh-Ritz step uses Q^H Q = I).
constexpr double QR_ONE_PASS = 1e-13;
// Indefinite S H: a Ritz pair with residual above this fraction of
// |lambda~| is spurious and holds no place in the locking prefix.
constexpr double SPURIOUS_REL = 0.1;

chase_ph_status finish(chase_ph_t h, const Err& e) {
  if (e) {
    if (h) {
      h->err = e.msg;
      if (e.st == CHASE_PH_ERR_HIP) h->dead = true;
    }
    return e.st;
  }
  return CHASE_PH_OK;
}

template <typename T>
Err dalloc(chase_ph_t h, T** p, size_t count) {
  void* q = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) return fail(CHASE_PH_ERR_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
  h->allocs.push_back(q);
  *p = reinterpret_cast<T*>(q);
  return ok();
}

// Small host-to-device copy from pageable host memory; waits for it so the
// host buffer may be released right after.
Err h2d(chase_ph_t h, void* dst, const void* src, size_t bytes) {
  CHASE_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->st));
  CHASE_HIP(hipStreamSynchronize(h->st));
  return ok();
}

// Structure flags of gemm(): see ZgemmArgs.
constexpr int GEMM_LOWER_ONLY = 1, GEMM_A_LOWER = 2, GEMM_B_UPPER = 4, GEMM_REAL = 8;

Err gemm(chase_ph_t h, int ta, int tb, int64_t M, int64_t N, int64_t K, c128 alpha, const c128* A, int64_t lda,
         const c128* B, int64_t ldb, c128 beta, c128* C, int64_t ldc, int64_t kneg = -1, bool split = true,
         int flags = 0) {
  ZgemmArgs g{};
  g.lower_only = (flags & GEMM_LOWER_ONLY) != 0;
  g.a_lower = (flags & GEMM_A_LOWER) != 0;
  g.b_upper = (flags & GEMM_B_UPPER) != 0;
  g.real_data = (flags & GEMM_REAL) != 0;
  g.transA = ta; g.transB = tb;
  g.M = M; g.N = N; g.K = K;
  g.alpha = alpha; g.beta = beta;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.kneg = kneg < 0 ? K : kneg;
  g.batch = 1;
  return zgemm(g, split ? h->ws : nullptr, split ? h->ws_bytes : 0, h->st);
}

// D in c64 and the mixed path's work buffers.  alloc_shadow only
// allocates; ensure_shadow also builds D32 the first time a stage call
// needs it; the solver builds it again inside every timed solve
// (refresh_shadow), so a solve's time includes the conversion.  D64 is
// allocated at create and built the same way (refresh_d64, on first use and
// inside every solve).
Err alloc_shadow(chase_ph_t h) {
  if (h->D32) return ok();
  CHASE_TRY(dalloc(h, &h->D32, (size_t)h->ldd * 2 * h->m));
  CHASE_TRY(dalloc(h, &h->W32, (size_t)h->n * h->nevex));
  CHASE_TRY(dalloc(h, &h->F1_32, (size_t)h->n * h->nevex));
  CHASE_TRY(dalloc(h, &h->FT_32, (size_t)h->n * h->nevex));
  CHASE_TRY(dalloc(h, &h->Rv, (size_t)h->n * h->nevex));
  CHASE_TRY(dalloc(h, &h->Rk, (size_t)h->n * h->nevex));
  CHASE_TRY(dalloc(h, &h->S32, (size_t)h->n * h->nevex));
  CHASE_TRY(dalloc(h, &h->R32, (size_t)h->n * h->nevex));
  CHASE_TRY(dalloc(h, &h->dpw, (size_t)h->nevex));
  return ok();
}

Err refresh_shadow(chase_ph_t h) {
  CHASE_TRY(alloc_shadow(h));
  CHASE_TRY(make_d<c64>(h->A, h->p.tda ? nullptr : h->B, h->ld, h->p.a_conj, h->D32, h->ldd, h->m, h->st));
  h->shadow_ready = true;
  return ok();
}

Err ensure_shadow(chase_ph_t h) {
  if (h->shadow_ready) return ok();
  return refresh_shadow(h);
}

Err refresh_d64(chase_ph_t h) {
  CHASE_TRY(make_d<c128>(h->A, h->p.tda ? nullptr : h->B, h->ld, h->p.a_conj, h->D64, h->ldd, h->m, h->st));
  h->d64_ready = true;
  return ok();
}


constexpr size_t PROF_MAX = 65536;

Err prof_begin(chase_ph_t h) {
  if (!h->prof || h->launches.size() >= PROF_MAX) return ok();
  const size_t i = 2 * h->launches.size();
  while (h->evpool.size() < i + 2) {
    // timing only: no system-scope fence on record (which would write back
    // and invalidate the caches around every timed launch); the times are
    // read after the caller has synchronised the device
    hipEvent_t e;
    CHASE_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    h->evpool.push_back(e);
  }
  CHASE_HIP(hipEventRecord(h->evpool[i], h->st));
  return ok();
}

// Real flops of one H X product on k columns in the real formulation:
// 4 n^2 k (2 n^2 k on K-real columns).
inline double hx_flops(double n, int k, bool kreal) { return (kreal ? 2.0 : 4.0) * n * n * k; }

Err prof_end(chase_ph_t h, int prec, int k, size_t elem, bool has_p, bool has_q, bool kreal = false) {
  if (!h->prof || h->launches.size() >= PROF_MAX) return ok();
  const size_t i = 2 * h->launches.size();
  CHASE_HIP(hipEventRecord(h->evpool[i + 1], h->st));
  const double n = (double)h->n, m = (double)h->m;
  const double rows = h->p.tda ? m : n;  // vectors of m rows on a TDA handle
  const double bytes = (2.0 * m * m + (2.0 + (has_p ? 1 : 0) + (has_q ? 1 : 0)) * rows * k) * elem;
  h->launches.push_back({prec, k, hx_flops(n, k, kreal), bytes});
  return ok();
}

// Y = alpha H X + beta P + gamma Q on k columns
Err apply64(chase_ph_t h, int k, const c128* X, int64_t ldx, c128* Y, int64_t ldy, double alpha = 1,
            const c128* P = nullptr, int64_t ldp = 0, double beta = 0, const c128* Q = nullptr, int64_t ldq = 0,
            double gamma = 0, int kreal = 0) {
  ApplyHArgs<double> a{};
  a.D = h->D64; a.ldd = h->ldd; a.m = h->m; a.k = k;
  a.yr = h->Yr; a.ldyr = h->ldyr; a.yrows = h->yrows; a.kcap = h->kcap;
  if (k > 0 && !h->d64_ready) CHASE_TRY(refresh_d64(h));
  a.X = X; a.ldx = ldx; a.Y = Y; a.ldy = ldy; a.P = P; a.ldp = ldp; a.Q = Q; a.ldq = ldq;
  a.alpha = alpha; a.beta = beta; a.gamma = gamma; a.kreal = kreal; a.tda = h->p.tda;
  if (k <= 0) return ok();
  CHASE_TRY(prof_begin(h));
  CHASE_TRY(launch_apply_h_f64(a, h->ws, h->ws_bytes, h->st));
  return prof_end(h, CHASE_PH_FP64, k, sizeof(c128), P != nullptr, Q != nullptr, kreal != 0 || h->p.tda);
}

Err apply32(chase_ph_t h, int k, const c64* X, int64_t ldx, c64* Y, int64_t ldy, float alpha = 1,
            const c64* P = nullptr, int64_t ldp = 0, float beta = 0, const c64* Q = nullptr, int64_t ldq = 0,
            float gamma = 0, const c64* S = nullptr, int64_t lds = 0, const float* dcol = nullptr) {
  ApplyHArgs<float> a{};
  a.D = h->D32; a.ldd = h->ldd; a.m = h->m; a.k = k;
  a.yr = reinterpret_cast<float*>(h->Yr); a.ldyr = h->ldyr; a.yrows = h->yrows; a.kcap = h->kcap;
  if (k > 0 && !h->shadow_ready) CHASE_TRY(refresh_shadow(h));
  a.D = h->D32;
  a.X = X; a.ldx = ldx; a.Y = Y; a.ldy = ldy; a.P = P; a.ldp = ldp; a.Q = Q; a.ldq = ldq;
  a.alpha = alpha; a.beta = beta; a.gamma = gamma;
  a.S = S; a.lds = lds; a.dcol = dcol; a.tda = h->p.tda;
  if (k <= 0) return ok();
  CHASE_TRY(prof_begin(h));
  CHASE_TRY(launch_apply_h_f32(a, h->ws, h->ws_bytes, h->st));
  return prof_end(h, CHASE_PH_FP32, k, sizeof(c64), P != nullptr, Q != nullptr, h->p.tda != 0);
}

// Scaled Chebyshev recurrence on H^2 (eq. 4.1, Zhou-Saad scaling); see
// chase_ph_filter.  Buffers: W (user, ldw), F1 and FT (ld n).  W_s lives in
// W for even s and in F1 for odd s; the second product of each degree
// writes W_{s} in place over W_{s-2}.
template <typename R, typename C>
Err filter_impl(chase_ph_t h, int k, C* W, int64_t ldw, const std::vector<int>& d, double mu1, double mu_nevex,
                double mu_n, C* F1, C* FT, int* launches, double* flops) {
  const int64_t n = h->n;
  const double c = 0.5 * (mu_n * mu_n + mu_nevex * mu_nevex);
  const double e = 0.5 * (mu_n * mu_n - mu_nevex * mu_nevex);
  const double sigma1 = e / (mu1 * mu1 - c);
  double sigma = sigma1;
  const int maxd = d[k - 1];
  int j0 = 0;
  auto app = [&](int kc, const C* X, int64_t ldx, C* Y, int64_t ldy, double al, const C* P, int64_t ldp, double be,
                 const C* Q, int64_t ldq, double ga) -> Err {
    ++*launches;
    *flops += hx_flops((double)n, kc, false);
    if constexpr (sizeof(R) == 4)
      return apply32(h, kc, X, ldx, Y, ldy, (float)al, P, ldp, (float)be, Q, ldq, (float)ga);
    else
      return apply64(h, kc, X, ldx, Y, ldy, al, P, ldp, be, Q, ldq, ga);
  };
  for (int s = 1; s <= maxd; ++s) {
    while (j0 < k && d[j0] < s) ++j0;
    const int kc = k - j0;
    C* cur = ((s - 1) % 2 == 0) ? W + (int64_t)j0 * ldw : F1 + (int64_t)j0 * n;
    const int64_t ldc = ((s - 1) % 2 == 0) ? ldw : n;
    C* prev = ((s - 1) % 2 == 0) ? F1 + (int64_t)j0 * n : W + (int64_t)j0 * ldw;
    const int64_t ldpv = ((s - 1) % 2 == 0) ? n : ldw;
    C* T = FT + (int64_t)j0 * n;
    CHASE_TRY(app(kc, cur, ldc, T, n, 1.0, nullptr, 0, 0.0, nullptr, 0, 0.0));
    if (s == 1) {
      CHASE_TRY(app(kc, T, n, prev, ldpv, sigma1 / e, cur, ldc, -sigma1 * c / e, nullptr, 0, 0.0));
    } else {
      const double sn = 1.0 / (2.0 / sigma1 - sigma);
      CHASE_TRY(app(kc, T, n, prev, ldpv, 2.0 * sn / e, cur, ldc, -2.0 * sn * c / e, prev, ldpv, -sigma * sn));
      sigma = sn;
    }
  }
  // odd degrees ended in F1: copy those column groups back into W
  int j = 0;
  while (j < k) {
    int j2 = j;
    while (j2 < k && d[j2] == d[j]) ++j2;
    if (d[j] % 2 == 1) {
      CHASE_HIP(hipMemcpy2DAsync(W + (int64_t)j * ldw, ldw * sizeof(C), F1 + (int64_t)j * n, n * sizeof(C),
                                 n * sizeof(C), j2 - j, hipMemcpyDeviceToDevice, h->st));
    }
    j = j2;
  }
  return ok();
}

// p_d(H^2) v evaluated as p_d(lambda^2) v + D_d / e with the correction
// D_d = e [p_d(H^2) - p_d(lambda^2)] v built in c64 from the FP64 residual
// r = H v - lambda v of each unit Ritz vector (lambda its Ritz value):
//   s = (H + lambda) r = (H^2 - lambda^2) v,   D_1 = sigma_1 s,
//   D_{j+1} = (2 sigma_{j+1} / e)(H^2 - c) D_j - sigma_j sigma_{j+1} D_{j-1}
//             + 2 sigma_{j+1} p_j(lambda^2) s,
// with p_j(lambda^2) = T_j(tau)/T_j(t_0) from the same scaled recurrence
// (tau = (lambda^2 - c)/e).  This is the scaled Chebyshev filter of eq. 4.1
// rearranged exactly (divided differences of T_d); the c64 rounding error is
// relative to the correction, which shrinks with the residual, so the c64
// products carry the filter to FP64 accuracy.  Columns sorted by degree;
// W (c128, in place) holds the unit Ritz vectors, R (c128) their residuals.
Err filter_correction(chase_ph_t h, int k, c128* W, int64_t ldw, const c128* R, int64_t ldr,
                      const std::vector<double>& lam, const std::vector<int>& d, double mu1, double mu_nevex,
                      double mu_n, double* flops) {
  if (k == 0) return ok();
  const int64_t n = h->n;
  const double c = 0.5 * (mu_n * mu_n + mu_nevex * mu_nevex);
  const double e = 0.5 * (mu_n * mu_n - mu_nevex * mu_nevex);
  const double sigma1 = e / (mu1 * mu1 - c);
  const int maxd = d[k - 1];
  // host scalars: sigma_j, p_j(lambda_col^2), source coefficients
  std::vector<double> sig(maxd + 1, 0.0);
  sig[1] = sigma1;
  for (int j = 1; j < maxd; ++j) sig[j + 1] = 1.0 / (2.0 / sigma1 - sig[j]);
  const int rows = std::max(1, maxd - 1);
  std::vector<float> coef((size_t)(rows + 1) * k, 0.0f);
  std::vector<double> pw(k);
  for (int col = 0; col < k; ++col) {
    const double tau = (lam[col] * lam[col] - c) / e;
    double pprev = 1.0, pcur = sigma1 * tau;  // p_0, p_1
    for (int j = 1; j < d[col]; ++j) {
      coef[(size_t)(j - 1) * k + col] = (float)(2.0 * sig[j + 1] * pcur);
      const double pn = 2.0 * sig[j + 1] * tau * pcur - sig[j] * sig[j + 1] * pprev;
      pprev = pcur;
      pcur = pn;
    }
    pw[col] = pcur;
    coef[(size_t)rows * k + col] = (float)lam[col];  // row `rows`: lambda for s
  }
  if (h->coef_cap < (int)coef.size()) {
    CHASE_TRY(dalloc(h, &h->dcoef, coef.size()));
    h->coef_cap = (int)coef.size();
  }
  CHASE_TRY(h2d(h, h->dcoef, coef.data(), coef.size() * sizeof(float)));
  CHASE_TRY(h2d(h, h->dpw, pw.data(), k * sizeof(double)));
  CHASE_TRY(convert_to_c64(R, ldr, h->R32, n, n, k, h->st));
  auto count = [&](int kc) { *flops += hx_flops((double)n, kc, false); };
  // s = H r + lambda r
  CHASE_TRY(apply32(h, k, h->R32, n, h->S32, n, 1.0f, nullptr, 0, 0.0f, nullptr, 0, 0.0f, h->R32, n,
                    h->dcoef + (size_t)rows * k));
  count(k);
  c64* B0 = h->W32;   // D_j for even j
  c64* B1 = h->F1_32; // D_j for odd j
  c64* T = h->FT_32;
  CHASE_TRY(scale_c64(h->S32, n, B1, n, n, k, (float)sigma1, h->st));  // D_1
  int j0 = 0;
  for (int j = 1; j < maxd; ++j) {
    while (j0 < k && d[j0] < j + 1) ++j0;
    const int kc = k - j0;
    c64* cur = (j % 2 ? B1 : B0) + (int64_t)j0 * n;
    c64* prev = (j % 2 ? B0 : B1) + (int64_t)j0 * n;
    const double sn = sig[j + 1];
    CHASE_TRY(apply32(h, kc, cur, n, T + (int64_t)j0 * n, n));
    count(kc);
    CHASE_TRY(apply32(h, kc, T + (int64_t)j0 * n, n, prev, n, (float)(2.0 * sn / e), cur, n, (float)(-2.0 * sn * c / e),
                      j >= 2 ? prev : nullptr, n, (float)(-sig[j] * sn), h->S32 + (int64_t)j0 * n, n,
                      h->dcoef + (size_t)(j - 1) * k + j0));
    count(kc);
  }
  // odd final degrees ended in B1
  int j = 0;
  while (j < k) {
    int j2 = j;
    while (j2 < k && d[j2] == d[j]) ++j2;
    if (d[j] % 2 == 1)
      CHASE_HIP(hipMemcpy2DAsync(B0 + (int64_t)j * n, n * sizeof(c64), B1 + (int64_t)j * n, n * sizeof(c64),
                                 n * sizeof(c64), j2 - j, hipMemcpyDeviceToDevice, h->st));
    j = j2;
  }
  return combine_correction(W, ldw, B0, n, h->dpw, 1.0 / e, n, k, h->st);
}

Err check_filter_args(chase_ph_t h, int k, int64_t ldw, const int32_t* degs, double mu1, double mu_nevex, double mu_n,
                      std::vector<int>& d) {
  if (k < 0 || k > h->nevex) return fail(CHASE_PH_ERR_ARG, "filter: k out of range [0, nevex]");
  if (ldw < h->n) return fail(CHASE_PH_ERR_ARG, "filter: ldw < n");
  if (!(mu1 > 0) || !(mu_nevex > mu1) || !(mu_n > mu_nevex))
    return fail(CHASE_PH_ERR_ARG, "filter: need 0 < mu1 < mu_nevex < mu_n");
  d.assign(k, h->p.deg);
  if (degs)
    for (int i = 0; i < k; ++i) d[i] = degs[i];
  for (int i = 0; i < k; ++i) {
    if (d[i] < 1) return fail(CHASE_PH_ERR_ARG, "filter: degree < 1");
    if (i && d[i] < d[i - 1]) return fail(CHASE_PH_ERR_ARG, "filter: degrees must be non-decreasing");
  }
  return ok();
}

Err filter_any(chase_ph_t h, int k, void* dW, int64_t ldw, const std::vector<int>& d, double mu1, double mu_nevex,
               double mu_n, int prec, double* flops) {
  if (k == 0) return ok();
  int launches = 0;
  double fl = 0;
  CHASE_HIP(hipEventRecord(h->e0, h->st));
  if (prec == CHASE_PH_FP32) {
    CHASE_TRY(ensure_shadow(h));
    CHASE_TRY((filter_impl<float, c64>(h, k, (c64*)dW, ldw, d, mu1, mu_nevex, mu_n, h->F1_32, h->FT_32, &launches, &fl)));
  } else {
    CHASE_TRY((filter_impl<double, c128>(h, k, (c128*)dW, ldw, d, mu1, mu_nevex, mu_n, h->F1, h->FT, &launches, &fl)));
  }
  CHASE_HIP(hipEventRecord(h->e1, h->st));
  CHASE_HIP(hipEventSynchronize(h->e1));
  float ms = 0;
  CHASE_HIP(hipEventElapsedTime(&ms, h->e0, h->e1));
  h->last_ms = ms;
  h->last_launches = launches;
  if (flops) *flops = fl;
  return ok();
}

// One Cholesky-QR pass: Xout = Xin L^{-H} with L L^H = Xin^H Xin + shift I.
// real: Xin is real (held in c128), and so are the Gram matrix, L and Xout.
// Lower triangle of the Gram matrix X^H X in Lbuf (padded with I).
Err gram_lower(chase_ph_t h, int k, int kp, const c128* X, int64_t ldx, c128* Lbuf, bool real, int64_t nr) {
  CHASE_TRY(fill_padded(Lbuf, kp, k, 0.0, 1.0, true, h->st));
  return gemm(h, 1, 0, k, k, nr, {1, 0}, X, ldx, X, ldx, {0, 0}, Lbuf, kp, -1, true,
              GEMM_LOWER_ONLY | (real ? GEMM_REAL : 0));
}

Err cholqr_pass(chase_ph_t h, int k, int kp, const c128* Xin, int64_t ldin, c128* Xout, int64_t ldout, c128* Lbuf,
                double shift, bool* failed, bool real = false, int64_t rows = 0, bool gram_ready = false) {
  const int rf = real ? GEMM_REAL : 0;
  const int64_t nr = rows > 0 ? rows : h->n;
  // Gram matrix: the Cholesky reads its lower triangle only
  if (!gram_ready) CHASE_TRY(gram_lower(h, k, kp, Xin, ldin, Lbuf, real, nr));
  if (shift != 0.0) CHASE_TRY(add_diag(Lbuf, kp, k, shift, h->st));
  CHASE_TRY(cholesky_lower(Lbuf, kp, h->dws, h->st, failed));
  if (*failed) return ok();
  CHASE_TRY(tri_inverse_lower(Lbuf, h->Li, kp, h->dws, h->st));
  return gemm(h, 0, 1, nr, k, k, {1, 0}, Xin, ldin, h->Li, kp, {0, 0}, Xout, ldout, -1, true, GEMM_B_UPPER | rf);
}

// Householder QR of X in place; with npre = 2, X is the output of two
// Cholesky-QR passes with factors L1, L2 and R also takes L2^H L1^H.
Err householder_fallback(chase_ph_t h, int k, c128* X, int64_t ldx, c128* R, int64_t ldr, int npre,
                         int64_t rows = 0) {
  const int kp = pad64(k);
  CHASE_TRY(householder_qr(X, ldx, rows > 0 ? rows : h->n, k, R ? h->G : nullptr, kp, h->hhw, h->st));
  if (!R) return ok();
  if (npre == 0) {
    CHASE_HIP(hipMemcpy2DAsync(R, ldr * sizeof(c128), h->G, kp * sizeof(c128), k * sizeof(c128), k,
                               hipMemcpyDeviceToDevice, h->st));
    return ok();
  }
  CHASE_TRY(gemm(h, 0, 1, k, k, k, {1, 0}, h->G, kp, h->L2, kp, {0, 0}, h->Tk, kp, -1, false));
  return gemm(h, 0, 1, k, k, k, {1, 0}, h->Tk, kp, h->L1, kp, {0, 0}, R, ldr, -1, false);
}

// CholeskyQR2; shifted CholeskyQR3 when its first factorisation breaks
// down; Householder QR when a factorisation of either breaks down later
// (*used_shift = 0, 1, 2).  A pass that breaks down leaves X untouched, so
// the Householder QR runs on the input block or, after two completed
// passes of the shifted variant, on their output (same leading spans).
// With householder = false the breakdown is only reported (*used_shift = 2,
// X unspecified): the solver then orthonormalises the K-real form instead.
// rows: rows of X (0: n).
Err qr_impl(chase_ph_t h, int k, c128* X, int64_t ldx, c128* R, int64_t ldr, int* used_shift,
            bool householder = true, bool real = false, int64_t rows = 0) {
  if (used_shift) *used_shift = 0;
  h->qr_one_pass = false;
  if (k == 0) return ok();
  const int kp = pad64(k);
  const int64_t n = rows > 0 ? rows : h->n;
  bool failed = false;
  CHASE_TRY(cholqr_pass(h, k, kp, X, ldx, h->Xt, n, h->L1, 0.0, &failed, real, n));
  int nf = 2;
  if (!failed && !R) {
    // Section 2 chooses the orthonormalisation by condition number: when
    // the first pass already left Q^H Q within QR_ONE_PASS of I (a
    // well-conditioned block), the second pass is skipped
    CHASE_TRY(gram_lower(h, k, kp, h->Xt, n, h->L2, real, n));
    CHASE_TRY(gram_deviation(h->L2, kp, k, h->dres, h->dws.dscalar, h->st));
    double dev = 0;
    CHASE_TRY(d2h_small(&dev, h->dws.dscalar, sizeof(double), h->dws, h->st));
    if (dev <= QR_ONE_PASS) {
      h->qr_one_pass = true;
      CHASE_HIP(hipMemcpy2DAsync(X, ldx * sizeof(c128), h->Xt, n * sizeof(c128), n * sizeof(c128), k,
                                 hipMemcpyDeviceToDevice, h->st));
      return ok();
    }
    CHASE_TRY(cholqr_pass(h, k, kp, h->Xt, n, X, ldx, h->L2, 0.0, &failed, real, n, true));
    if (failed) {
      if (used_shift) *used_shift = 2;
      return householder ? householder_fallback(h, k, X, ldx, R, ldr, 0, n) : ok();
    }
  } else if (!failed) {
    CHASE_TRY(cholqr_pass(h, k, kp, h->Xt, n, X, ldx, h->L2, 0.0, &failed, real, n));
    if (failed) {
      if (used_shift) *used_shift = 2;
      return householder ? householder_fallback(h, k, X, ldx, R, ldr, 0, n) : ok();
    }
  } else {
    if (used_shift) *used_shift = 1;
    // shifted CholeskyQR3: s = 11 (n k + k (k + 1)) u ||X||_F^2
    CHASE_TRY(fill_padded(h->G, kp, k, 0.0, 1.0, true, h->st));
    CHASE_TRY(gemm(h, 1, 0, k, k, n, {1, 0}, X, ldx, X, ldx, {0, 0}, h->G, kp, -1, true,
                   GEMM_LOWER_ONLY | (real ? GEMM_REAL : 0)));
    CHASE_TRY(trace(h->G, kp, k, h->dws.dscalar, h->st));
    double fro2 = 0;
    CHASE_TRY(d2h_small(&fro2, h->dws.dscalar, sizeof(double), h->dws, h->st));
    const double shift = 11.0 * ((double)n * k + (double)k * (k + 1)) * U_ROUND * fro2;
    CHASE_TRY(cholqr_pass(h, k, kp, X, ldx, h->Xt, n, h->L1, shift, &failed, real, n));
    if (!failed) CHASE_TRY(cholqr_pass(h, k, kp, h->Xt, n, X, ldx, h->L2, 0.0, &failed, real, n));
    if (failed) {
      if (used_shift) *used_shift = 2;
      return householder ? householder_fallback(h, k, X, ldx, R, ldr, 0, n) : ok();
    }
    CHASE_TRY(cholqr_pass(h, k, kp, X, ldx, h->Xt, n, h->L3, 0.0, &failed, real, n));
    if (failed) {
      if (used_shift) *used_shift = 2;
      return householder ? householder_fallback(h, k, X, ldx, R, ldr, 2, n) : ok();
    }
    CHASE_HIP(hipMemcpy2DAsync(X, ldx * sizeof(c128), h->Xt, n * sizeof(c128), n * sizeof(c128), k,
                               hipMemcpyDeviceToDevice, h->st));
    nf = 3;
  }
  if (R) {
    // R = L_nf^H ... L_1^H
    if (nf == 2) {
      CHASE_TRY(gemm(h, 1, 1, k, k, k, {1, 0}, h->L2, kp, h->L1, kp, {0, 0}, R, ldr, -1, false));
    } else {
      CHASE_TRY(gemm(h, 1, 1, k, k, k, {1, 0}, h->L3, kp, h->L2, kp, {0, 0}, h->Tk, kp, -1, false));
      CHASE_TRY(gemm(h, 0, 1, k, k, k, {1, 0}, h->Tk, kp, h->L1, kp, {0, 0}, R, ldr, -1, false));
    }
  }
  return ok();
}

// Back-up Rayleigh quotient of Section 5.3 on Q and T = H Q; see
// chase_ph_oblique_rr_backup.  Buffers: P and then G in G, Q^H T in Tk,
// N and then N - D in Nb, D in dres, Schur vectors in Ev, eigenvectors of T
// in Li (transposed work copy in L3), eigenvectors of G in Ys.
Err rr_backup(chase_ph_t h, int k, const c128* Q, int64_t ldq, const c128* T, int64_t ldt, double* ritz, c128* Zpos,
              int64_t ldz) {
  const int kp = pad64(k);
  const int64_t m = h->m, n = h->n;
  CHASE_TRY(gemm(h, 1, 0, k, k, n, {1, 0}, Q, ldq, T, ldt, {0, 0}, h->G, kp, m));   // Q^H S H Q
  CHASE_TRY(gemm(h, 1, 0, k, k, n, {1, 0}, Q, ldq, T, ldt, {0, 0}, h->Tk, kp));     // Q^H H Q
  CHASE_TRY(gemm(h, 1, 0, k, k, n, {1, 0}, Q, ldq, Q, ldq, {0, 0}, h->Nb, kp, m));  // N = Q^H S Q
  CHASE_TRY(backup_diag(h->Nb, kp, k, BACKUP_DIAG_MIN, h->dres, h->st));            // D; Nb <- N - D
  CHASE_TRY(gemm(h, 0, 0, k, k, k, {-1, 0}, h->Nb, kp, h->Tk, kp, {1, 0}, h->G, kp, -1, false));
  CHASE_TRY(scale_rows_inv(h->G, kp, k, h->dres, h->st));                           // G = D^{-1} [...]
  int qs = 0;
  CHASE_TRY(nonsym_eig(h->G, h->Ev, kp, k, h->Wev, h->L3, h->Li, h->gw, h->st, &qs));
  if (qs != 0)
    return fail(CHASE_PH_ERR_SINGULAR_QSQ, "back-up Rayleigh quotient: QR iteration did not converge for k = " +
                                               std::to_string(k));
  CHASE_TRY(gemm(h, 0, 0, k, k, k, {1, 0}, h->Ev, kp, h->Li, kp, {0, 0}, h->Ys, kp, -1, false));  // Z Y
  CHASE_TRY(select_by_real_part(h->Wev, k, h->Ys, kp, h->dperm, h->dlam, Zpos, ldz, h->st));
  if (ritz) {
    CHASE_TRY(d2h_small(ritz, h->dlam, sizeof(double) * (k / 2), h->dws, h->st));
  }
  return ok();
}

// Oblique Rayleigh-Ritz with the dual basis of eq. 4.6 for any S H: the
// quotient of eq. 4.7, G = (Q^H S Q)^{-1} Q^H S H Q, by a general
// eigensolver (nothing factors Q^H S H Q, so S H may be indefinite; Section
// 5.3, last paragraph).  Q^H S Q = Q_N R (Householder QR), G = R^{-1} Q_N^H P
// with R^{-1} = ((R^H)^{-1})^H from the lower triangular inverse.  *singular
// is set (and nothing else done) when min |R_ii| <= 1e3 u max |R_ii|.
// T = H Q is given (n x k, ldt).
Err rr_general(chase_ph_t h, int k, const c128* Q, int64_t ldq, const c128* T, int64_t ldt, double* ritz, c128* Zpos,
               int64_t ldz, bool* singular) {
  const int kp = pad64(k);
  const int64_t m = h->m, n = h->n;
  *singular = false;
  CHASE_TRY(gemm(h, 1, 0, k, k, n, {1, 0}, Q, ldq, T, ldt, {0, 0}, h->G, kp, m));   // P = Q^H S H Q
  CHASE_TRY(gemm(h, 1, 0, k, k, n, {1, 0}, Q, ldq, Q, ldq, {0, 0}, h->Nb, kp, m));  // N = Q^H S Q
  CHASE_TRY(householder_qr(h->Nb, kp, k, k, h->L3, kp, h->hhw, h->st));            // N = Q_N R
  std::vector<c128> rdiag(k);
  CHASE_HIP(hipMemcpy2DAsync(rdiag.data(), sizeof(c128), h->L3, (kp + 1) * sizeof(c128), sizeof(c128), k,
                             hipMemcpyDeviceToHost, h->st));
  CHASE_HIP(hipStreamSynchronize(h->st));
  double rmin = 1e300, rmax = 0;
  for (const c128& z : rdiag) {
    const double a = std::hypot(z.re, z.im);
    rmin = std::min(rmin, a);
    rmax = std::max(rmax, a);
  }
  if (!(rmin > 1e3 * U_ROUND * rmax)) {
    *singular = true;
    return ok();
  }
  CHASE_TRY(gemm(h, 1, 0, k, k, k, {1, 0}, h->Nb, kp, h->G, kp, {0, 0}, h->Tk, kp));  // C = Q_N^H P
  CHASE_TRY(fill_padded(h->L1, kp, k, 0.0, 1.0, true, h->st));
  CHASE_TRY(conj_transpose(h->L3, kp, h->L1, kp, k, h->st));                        // R^H (lower)
  CHASE_TRY(tri_inverse_lower(h->L1, h->Li, kp, h->dws, h->st));                    // (R^H)^{-1}
  CHASE_TRY(gemm(h, 1, 0, k, k, k, {1, 0}, h->Li, kp, h->Tk, kp, {0, 0}, h->G, kp, -1, false));  // G = R^{-1} C
  int qs = 0;
  CHASE_TRY(nonsym_eig(h->G, h->Ev, kp, k, h->Wev, h->L3, h->Li, h->gw, h->st, &qs));
  if (qs != 0)
    return fail(CHASE_PH_ERR_SINGULAR_QSQ, "general Rayleigh quotient: QR iteration did not converge for k = " +
                                               std::to_string(k));
  CHASE_TRY(gemm(h, 0, 0, k, k, k, {1, 0}, h->Ev, kp, h->Li, kp, {0, 0}, h->Ys, kp, -1, false));  // Z Y
  CHASE_TRY(select_by_real_part(h->Wev, k, h->Ys, kp, h->dperm, h->dlam, Zpos, ldz, h->st));
  if (ritz) {
    CHASE_TRY(d2h_small(ritz, h->dlam, sizeof(double) * (k / 2), h->dws, h->st));
  }
  return ok();
}

// Alg. 2 (inverse Rayleigh quotient); see chase_ph_oblique_rr.
// backup: -1 never uses the back-up quotient of Section 5.3 (a singular
// Q^H S Q is reported), 0 uses it when Alg. 2 resolves fewer than k/2
// positive values, 1 always (*used_backup reports which ran); 2 runs the
// general quotient of eq. 4.7 instead of Alg. 2 (indefinite S H) and the
// back-up quotient when Q^H S Q is singular; 3 the general quotient only
// (a singular Q^H S Q is reported).
// kreal_q: every column of Q is K-real, so T = H Q takes half the products.
// In a K-real basis the quotient G below is i times a real antisymmetric
// matrix, whose zero diagonal slows the Jacobi sweeps down; the columns 2j
// and 2j + 1 of Q and T (the two K-real vectors of one pair) are therefore
// recombined as (q_2j +- i q_2j+1) / sqrt(2) (unitary: the Ritz pairs do not
// change), which gives G a nonzero diagonal.  Q is modified in place then.
Err rr_impl(chase_ph_t h, int k, const c128* Q, int64_t ldq, double* ritz, c128* Zpos, int64_t ldz, c128* T,
            int64_t ldt, bool kreal_q = false, int backup = -1, bool* used_backup = nullptr) {
  const int kp = pad64(k);
  const int64_t m = h->m, n = h->n;
  CHASE_TRY(apply64(h, k, Q, ldq, T, ldt, 1, nullptr, 0, 0, nullptr, 0, 0, kreal_q ? 1 : 0));  // T = H Q
  if (kreal_q) {
    CHASE_TRY(pair_mix(const_cast<c128*>(Q), ldq, n, k / 2, h->st));
    CHASE_TRY(pair_mix(T, ldt, n, k / 2, h->st));  // = H (Q after the mix)
  }
  if (used_backup) *used_backup = backup == 1;
  if (backup == 1) return rr_backup(h, k, Q, ldq, T, ldt, ritz, Zpos, ldz);
  if (backup == 2 || backup == 3) {
    bool singular = false;
    CHASE_TRY(rr_general(h, k, Q, ldq, T, ldt, ritz, Zpos, ldz, &singular));
    if (!singular) return ok();
    if (backup == 3) return fail(CHASE_PH_ERR_SINGULAR_QSQ, "general Rayleigh quotient: Q^H S Q numerically singular");
    if (used_backup) *used_backup = true;
    return rr_backup(h, k, Q, ldq, T, ldt, ritz, Zpos, ldz);
  }
  CHASE_TRY(fill_padded(h->G, kp, k, 0.0, 1.0, true, h->st));
  CHASE_TRY(gemm(h, 1, 0, k, k, n, {1, 0}, Q, ldq, T, ldt, {0, 0}, h->G, kp, m, true,
                 GEMM_LOWER_ONLY));  // M = Q^H S T (Hermitian; the Cholesky reads the lower triangle)
  bool failed = false;
  CHASE_TRY(cholesky_lower(h->G, kp, h->dws, h->st, &failed));                // L L^H = M
  if (failed) return fail(CHASE_PH_ERR_NOT_DEFINITE, "Cholesky of Q^H S H Q failed (SH not positive definite on range(Q))");
  CHASE_TRY(tri_inverse_lower(h->G, h->Li, kp, h->dws, h->st));
  CHASE_TRY(fill_padded(h->Nb, kp, k, 1.0, 0.0, true, h->st));              // N = I - 2 Q2^H Q2
  CHASE_TRY(gemm(h, 1, 0, k, k, m, {-2, 0}, Q + m, ldq, Q + m, ldq, {1, 0}, h->Nb, kp));
  CHASE_TRY(gemm(h, 0, 1, kp, kp, kp, {1, 0}, h->Nb, kp, h->Li, kp, {0, 0}, h->Tk, kp, -1, false,
                 GEMM_B_UPPER));  // N L^{-H}
  CHASE_TRY(gemm(h, 0, 0, kp, kp, kp, {1, 0}, h->Li, kp, h->Tk, kp, {0, 0}, h->G, kp, -1, false,
                 GEMM_A_LOWER));  // L^{-1} N L^{-H}
  int sweeps = 0;
  CHASE_TRY(jacobi_eigh(h->G, h->Ev, kp, h->dws, h->st, h->p.rr_max_sweeps, &sweeps));
  h->last_sweeps = sweeps;
  int npos = 0, nneg = 0;
  CHASE_TRY(select_positive(h->G, h->Ev, k, kp, h->Ys, h->dlam, h->dws, h->st, &npos, &nneg));
  if ((npos != k / 2 || nneg != k / 2) && backup == 0) {
    if (used_backup) *used_backup = true;
    return rr_backup(h, k, Q, ldq, T, ldt, ritz, Zpos, ldz);
  }
  if (npos != k / 2 || nneg != k / 2)
    return fail(CHASE_PH_ERR_SINGULAR_QSQ, "Q^H S Q numerically singular: " + std::to_string(npos) + " positive / " +
                                               std::to_string(nneg) + " negative resolved Ritz values for k = " +
                                               std::to_string(k));
  CHASE_TRY(gemm(h, 1, 0, k, k / 2, k, {1, 0}, h->Li, kp, h->Ys, kp, {0, 0}, Zpos, ldz, -1, false));  // Z = L^{-H} Y
  if (ritz) {
    CHASE_TRY(d2h_small(ritz, h->dlam, sizeof(double) * (k / 2), h->dws, h->st));
  }
  return ok();
}

Err resid_impl(chase_ph_t h, int k, int kk, const c128* Q, int64_t ldq, const c128* T, int64_t ldt, const c128* Zpos,
               int64_t ldz, const double* ritz_host, c128* V, int64_t ldv, double* resid, c128* Rout = nullptr) {
  if (kk == 0) return ok();
  const int64_t n = h->n;
  CHASE_TRY(gemm(h, 0, 0, n, kk, k, {1, 0}, Q, ldq, Zpos, ldz, {0, 0}, V, ldv, -1, false));
  CHASE_TRY(gemm(h, 0, 0, n, kk, k, {1, 0}, T, ldt, Zpos, ldz, {0, 0}, h->TZ, n, -1, false));
  if (ritz_host) CHASE_TRY(h2d(h, h->dlam, ritz_host, sizeof(double) * kk));
  CHASE_TRY(residual_norms(V, ldv, h->TZ, n, h->dlam, n, kk, h->dres, Rout, n, h->st));
  CHASE_TRY(d2h_small(resid, h->dres, sizeof(double) * kk, h->dws, h->st));
  return ok();
}

// Symmetric tridiagonal eigenproblem of Lanczos (tiny): cyclic Jacobi on
// the dense matrix; returns eigenvalues and the first and last rows of the
// eigenvector matrix.
void tridiag_eig(const std::vector<double>& a, const std::vector<double>& b, std::vector<double>& th,
                 std::vector<double>& first, std::vector<double>& last) {
  const int s = (int)a.size();
  std::vector<double> M(s * s, 0.0), V(s * s, 0.0);
  for (int i = 0; i < s; ++i) {
    M[i * s + i] = a[i];
    V[i * s + i] = 1.0;
    if (i + 1 < s) M[i * s + i + 1] = M[(i + 1) * s + i] = b[i];
  }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j) {
        tot += M[i * s + j] * M[i * s + j];
        if (i != j) off += M[i * s + j] * M[i * s + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < s; ++p)
      for (int q = p + 1; q < s; ++q) {
        const double apq = M[p * s + q];
        if (apq == 0.0) continue;
        const double tau = (M[q * s + q] - M[p * s + p]) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        for (int r = 0; r < s; ++r) {  // columns
          const double mp = M[r * s + p], mq = M[r * s + q];
          M[r * s + p] = c * mp - sn * mq;
          M[r * s + q] = sn * mp + c * mq;
        }
        for (int r = 0; r < s; ++r) {  // rows
          const double mp = M[p * s + r], mq = M[q * s + r];
          M[p * s + r] = c * mp - sn * mq;
          M[q * s + r] = sn * mp + c * mq;
        }
        for (int r = 0; r < s; ++r) {
          const double vp = V[r * s + p], vq = V[r * s + q];
          V[r * s + p] = c * vp - sn * vq;
          V[r * s + q] = sn * vp + c * vq;
        }
      }
  }
  th.resize(s);
  first.resize(s);
  last.resize(s);
  for (int i = 0; i < s; ++i) {
    th[i] = M[i * s + i];
    first[i] = V[0 * s + i];
    last[i] = V[(s - 1) * s + i];
  }
}

// Spectral estimates mu_1, mu_nevex, mu_n (Section 4.1) from Lanczos runs,
// one product with H per step; start vectors are the gamma-scaled caller
// draws.  Definite S H: Lanczos on H in the S H inner product,
//   w = H v, alpha = w^H S w, r = w - alpha v - beta v_prev, z = H r,
//   beta^2 = r^H S z, v <- r / beta, w <- z / beta;
// mu_nevex is the quantile nevex / m of the density on the positive axis.
// Indefinite S H (the S H inner product is then indefinite): Hermitian
// Lanczos on S H in the Euclidean inner product, the same recurrence with
// w = S H v, alpha = v^H w, z = S H r and beta^2 = r^H r; the |theta| are
// the singular values of H, mu_nevex is their quantile nevex / m on the
// folded axis.
// The Lanczos recurrence, one product per step, on nv = lanczos_vecs runs
// at once over `rows`-row vectors whose starts are in lv (ld rows):
//   w = op(v), alpha = <w, w> or <v, w>, r = w - alpha v - beta v_prev,
//   z = op(r), beta^2 = <r, z> or <r, r>, v <- r / beta, w <- z / beta
// (first forms with sh_inner, the S H inner product where op = H; second
// forms for a Hermitian op in the Euclidean product).  Returns alpha and
// beta^2 of every run and step on the host ([j * nv + r]).
template <typename Op, typename Dots>
Err lanczos_recurrence(chase_ph_t h, int64_t rows, bool sh_inner, Op op, Dots dots, std::vector<double>& ha,
                       std::vector<double>& hb) {
  const int nv = h->p.lanczos_vecs, steps = h->p.lanczos_steps;
  double* alpha = h->dab;
  double* bsq = h->dab + (size_t)steps * nv;
  double* b0 = h->dab + (size_t)2 * steps * nv;
  CHASE_HIP(hipMemsetAsync(h->lvp, 0, sizeof(c128) * rows * nv, h->st));
  CHASE_TRY(op(h->lv, h->lw));
  CHASE_TRY(dots(h->lv, sh_inner ? h->lw : h->lv, b0));
  CHASE_TRY(lanczos_advance(h->lvp, h->lv, h->lw, h->lv, h->lw, rows, rows, nv, b0, false, h->st));
  for (int j = 0; j < steps; ++j) {
    CHASE_TRY(dots(sh_inner ? h->lw : h->lv, h->lw, alpha + (size_t)j * nv));
    CHASE_TRY(lanczos_residual(h->lw, h->lv, h->lvp, h->lr, rows, rows, nv, alpha + (size_t)j * nv,
                               j ? bsq + (size_t)(j - 1) * nv : nullptr, h->st));
    CHASE_TRY(op(h->lr, h->lz));
    CHASE_TRY(dots(h->lr, sh_inner ? h->lz : h->lr, bsq + (size_t)j * nv));
    if (j + 1 < steps)
      CHASE_TRY(lanczos_advance(h->lvp, h->lv, h->lw, h->lr, h->lz, rows, rows, nv, bsq + (size_t)j * nv, true, h->st));
  }
  ha.assign((size_t)steps * nv, 0.0);
  hb.assign((size_t)steps * nv, 0.0);
  CHASE_HIP(hipMemcpyAsync(ha.data(), alpha, sizeof(double) * ha.size(), hipMemcpyDeviceToHost, h->st));
  CHASE_HIP(hipMemcpyAsync(hb.data(), bsq, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, h->st));
  CHASE_HIP(hipStreamSynchronize(h->st));
  return ok();
}

Err lanczos_impl(chase_ph_t h, const c128* dLz, int64_t ldlz, double* mu1, double* mu_nevex, double* mu_n) {
  const int nv = h->p.lanczos_vecs, steps = h->p.lanczos_steps;
  const int64_t n = h->n, m = h->m;
  const bool definite = h->p.definite != 0;
  // Y = (S) H X for the indefinite recurrence's sign flip
  auto op = [&](const c128* X, c128* Y) -> Err {
    CHASE_TRY(apply64(h, nv, X, n, Y, n));
    if (!definite) CHASE_TRY(scale_lower_half(Y, n, Y, n, m, nv, -1.0, h->st));
    return ok();
  };
  auto dots = [&](const c128* X, const c128* Y, double* out) -> Err {
    return definite ? s_dots(X, n, Y, n, m, nv, out, h->st) : plain_dots(X, n, Y, n, m, nv, out, h->st);
  };
  CHASE_TRY(scale_lower_half(dLz, ldlz, h->lv, n, m, nv, h->p.gamma, h->st));
  std::vector<double> ha, hb;
  CHASE_TRY(lanczos_recurrence(h, n, definite, op, dots, ha, hb));
  double m1 = 1e300, mn = 0;
  std::vector<std::pair<double, double>> pos;  // (theta, weight)
  for (int r = 0; r < nv; ++r) {
    std::vector<double> a(steps), b(steps);
    for (int j = 0; j < steps; ++j) {
      a[j] = ha[(size_t)j * nv + r];
      b[j] = std::sqrt(std::max(hb[(size_t)j * nv + r], 0.0));
    }
    std::vector<double> th, f, l;
    tridiag_eig(a, b, th, f, l);
    int imax = 0;
    for (int i = 0; i < steps; ++i) {
      m1 = std::min(m1, std::fabs(th[i]));
      if (std::fabs(th[i]) > std::fabs(th[imax])) imax = i;
    }
    mn = std::max(mn, std::fabs(th[imax]) + std::fabs(b[steps - 1] * l[imax]));
    for (int i = 0; i < steps; ++i) {
      if (definite && th[i] > 0) pos.push_back({th[i], f[i] * f[i] / nv});
      if (!definite) pos.push_back({std::fabs(th[i]), f[i] * f[i] / nv});
    }
  }
  std::sort(pos.begin(), pos.end());
  double tot = 0;
  for (auto& pw : pos) tot += pw.second;
  double cum = 0, mnev = pos.empty() ? 0.5 * (m1 + mn) : pos.back().first;
  const double target = (double)h->nevex / (double)h->m;
  for (auto& pw : pos) {
    cum += pw.second / tot;
    if (cum >= target) {
      mnev = pw.first;
      break;
    }
  }
  if (mnev <= m1) {
    mnev = 0.5 * (m1 + mn);
    for (auto& pw : pos)
      if (pw.first > m1 * (1.0 + 1e-8)) {
        mnev = pw.first;
        break;
      }
  }
  mnev = std::min(mnev, 0.99 * mn);
  *mu1 = m1;
  *mu_nevex = mnev;
  *mu_n = mn;
  return ok();
}

// ---------------------------------------------------------------- TDA
// Hermitian ChASE on A alone (Alg. 1; B = 0 in Section 1.1).  The H X
// kernels run on D = [A, i A] and give A X on m-row columns.

// Lanczos density of A: Ritz values of every run with Gauss weights
// |first eigenvector component|^2 / runs, ascending, plus the upper bound
// mu_m = max over runs of (largest Ritz value + |beta_last z_last|).
struct TdaDensity {
  std::vector<std::pair<double, double>> tw;  // (theta, weight), ascending theta
  double mu1 = 0, mu_m = 0;
};

Err tda_lanczos(chase_ph_t h, const c128* dLz, int64_t ldlz, TdaDensity* d) {
  const int nv = h->p.lanczos_vecs, steps = h->p.lanczos_steps;
  const int64_t m = h->m;
  auto op = [&](const c128* X, c128* Y) -> Err { return apply64(h, nv, X, m, Y, m); };
  auto dots = [&](const c128* X, const c128* Y, double* out) -> Err {
    return row_dots(X, m, Y, m, m, nv, out, h->st);
  };
  CHASE_HIP(hipMemcpy2DAsync(h->lv, m * sizeof(c128), dLz, ldlz * sizeof(c128), m * sizeof(c128), nv,
                             hipMemcpyDeviceToDevice, h->st));
  std::vector<double> ha, hb;
  CHASE_TRY(lanczos_recurrence(h, m, false, op, dots, ha, hb));
  d->tw.clear();
  d->mu_m = -1e300;
  for (int r = 0; r < nv; ++r) {
    std::vector<double> a(steps), b(steps);
    for (int j = 0; j < steps; ++j) {
      a[j] = ha[(size_t)j * nv + r];
      b[j] = std::sqrt(std::max(hb[(size_t)j * nv + r], 0.0));
    }
    std::vector<double> th, f, l;
    tridiag_eig(a, b, th, f, l);
    int imax = 0;
    for (int i = 1; i < steps; ++i)
      if (th[i] > th[imax]) imax = i;
    d->mu_m = std::max(d->mu_m, th[imax] + std::fabs(b[steps - 1] * l[imax]));
    for (int i = 0; i < steps; ++i) d->tw.push_back({th[i], f[i] * f[i] / nv});
  }
  std::sort(d->tw.begin(), d->tw.end());
  d->mu1 = d->tw.front().first;
  return ok();
}

// Smallest Ritz value at which the weight accumulated from the left end
// reaches frac of the total.
double tda_quantile(const TdaDensity& d, double frac) {
  double tot = 0;
  for (const auto& p : d.tw) tot += p.second;
  double cum = 0;
  for (const auto& p : d.tw) {
    cum += p.second;
    if (cum / tot >= frac) return p.first;
  }
  return d.tw.back().first;
}

// mu_nevex of Alg. 1: the density quantile nevex / m, moved off mu_1 and
// kept 1% of the interval below mu_m.
double tda_mu_nevex(const TdaDensity& d, int nevex, int64_t m) {
  double q = tda_quantile(d, (double)nevex / (double)m);
  if (q <= d.mu1) {
    q = 0.5 * (d.mu1 + d.mu_m);
    const double lim = d.mu1 + 1e-8 * std::max(1.0, std::fabs(d.mu1));
    for (const auto& p : d.tw)
      if (p.first > lim) {
        q = p.first;
        break;
      }
  }
  return std::min(q, d.mu_m - 0.01 * (d.mu_m - d.mu1));
}

// Automatic nex: per candidate, omega_nev and omega_nevex are density
// quantiles; the filter on [omega_nevex, mu_m] reduces the nev-th pair by
// 1 / |T_deg(t)|, t = |omega_nev - c| / e, per iteration; the iterations
// to take a residual of mu_m - mu_1 to tol times (nev + nex) is the filter
// work, minimised over the candidates (the first of equal costs).
int tda_auto_nex(const TdaDensity& d, int64_t m, int nev, int deg, double tol, const std::vector<int>& cands) {
  int best = -1;
  double best_cost = 0;
  for (int nex : cands) {
    const double om_nev = tda_quantile(d, (double)nev / (double)m);
    const double om_nevex = tda_quantile(d, (double)(nev + nex) / (double)m);
    if (om_nevex <= om_nev || om_nevex >= d.mu_m) continue;
    const double c = 0.5 * (d.mu_m + om_nevex), e = 0.5 * (d.mu_m - om_nevex);
    const double t = std::fabs((om_nev - c) / e);
    const double rho = t + std::sqrt(t * t - 1.0);
    const double factor = 2.0 / (std::pow(rho, deg) + std::pow(rho, -deg));
    const double its = std::ceil(std::log(tol / (d.mu_m - d.mu1)) / std::log(factor));
    const double cost = its * (nev + nex);
    if (best < 0 || cost < best_cost) {
      best = nex;
      best_cost = cost;
    }
  }
  return best < 0 ? cands.back() : best;
}

// Candidates of the automatic nex: ceil(j nex_max / 8), j = 1..8, distinct.
std::vector<int> tda_nex_candidates(int nex_max) {
  std::vector<int> c;
  for (int j = 1; j <= 8; ++j) {
    const int v = (int)ceil_div((int64_t)j * nex_max, 8);
    if (v >= 1 && (c.empty() || v != c.back())) c.push_back(v);
  }
  return c;
}

// In place W <- p_deg(A) W (m x k, ldw): the scaled Chebyshev recurrence of
// eq. 2.1 on [mu_nevex, mu_m], normalised at mu_1,
//   W_1 = (sigma_1 / e)(A - c) W_0,
//   W_{s+1} = (2 sigma_{s+1} / e)(A - c) W_s - sigma_s sigma_{s+1} W_{s-1},
// one H X call (TDA mode) per degree with the update fused; W_s alternates
// between W and F1 (ld m).
Err filter_tda(chase_ph_t h, int k, c128* W, int64_t ldw, int deg, double mu1, double mu_nevex, double mu_m,
               double* flops) {
  if (k == 0) return ok();
  const int64_t m = h->m;
  const double c = 0.5 * (mu_m + mu_nevex), e = 0.5 * (mu_m - mu_nevex);
  const double s1 = e / (mu1 - c);
  c128* cur = h->F1;
  int64_t ldc = m;
  c128* prev = W;
  int64_t ldp = ldw;
  CHASE_TRY(apply64(h, k, W, ldw, h->F1, m, s1 / e, W, ldw, -s1 * c / e));
  double sigma = s1;
  for (int s = 1; s < deg; ++s) {
    const double sn = 1.0 / (2.0 / s1 - sigma);
    CHASE_TRY(apply64(h, k, cur, ldc, prev, ldp, 2.0 * sn / e, cur, ldc, -2.0 * sn * c / e, prev, ldp, -sigma * sn));
    std::swap(cur, prev);
    std::swap(ldc, ldp);
    sigma = sn;
  }
  if (cur != W)
    CHASE_HIP(hipMemcpy2DAsync(W, ldw * sizeof(c128), cur, ldc * sizeof(c128), m * sizeof(c128), k,
                               hipMemcpyDeviceToDevice, h->st));
  *flops += deg * hx_flops((double)h->n, k, true);
  return ok();
}

// Phase timer on its own event pair (the stage calls it brackets record
// the handle's e0/e1 for chase_ph_last_timing).
struct Timer {
  chase_ph_t h;
  hipEvent_t a = nullptr, b = nullptr;
  explicit Timer(chase_ph_t hh) : h(hh) {}
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  Err start() {
    if (!a) {
      CHASE_HIP(hipEventCreate(&a));
      CHASE_HIP(hipEventCreate(&b));
    }
    CHASE_HIP(hipEventRecord(a, h->st));
    return ok();
  }
  Err stop(double* acc) {
    CHASE_HIP(hipEventRecord(b, h->st));
    CHASE_HIP(hipEventSynchronize(b));
    float ms = 0;
    CHASE_HIP(hipEventElapsedTime(&ms, a, b));
    *acc += ms * 1e-3;
    return ok();
  }
};

Err solve_impl(chase_ph_t h, const c128* W0, int64_t ldw0, const c128* Lz, int64_t ldlz, double* evals, c128* V,
               int64_t ldv, double* resid_out, chase_ph_info* info, bool* converged) {
  const chase_ph_params& p = h->p;
  const int64_t n = h->n, m = h->m;
  const int nev = p.nev, nevex = h->nevex;
  chase_ph_info inf{};
  if (info) {
    inf.resid_history = info->resid_history;
    inf.resid_history_len = info->resid_history_len;
  }
  inf.switch_iter = -1;
  Timer tm(h);
  hipEvent_t t0, t1;
  CHASE_HIP(hipEventCreate(&t0));
  CHASE_HIP(hipEventCreate(&t1));
  CHASE_HIP(hipEventRecord(t0, h->st));

  CHASE_TRY(refresh_d64(h));  // the real operand D of every c128 H X product, inside the timed solve
  CHASE_TRY(scale_lower_half(W0, ldw0, h->Wk, n, m, nevex, p.gamma, h->st));  // Alg. 3, line 1 / Section 4.6
  double mu1, mu_nevex, mu_n;
  CHASE_TRY(tm.start());
  CHASE_TRY(lanczos_impl(h, Lz, ldlz, &mu1, &mu_nevex, &mu_n));
  CHASE_TRY(tm.stop(&inf.t_lanczos));
  inf.mu1 = mu1;
  inf.mu_nevex0 = mu_nevex;
  inf.mu_n = mu_n;
  const bool verbose = std::getenv("CHASE_PH_VERBOSE") != nullptr;
  if (verbose) std::fprintf(stderr, "[chase_ph] lanczos mu1=%.6g mu_nevex=%.6g mu_n=%.6g\n", mu1, mu_nevex, mu_n);
  if (!std::isfinite(mu1) || !std::isfinite(mu_n) || !std::isfinite(mu_nevex) || !(mu1 > 0) || !(mu_nevex > mu1) ||
      !(mu_n > mu_nevex))
    return fail(CHASE_PH_ERR_NOT_DEFINITE, "Lanczos spectral estimates invalid (SH not positive definite?)");
  const bool mixed = p.precision == CHASE_PH_MIXED;
  const bool definite = p.definite != 0;
  if (mixed) CHASE_TRY(refresh_shadow(h));

  int locked = 0;
  int lq = 0;  // locked pairs whose basis columns are in Xs[:, 0 : 2 lq]
  std::vector<double> lam_locked, res_locked;
  std::vector<int> degs(nevex, p.deg);
  std::vector<double> ritz(nevex), res(nevex);
  // Filter mode per Ritz pair (ascending order of the current search
  // block): 0 = c128, 1 = c64 residual correction, 2 = plain c64.  The FP64
  // path uses mode 0 throughout.  The mixed path starts in mode 2 (no Ritz
  // pairs yet), moves every pair to mode 1 once it has a Ritz value and an
  // FP64 residual (above switch_tol > 0 a pair stays in mode 2), and moves a
  // pair to mode 0 only if its residual stagnates close to tol.
  std::vector<char> mode(nevex, mixed ? 2 : 0);
  std::vector<double> prev_res(nevex, 1e300), lamcol(nevex, 0.0);
  int g0 = mixed ? 0 : nevex, g1 = 0;  // W columns: [mode 0 | mode 1 | mode 2]
  int hist_pos = 0;
  *converged = false;
  for (int it = 0; it < p.max_iter; ++it) {
    const int kw = nevex - locked;
    double fl = 0;
    CHASE_TRY(tm.start());
    if (g0 > 0) {
      std::vector<int> d0(degs.begin(), degs.begin() + g0);
      CHASE_TRY(filter_any(h, g0, h->Wk, n, d0, mu1, mu_nevex, mu_n, CHASE_PH_FP64, &fl));
      inf.filter_flops += fl;
      if (inf.switch_iter < 0 && mixed) inf.switch_iter = it;
    }
    if (g1 > 0) {
      fl = 0;
      std::vector<int> d1(degs.begin() + g0, degs.begin() + g0 + g1);
      std::vector<double> l1(lamcol.begin() + g0, lamcol.begin() + g0 + g1);
      CHASE_TRY(filter_correction(h, g1, h->Wk + (int64_t)g0 * n, n, h->Rk + (int64_t)g0 * n, n, l1, d1, mu1,
                                  mu_nevex, mu_n, &fl));
      inf.filter_flops_fp32 += fl;
      inf.filter_flops += fl;
    }
    if (g0 + g1 < kw) {
      const int c0 = g0 + g1, k32 = kw - c0;
      fl = 0;
      std::vector<int> d2(degs.begin() + c0, degs.begin() + kw);
      CHASE_TRY(convert_to_c64(h->Wk + (int64_t)c0 * n, n, h->W32, n, n, k32, h->st));
      CHASE_TRY(filter_any(h, k32, h->W32, n, d2, mu1, mu_nevex, mu_n, CHASE_PH_FP32, &fl));
      CHASE_TRY(convert_to_c128(h->W32, n, h->Wk + (int64_t)c0 * n, n, n, k32, h->st));
      inf.filter_flops_fp32 += fl;
      inf.filter_flops += fl;
    }
    CHASE_TRY(tm.stop(&inf.t_filter));
    // assemble [S Y+, S K conj(Y+), W+, K conj(W+)] and orthonormalise
    // (eq. 4.5).  The columns of the locked pairs (Y+ locked) keep their
    // orthonormal basis in the first 2 lq columns of Xs from the iteration
    // they were locked in; only the pairs locked since then and the
    // unlocked block are built, projected off that basis (block
    // Gram-Schmidt, twice) and orthonormalised.  The basis of the unlocked
    // part, which the Rayleigh-Ritz step uses, spans the same space as a QR
    // of the whole block would give.
    CHASE_TRY(tm.start());
    const int ln = locked - lq;
    c128* Xn = h->Xs + (int64_t)2 * lq * n;
    const int kxn = 2 * ln + 2 * kw;
    const double qr_flops = 16.0 * n * (double)kxn * kxn + 64.0 * n * (double)lq * kxn;
    // The basis is built from K-real vectors: each pair (x, J x) of the
    // block, J x = K conj(x), is replaced by u = (x + J x) / 2 and
    // v = (x - J x) / (2i), which span the same space and are K-real, and
    // the projection and the Cholesky QR run on their real coordinates
    // (inner products of K-real vectors are real).  The orthonormal basis
    // is then K-real too, so H Q takes half the products (H [a; conj(a)] =
    // [t; -conj(t)], t = [A B] [a; conj(a)]) and the span is the one the
    // complex block would give.  The coordinates go to Tq (free until the
    // Rayleigh-Ritz step), the pair of each generator in adjacent columns;
    // those of the locked basis, for the projection, to Xt.
    CHASE_TRY(kreal_build(h->Ylock + (int64_t)lq * n, n, ln, h->Wk, n, kw, h->Tq, n, m, h->st));
    if (lq > 0) {
      CHASE_TRY(kreal_coords(h->Xs, n, m, 2 * lq, h->Xt, n, h->st));
      for (int pass = 0; pass < 2; ++pass) {
        CHASE_TRY(gemm(h, 1, 0, 2 * lq, kxn, n, {1, 0}, h->Xt, n, h->Tq, n, {0, 0}, h->G, h->kp, -1, true,
                       GEMM_REAL));  // C = Qp^T X
        CHASE_TRY(gemm(h, 0, 0, n, kxn, 2 * lq, {-1, 0}, h->Xt, n, h->G, h->kp, {1, 0}, h->Tq, n, -1, true,
                       GEMM_REAL));  // X -= Qp C
      }
    }
    int used = 0;
    CHASE_TRY(qr_impl(h, kxn, h->Tq, n, nullptr, 0, &used, false, true));
    if (used != 2) {
      CHASE_TRY(kreal_unpack(h->Tq, n, m, kxn, h->st));
      CHASE_HIP(hipMemcpy2DAsync(Xn, n * sizeof(c128), h->Tq, n * sizeof(c128), n * sizeof(c128), kxn,
                                 hipMemcpyDeviceToDevice, h->st));
    }
    if (used == 2) {
      // Numerically rank-deficient block: Householder QR of the real
      // coordinates of the K-real parts of all pairs, locked ones first, so
      // that the locked span keeps its leading columns.  Its completion
      // directions would be K-real, hence S-neutral, which leaves Q^H S Q
      // nearly singular and slows the oblique Rayleigh-Ritz down; so every
      // unlocked pair whose coordinates R shows dependent (|R_jj| <= 1e3 u
      // max |R_ii|) gets the coordinates of the unit vectors e_r and
      // i e_r in the top half (the S-definite pair [e_r; 0], [0; e_r] once
      // recombined, Section 4.6), and the QR is repeated.
      const int kall = 2 * locked + 2 * kw;
      CHASE_TRY(kreal_build(h->Ylock, n, locked, h->Wk, n, kw, h->Xs, n, m, h->st));
      CHASE_TRY(householder_qr(h->Xs, n, n, kall, h->G, h->kp, h->hhw, h->st));
      std::vector<c128> rdiag(kall);
      CHASE_HIP(hipMemcpy2DAsync(rdiag.data(), sizeof(c128), h->G, (h->kp + 1) * sizeof(c128), sizeof(c128), kall,
                                 hipMemcpyDeviceToHost, h->st));
      CHASE_HIP(hipStreamSynchronize(h->st));
      double rmax = 0;
      for (const c128& z : rdiag) rmax = std::max(rmax, std::fabs(z.re));
      std::vector<int> refill;
      for (int q = locked; q < locked + kw; ++q)
        if (std::fabs(rdiag[2 * q].re) <= 1e3 * U_ROUND * rmax || std::fabs(rdiag[2 * q + 1].re) <= 1e3 * U_ROUND * rmax)
          refill.push_back(q);
      if (!refill.empty()) {
        CHASE_TRY(kreal_build(h->Ylock, n, locked, h->Wk, n, kw, h->Xs, n, m, h->st));
        for (size_t t = 0; t < refill.size(); ++t) {
          const int64_t r = ((int64_t)refill[t] * 7919) % m;
          CHASE_TRY(unit_column(h->Xs + (int64_t)2 * refill[t] * n, n, r, h->st));
          CHASE_TRY(unit_column(h->Xs + (int64_t)(2 * refill[t] + 1) * n, n, m + r, h->st));
        }
        CHASE_TRY(householder_qr(h->Xs, n, n, kall, nullptr, 0, h->hhw, h->st));
      }
      CHASE_TRY(kreal_unpack(h->Xs, n, m, kall, h->st));
    }
    lq = locked;
    inf.shifted_qr_used += used == 1;
    inf.householder_qr_used += used == 2;
    inf.qr_one_pass += h->qr_one_pass;
    CHASE_TRY(tm.stop(&inf.t_qr));
    // oblique RR on the non-locked part (Alg. 2)
    const c128* Q = h->Xs + (int64_t)2 * locked * n;
    const int kq = 2 * kw;
    CHASE_TRY(tm.start());
    bool used_backup = false;
    const int rr_mode = p.rr_backup ? 1 : (definite ? 0 : 2);
    h->last_sweeps = 0;
    CHASE_TRY(rr_impl(h, kq, Q, n, ritz.data(), h->Zp, h->kmax, h->Tq, n, true, rr_mode, &used_backup));
    inf.rr_sweeps_max = std::max(inf.rr_sweeps_max, h->last_sweeps);
    inf.backup_rr_used += used_backup;
    inf.general_rr_used += rr_mode == 2 && !used_backup;
    CHASE_TRY(tm.stop(&inf.t_rr));
    // half back-transform and residuals (Section 4.5)
    CHASE_TRY(tm.start());
    CHASE_TRY(resid_impl(h, kq, kw, Q, n, h->Tq, n, h->Zp, h->kmax, nullptr, h->Vt, n, res.data(),
                         mixed ? h->Rv : nullptr));
    CHASE_TRY(tm.stop(&inf.t_resid));
    inf.rr_flops += hx_flops((double)n, kq, true) + 12.0 * n * (double)kq * kq + qr_flops;
    if (inf.resid_history && hist_pos + kw <= inf.resid_history_len) {
      std::copy(res.begin(), res.begin() + kw, inf.resid_history + hist_pos);
      hist_pos += kw;
    }
    // locking: contiguous prefix of the wanted pairs with residual <= tol
    // (and a positive Ritz value: the back-up quotient may complete the
    // positive half with non-positive values, which come last).  With an
    // indefinite S H the Ritz values obey no min-max ordering and a
    // spurious one (residual above SPURIOUS_REL |lambda~|) may sit ahead of
    // converged pairs: such pairs hold no place in the prefix.
    std::vector<int> cand, sel, rest;
    for (int i = 0; i < kw; ++i)
      if (definite || res[i] <= SPURIOUS_REL * std::fabs(ritz[i])) cand.push_back(i);
    int nlock = 0;
    while (nlock < std::min(nev - locked, (int)cand.size()) && res[cand[nlock]] <= p.tol && ritz[cand[nlock]] > 0)
      ++nlock;
    sel.assign(cand.begin(), cand.begin() + nlock);
    for (int i = 0, t = 0; i < kw; ++i) {
      if (t < nlock && sel[t] == i) {
        ++t;
        continue;
      }
      rest.push_back(i);
    }
    const bool prefix = nlock == 0 || sel[nlock - 1] == nlock - 1;
    if (nlock > 0 && prefix)
      CHASE_HIP(hipMemcpy2DAsync(h->Ylock + (int64_t)locked * n, n * sizeof(c128), h->Vt, n * sizeof(c128),
                                 n * sizeof(c128), nlock, hipMemcpyDeviceToDevice, h->st));
    if (nlock > 0 && !prefix) {
      CHASE_TRY(h2d(h, h->dperm, sel.data(), sizeof(int) * nlock));
      CHASE_TRY(gather_columns(h->Vt, n, h->Ylock + (int64_t)locked * n, n, n, nlock, h->dperm, h->st));
    }
    for (int i = 0; i < nlock; ++i) {
      lam_locked.push_back(ritz[sel[i]]);
      res_locked.push_back(res[sel[i]]);
    }
    // largest non-converged positive Ritz value; the interval only narrows (Section 4.1)
    const double lmax = *std::max_element(ritz.begin(), ritz.begin() + kw);
    if (lmax > 0) mu_nevex = std::min(mu_nevex, lmax);
    if (verbose) {
      std::fprintf(stderr,
                   "[chase_ph] it=%d locked=%d kw=%d prec=%s n_fp64=%d nlock=%d ritz[0]=%.12g ritz[kw-1]=%.8g "
                   "res[0]=%.3e res[nev-1]=%.3e res[kw-1]=%.3e mu_nevex=%.8g shifted=%d sweeps=%d\n",
                   it, locked, kw, g0 == kw ? "fp64" : (g1 ? "corr" : "fp32"), g0, nlock, ritz[0], ritz[kw - 1],
                   res[0], res[std::min(nev - locked, kw) - 1], res[kw - 1], mu_nevex, used, h->last_sweeps);
    }
    locked += nlock;
    inf.iterations = it + 1;
    if (locked >= nev) {
      *converged = true;
      break;
    }
    const int kn = kw - nlock;
    // filter mode of each remaining pair for the next iteration
    std::vector<char> nmode(kn);
    std::vector<double> npr(kn);
    for (int j = 0; j < kn; ++j) {
      const int i = rest[j];
      const double r = res[i];
      char md = mode[i];
      if (mixed && md == 2 && !(p.switch_tol > 0 && r > p.switch_tol)) md = 1;
      if (mixed && md == 1 && r < 1e3 * p.tol && r > 0.7 * prev_res[i]) md = 0;
      nmode[j] = md;
      npr[j] = r;
    }
    // next search block W+ <- unconverged Ritz vectors, grouped by filter
    // mode, each group ordered by degree
    std::vector<int> nd(kn, p.deg);
    std::vector<int> perm(kn);
    std::iota(perm.begin(), perm.end(), 0);
    if (p.opt_deg) {
      const double c = 0.5 * (mu_n * mu_n + mu_nevex * mu_nevex);
      const double e = 0.5 * (mu_n * mu_n - mu_nevex * mu_nevex);
      for (int j = 0; j < kn; ++j) {
        const double l = ritz[rest[j]], r = res[rest[j]];
        const double t = std::fabs((l * l - c) / e);
        int d;
        if (t <= 1.0 + 1e-12 || r <= p.tol) {
          d = r > p.tol ? p.deg_max : p.deg_min;
        } else {
          const double rho = t + std::sqrt(t * t - 1.0);
          d = (int)std::ceil(std::log(r / p.tol) / std::log(rho));
          d = std::min(std::max(d, p.deg_min), p.deg_max);
        }
        nd[j] = d;
      }
    }
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
      if (nmode[a] != nmode[b]) return nmode[a] < nmode[b];
      return nd[a] < nd[b];
    });
    std::vector<int> src(kn);
    degs.assign(kn, p.deg);
    g0 = 0;
    g1 = 0;
    for (int j = 0; j < kn; ++j) {
      src[j] = rest[perm[j]];
      degs[j] = nd[perm[j]];
      lamcol[j] = ritz[rest[perm[j]]];
      g0 += nmode[j] == 0;
      g1 += nmode[j] == 1;
    }
    // state stays indexed by Ritz order (pairs keep their order across iterations)
    for (int j = 0; j < kn; ++j) {
      mode[j] = nmode[j];
      prev_res[j] = npr[j];
    }
    CHASE_TRY(h2d(h, h->dperm, src.data(), sizeof(int) * kn));
    CHASE_TRY(gather_columns(h->Vt, n, h->Wk, n, n, kn, h->dperm, h->st));
    if (mixed) CHASE_TRY(gather_columns(h->Rv, n, h->Rk, n, n, kn, h->dperm, h->st));
  }
  CHASE_HIP(hipEventRecord(t1, h->st));
  CHASE_HIP(hipEventSynchronize(t1));
  float ms = 0;
  CHASE_HIP(hipEventElapsedTime(&ms, t0, t1));
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  inf.t_total = ms * 1e-3;
  inf.locked = locked;
  const int nout = std::min(locked, nev);
  // ascending output (pairs locked out of order only in the indefinite case)
  std::vector<int> order(nout);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return lam_locked[a] < lam_locked[b]; });
  bool sorted = true;
  for (int i = 0; i < nout; ++i) {
    evals[i] = lam_locked[order[i]];
    if (resid_out) resid_out[i] = res_locked[order[i]];
    sorted = sorted && order[i] == i;
  }
  if (nout > 0 && sorted)
    CHASE_HIP(hipMemcpy2DAsync(V, ldv * sizeof(c128), h->Ylock, n * sizeof(c128), n * sizeof(c128), nout,
                               hipMemcpyDeviceToDevice, h->st));
  if (nout > 0 && !sorted) {
    CHASE_TRY(h2d(h, h->dperm, order.data(), sizeof(int) * nout));
    CHASE_TRY(gather_columns(h->Ylock, n, V, ldv, n, nout, h->dperm, h->st));
  }
  CHASE_HIP(hipStreamSynchronize(h->st));
  if (info) *info = inf;
  return ok();
}

// Alg. 1 on the Hermitian A: Lanczos estimates, then per outer iteration
// filter, Cholesky QR of [Y, W], Rayleigh-Ritz G = Q^H A Q (eq. 2.2) by
// block Jacobi and an ascending sort, residuals of the unit Ritz vectors
// and locking of the leading converged pairs.  All blocks have m rows
// (leading dimension m in the handle's buffers).
Err solve_tda_impl(chase_ph_t h, const c128* W0, int64_t ldw0, const c128* Lz, int64_t ldlz, double* evals, c128* V,
                   int64_t ldv, double* resid_out, chase_ph_info* info, bool* converged) {
  const chase_ph_params& p = h->p;
  const int64_t m = h->m;
  const int nev = p.nev;
  chase_ph_info inf{};
  if (info) {
    inf.resid_history = info->resid_history;
    inf.resid_history_len = info->resid_history_len;
  }
  inf.switch_iter = -1;
  Timer tm(h);
  hipEvent_t t0, t1;
  CHASE_HIP(hipEventCreate(&t0));
  CHASE_HIP(hipEventCreate(&t1));
  CHASE_HIP(hipEventRecord(t0, h->st));
  CHASE_TRY(refresh_d64(h));  // D = [A, i A], inside the timed solve

  CHASE_TRY(tm.start());
  TdaDensity dens;
  CHASE_TRY(tda_lanczos(h, Lz, ldlz, &dens));
  int nex = p.nex;
  if (p.nex_auto) nex = tda_auto_nex(dens, m, nev, p.deg, p.tol, tda_nex_candidates(p.nex));
  const int nevex = nev + nex;
  const double mu1 = dens.mu1, mu_m = dens.mu_m;
  double mu_nevex = tda_mu_nevex(dens, nevex, m);
  CHASE_TRY(tm.stop(&inf.t_lanczos));
  inf.mu1 = mu1;
  inf.mu_nevex0 = mu_nevex;
  inf.mu_n = mu_m;
  inf.nex_used = nex;
  if (!std::isfinite(mu1) || !std::isfinite(mu_m) || !(mu_nevex > mu1) || !(mu_m > mu_nevex))
    return fail(CHASE_PH_ERR_ARG, "TDA: Lanczos spectral estimates degenerate (is A a multiple of I?)");
  const bool verbose = std::getenv("CHASE_PH_VERBOSE") != nullptr;
  if (verbose)
    std::fprintf(stderr, "[chase_ph] tda lanczos mu1=%.6g mu_nevex=%.6g mu_m=%.6g nex=%d\n", mu1, mu_nevex, mu_m, nex);

  CHASE_HIP(hipMemcpy2DAsync(h->Wk, m * sizeof(c128), W0, ldw0 * sizeof(c128), m * sizeof(c128), nevex,
                             hipMemcpyDeviceToDevice, h->st));
  int locked = 0, hist_pos = 0;
  std::vector<double> lam_locked, res_locked, ritz(nevex), res(nevex);
  std::vector<int> order(nevex);
  *converged = false;
  for (int it = 0; it < p.max_iter; ++it) {
    const int kw = nevex - locked;
    const int kt = pad64(kw);
    // filter (eq. 2.1)
    CHASE_TRY(tm.start());
    CHASE_TRY(filter_tda(h, kw, h->Wk, m, p.deg, mu1, mu_nevex, mu_m, &inf.filter_flops));
    CHASE_TRY(tm.stop(&inf.t_filter));
    // orthonormalise [Y, W]; Q = the columns after the locked ones
    CHASE_TRY(tm.start());
    if (locked > 0)
      CHASE_HIP(hipMemcpy2DAsync(h->Xs, m * sizeof(c128), h->Ylock, m * sizeof(c128), m * sizeof(c128), locked,
                                 hipMemcpyDeviceToDevice, h->st));
    CHASE_HIP(hipMemcpy2DAsync(h->Xs + (int64_t)locked * m, m * sizeof(c128), h->Wk, m * sizeof(c128),
                               m * sizeof(c128), kw, hipMemcpyDeviceToDevice, h->st));
    int used = 0;
    CHASE_TRY(qr_impl(h, nevex, h->Xs, m, nullptr, 0, &used, true, false, m));
    inf.shifted_qr_used += used == 1;
    inf.householder_qr_used += used == 2;
    inf.qr_one_pass += h->qr_one_pass;
    CHASE_TRY(tm.stop(&inf.t_qr));
    const c128* Q = h->Xs + (int64_t)locked * m;
    // Rayleigh-Ritz: G = Q^H (A Q), G Z = Z Omega, ascending
    CHASE_TRY(tm.start());
    CHASE_TRY(apply64(h, kw, Q, m, h->Tq, m));
    CHASE_TRY(fill_padded(h->G, kt, kw, 0.0, 0.0, true, h->st));
    CHASE_TRY(gemm(h, 1, 0, kw, kw, m, {1, 0}, Q, m, h->Tq, m, {0, 0}, h->G, kt));
    int sweeps = 0;
    CHASE_TRY(jacobi_eigh(h->G, h->Ev, kt, h->dws, h->st, p.rr_max_sweeps, &sweeps));
    inf.rr_sweeps_max = std::max(inf.rr_sweeps_max, sweeps);
    CHASE_TRY(diag_real(h->G, kt, kw, h->dlam, h->st));
    std::vector<double> om(kw);
    CHASE_TRY(d2h_small(om.data(), h->dlam, sizeof(double) * kw, h->dws, h->st));
    std::iota(order.begin(), order.begin() + kw, 0);
    std::stable_sort(order.begin(), order.begin() + kw, [&](int a, int b) { return om[a] < om[b]; });
    for (int j = 0; j < kw; ++j) ritz[j] = om[order[j]];
    CHASE_TRY(h2d(h, h->dperm, order.data(), sizeof(int) * kw));
    CHASE_TRY(gather_columns(h->Ev, kt, h->Ys, kt, kw, kw, h->dperm, h->st));
    CHASE_TRY(tm.stop(&inf.t_rr));
    inf.rr_flops += hx_flops((double)h->n, kw, true) + 8.0 * m * (double)kw * kw + 16.0 * m * (double)nevex * nevex;
    // residuals ||A w - omega w|| of the unit Ritz vectors w = Q z
    CHASE_TRY(tm.start());
    CHASE_TRY(gemm(h, 0, 0, m, kw, kw, {1, 0}, Q, m, h->Ys, kt, {0, 0}, h->Vt, m, -1, false));
    CHASE_TRY(gemm(h, 0, 0, m, kw, kw, {1, 0}, h->Tq, m, h->Ys, kt, {0, 0}, h->TZ, m, -1, false));
    CHASE_TRY(h2d(h, h->dlam, ritz.data(), sizeof(double) * kw));
    CHASE_TRY(residual_norms(h->Vt, m, h->TZ, m, h->dlam, m, kw, h->dres, nullptr, 0, h->st));
    CHASE_TRY(d2h_small(res.data(), h->dres, sizeof(double) * kw, h->dws, h->st));
    CHASE_TRY(tm.stop(&inf.t_resid));
    if (inf.resid_history && hist_pos + kw <= inf.resid_history_len) {
      std::copy(res.begin(), res.begin() + kw, inf.resid_history + hist_pos);
      hist_pos += kw;
    }
    // lock the leading converged pairs among the first nev - locked
    int nl = 0;
    while (nl < nev - locked && res[nl] <= p.tol) ++nl;
    if (verbose)
      std::fprintf(stderr, "[chase_ph] tda it %d: k=%d locked %d+%d omega_1=%.6g max resid %.3g\n", it, kw, locked,
                   nl, ritz[0], *std::max_element(res.begin(), res.begin() + kw));
    if (nl > 0)
      CHASE_HIP(hipMemcpy2DAsync(h->Ylock + (int64_t)locked * m, m * sizeof(c128), h->Vt, m * sizeof(c128),
                                 m * sizeof(c128), nl, hipMemcpyDeviceToDevice, h->st));
    for (int j = 0; j < nl; ++j) {
      lam_locked.push_back(ritz[j]);
      res_locked.push_back(res[j]);
    }
    if (kw - nl > 0)
      CHASE_HIP(hipMemcpy2DAsync(h->Wk, m * sizeof(c128), h->Vt + (int64_t)nl * m, m * sizeof(c128),
                                 m * sizeof(c128), kw - nl, hipMemcpyDeviceToDevice, h->st));
    mu_nevex = std::min(mu_nevex, ritz[kw - 1]);
    locked += nl;
    inf.iterations = it + 1;
    if (locked >= nev) {
      *converged = true;
      break;
    }
  }
  CHASE_HIP(hipEventRecord(t1, h->st));
  CHASE_HIP(hipEventSynchronize(t1));
  float ms = 0;
  CHASE_HIP(hipEventElapsedTime(&ms, t0, t1));
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  inf.t_total = ms * 1e-3;
  inf.locked = locked;
  const int nout = std::min(locked, nev);
  std::vector<int> out(nout);
  std::iota(out.begin(), out.end(), 0);
  std::stable_sort(out.begin(), out.end(), [&](int a, int b) { return lam_locked[a] < lam_locked[b]; });
  for (int i = 0; i < nout; ++i) {
    evals[i] = lam_locked[out[i]];
    if (resid_out) resid_out[i] = res_locked[out[i]];
  }
  if (nout > 0) {
    CHASE_TRY(h2d(h, h->dperm, out.data(), sizeof(int) * nout));
    CHASE_TRY(gather_columns(h->Ylock, m, V, ldv, m, nout, h->dperm, h->st));
  }
  CHASE_HIP(hipStreamSynchronize(h->st));
  if (info) *info = inf;
  return ok();
}

// Eigenvalue adjoint (a9): g and the weights gt live in the handle's
// workspace; the two m x m outputs come from one launch (adjoint.hip).
Err backward_impl(chase_ph_t h, int nev, const c128* V, int64_t ldv, const double* g, c128* GA, c128* GB, int64_t ldg) {
  if ((size_t)2 * nev * sizeof(double) > h->ws_bytes)
    return fail(CHASE_PH_ERR_ARG, "eigval_backward: nev exceeds the handle's workspace");
  double* dg = reinterpret_cast<double*>(h->ws);
  double* dgt = dg + nev;
  CHASE_HIP(hipMemcpyAsync(dg, g, nev * sizeof(double), hipMemcpyHostToDevice, h->st));
  CHASE_TRY(adjoint_contract(V, ldv, h->m, nev, dg, dgt, GA, GB, ldg, h->st));
  CHASE_HIP(hipStreamSynchronize(h->st));
  return ok();
}

Err create_impl(const chase_ph_params* p, const void* dA, const void* dB, int64_t ld, void* stream, chase_ph_t h) {
  h->p = *p;
  h->A = (const c128*)dA;
  h->B = (const c128*)dB;
  h->ld = ld;
  h->st = (hipStream_t)stream;
  h->m = p->m;
  h->n = 2 * p->m;
  h->nevex = p->nev + p->nex;
  h->kmax = 2 * h->nevex;
  h->kp = pad64(h->kmax);
  const int64_t n = h->n;
  const size_t kp2 = (size_t)h->kp * h->kp;
  CHASE_HIP(hipEventCreate(&h->e0));
  CHASE_HIP(hipEventCreate(&h->e1));
  h->ldd = (h->m + 63) / 64 * 64;
  CHASE_TRY(dalloc(h, &h->D64, (size_t)h->ldd * 2 * h->m));
  h->kcap = std::max(h->kmax, 512);
  h->ldyr = 4 * (int64_t)h->kcap + 8;
  h->yrows = (h->m + 31) / 32 * 32;
  CHASE_TRY(dalloc(h, &h->Yr, (size_t)h->ldyr * h->yrows));
  CHASE_TRY(dalloc(h, &h->F1, (size_t)n * h->nevex));
  CHASE_TRY(dalloc(h, &h->FT, (size_t)n * h->nevex));
  CHASE_TRY(dalloc(h, &h->Xs, (size_t)n * h->kmax));
  CHASE_TRY(dalloc(h, &h->Xt, (size_t)n * h->kmax));
  CHASE_TRY(dalloc(h, &h->Tq, (size_t)n * h->kmax));
  CHASE_TRY(dalloc(h, &h->Vt, (size_t)n * h->nevex));
  CHASE_TRY(dalloc(h, &h->TZ, (size_t)n * h->nevex));
  CHASE_TRY(dalloc(h, &h->hhw.Vb, (size_t)n * HH_PANEL));
  CHASE_TRY(dalloc(h, &h->hhw.Tb, (size_t)HH_PANEL * h->kmax));
  CHASE_TRY(dalloc(h, &h->hhw.W1, (size_t)HH_PANEL * h->kmax));
  CHASE_TRY(dalloc(h, &h->hhw.W2, (size_t)HH_PANEL * h->kmax));
  CHASE_TRY(dalloc(h, &h->hhw.taus, (size_t)h->kmax));
  CHASE_TRY(dalloc(h, &h->hhw.part, (size_t)HH_PARTS));
  CHASE_TRY(dalloc(h, &h->hhw.dpart, (size_t)HH_PARTS * HH_PANEL));
  CHASE_TRY(dalloc(h, &h->hhw.dsign, (size_t)h->kmax));
  h->hhw.Q = h->Xt;
  h->hhw.kmax = h->kmax;
  CHASE_TRY(dalloc(h, &h->gw.v, (size_t)h->kmax));
  CHASE_TRY(dalloc(h, &h->gw.tau, 1));
  CHASE_TRY(dalloc(h, &h->gw.status, 1));
  CHASE_TRY(dalloc(h, &h->Wev, (size_t)h->kmax));
  CHASE_TRY(dalloc(h, &h->G, kp2));
  CHASE_TRY(dalloc(h, &h->L1, kp2));
  CHASE_TRY(dalloc(h, &h->L2, kp2));
  CHASE_TRY(dalloc(h, &h->L3, kp2));
  CHASE_TRY(dalloc(h, &h->Li, kp2));
  CHASE_TRY(dalloc(h, &h->Nb, kp2));
  CHASE_TRY(dalloc(h, &h->Tk, kp2));
  CHASE_TRY(dalloc(h, &h->Ev, kp2));
  CHASE_TRY(dalloc(h, &h->Ys, kp2));
  CHASE_TRY(dalloc(h, &h->Zp, (size_t)h->kmax * h->nevex));
  CHASE_TRY(dalloc(h, &h->Ylock, (size_t)n * std::max(1, p->nev)));
  CHASE_TRY(dalloc(h, &h->Wk, (size_t)n * h->nevex));
  CHASE_TRY(dalloc(h, &h->dlam, (size_t)h->kmax));
  CHASE_TRY(dalloc(h, &h->dres, (size_t)h->kmax));
  CHASE_TRY(dalloc(h, &h->dperm, (size_t)h->kmax));
  const int nv = std::max(1, p->lanczos_vecs);
  CHASE_TRY(dalloc(h, &h->lv, (size_t)n * nv));
  CHASE_TRY(dalloc(h, &h->lvp, (size_t)n * nv));
  CHASE_TRY(dalloc(h, &h->lw, (size_t)n * nv));
  CHASE_TRY(dalloc(h, &h->lr, (size_t)n * nv));
  CHASE_TRY(dalloc(h, &h->lz, (size_t)n * nv));
  CHASE_TRY(dalloc(h, &h->dab, (size_t)(2 * std::max(1, p->lanczos_steps) + 1) * nv));
  CHASE_TRY(dalloc(h, &h->dws.small, 64 * 64));
  CHASE_TRY(dalloc(h, &h->dws.panel, (size_t)h->kp * 64));
  CHASE_TRY(dalloc(h, &h->dws.tmp, (size_t)h->kp * 64));
  CHASE_TRY(dalloc(h, &h->dws.U, (size_t)h->kp * 64));
  CHASE_TRY(dalloc(h, &h->dws.flag, 4));
  CHASE_TRY(dalloc(h, &h->dws.pflag, (size_t)h->kp / 8 + 1));
  CHASE_TRY(dalloc(h, &h->dws.dscalar, 4));
  // pinned host staging for the small reads of every iteration (flags,
  // counts, Ritz values, residuals: at most kmax doubles)
  h->dws.hpin_bytes = std::max<size_t>(4096, sizeof(double) * (size_t)h->kmax);
  CHASE_HIP(hipHostMalloc(&h->dws.hpin, h->dws.hpin_bytes, hipHostMallocDefault));
  // zgemm split-K partials (up to 8 k x k blocks) and apply_h split-K
  // partials (up to 8 x m x 2 nevex complex), within [16 MiB, 1 GiB]
  h->ws_bytes = std::max(kp2 * sizeof(c128) * 8, (size_t)8 * h->m * h->kmax * sizeof(c128));
  h->ws_bytes = std::min<size_t>((size_t)1 << 30, std::max<size_t>((size_t)16 << 20, h->ws_bytes));
  CHASE_TRY(dalloc(h, (char**)&h->ws, h->ws_bytes));
  h->dws.gemm_ws = h->ws;
  h->dws.gemm_ws_bytes = h->ws_bytes;
  h->hhw.gemm_ws = h->ws;
  h->hhw.gemm_ws_bytes = h->ws_bytes;
  if (p->precision == CHASE_PH_MIXED) CHASE_TRY(alloc_shadow(h));
  return ok();
}

}  // namespace

extern "C" {

void chase_ph_default_params(chase_ph_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->deg = 20;
  p->deg_min = 8;
  p->deg_max = 20;
  p->opt_deg = 0;
  p->max_iter = 25;
  p->tol = 1e-10;
  p->precision = CHASE_PH_FP64;
  p->switch_tol = 0.0;
  p->gamma = 1e-3;
  p->lanczos_steps = 26;
  p->lanczos_vecs = 4;
  p->a_conj = 0;
  p->definite = 1;
  p->rr_max_sweeps = 40;
}

chase_ph_status chase_ph_create(const chase_ph_params* p, const void* dA, const void* dB, int64_t ld, void* hip_stream,
                                chase_ph_t* out) {
  if (!out) return CHASE_PH_ERR_ARG;
  *out = nullptr;
  if (!p || (p->tda != 0 && p->tda != 1) || (p->nex_auto != 0 && p->nex_auto != 1)) return CHASE_PH_ERR_ARG;
  // TDA (Alg. 1): FP64 filter of fixed degree, B not read; nex_auto needs it
  if ((p->tda && (p->precision != CHASE_PH_FP64 || p->opt_deg)) || (p->nex_auto && (!p->tda || p->nex < 1)))
    return CHASE_PH_ERR_ARG;
  if (!dA || (!dB && !p->tda) || p->m <= 0 || ld < p->m || p->nev <= 0 || p->nex < 0 || p->nev + p->nex > p->m ||
      p->deg < 1 || p->max_iter < 1 || !(p->tol > 0) || p->lanczos_steps < 2 || p->lanczos_steps % 2 != 0 ||
      p->lanczos_vecs < 1 || (p->precision != CHASE_PH_FP64 && p->precision != CHASE_PH_MIXED) ||
      (p->opt_deg && (p->deg_min < 1 || p->deg_max < p->deg_min)) || (p->rr_backup != 0 && p->rr_backup != 1) ||
      (p->definite != 0 && p->definite != 1) || p->rr_max_sweeps < 1)
    return CHASE_PH_ERR_ARG;
  chase_ph_t h = new (std::nothrow) chase_ph_s;
  if (!h) return CHASE_PH_ERR_ALLOC;
  Err e = create_impl(p, dA, dB, ld, hip_stream, h);
  if (e) {
    chase_ph_destroy(h);
    return e.st;
  }
  *out = h;
  return CHASE_PH_OK;
}

chase_ph_status chase_ph_destroy(chase_ph_t h) {
  if (!h) return CHASE_PH_OK;
  if (h->st) (void)hipStreamSynchronize(h->st);
  else (void)hipDeviceSynchronize();
  for (void* q : h->allocs) (void)hipFree(q);
  if (h->dws.hpin) (void)hipHostFree(h->dws.hpin);
  for (hipEvent_t e : h->evpool) (void)hipEventDestroy(e);
  if (h->e0) (void)hipEventDestroy(h->e0);
  if (h->e1) (void)hipEventDestroy(h->e1);
  delete h;
  return CHASE_PH_OK;
}

const char* chase_ph_last_error(chase_ph_t h) { return h ? h->err.c_str() : chase::noalloc_last_error(); }

#define CHECK_HANDLE(h)                                   \
  do {                                                    \
    if (!(h)) return CHASE_PH_ERR_ARG;                    \
    if ((h)->dead) {                                      \
      (h)->err = "handle unusable after a HIP error";     \
      return CHASE_PH_ERR_HIP;                            \
    }                                                     \
  } while (0)

// Stage calls of the pseudo-hermitian solver, not defined on a TDA handle.
#define CHECK_PH_HANDLE(h)                                                            \
  do {                                                                                \
    CHECK_HANDLE(h);                                                                  \
    if ((h)->p.tda) return finish(h, fail(CHASE_PH_ERR_ARG, "stage call not defined on a TDA handle")); \
  } while (0)

chase_ph_status chase_ph_apply_h(chase_ph_t h, int32_t k, const void* dX, int64_t ldx, void* dY, int64_t ldy,
                                 int32_t prec) {
  CHECK_HANDLE(h);
  const int64_t rows = h->p.tda ? h->m : h->n;
  if (k < 0 || (k > 0 && (!dX || !dY)) || ldx < rows || ldy < rows ||
      (prec != CHASE_PH_FP64 && prec != CHASE_PH_FP32 && prec != CHASE_PH_FP64_KREAL) ||
      (h->p.tda && prec == CHASE_PH_FP64_KREAL))
    return finish(h, fail(CHASE_PH_ERR_ARG, "apply_h: bad arguments"));
  if (k == 0) return CHASE_PH_OK;
  Err e = ok();
  if (hipEventRecord(h->e0, h->st) != hipSuccess) return finish(h, fail(CHASE_PH_ERR_HIP, "event record"));
  if (prec == CHASE_PH_FP32) {
    e = ensure_shadow(h);
    if (!e) e = apply32(h, k, (const c64*)dX, ldx, (c64*)dY, ldy);
  } else {
    e = apply64(h, k, (const c128*)dX, ldx, (c128*)dY, ldy, 1, nullptr, 0, 0, nullptr, 0, 0,
                prec == CHASE_PH_FP64_KREAL ? 1 : 0);
  }
  if (e) return finish(h, e);
  float ms = 0;
  if (hipEventRecord(h->e1, h->st) != hipSuccess || hipEventSynchronize(h->e1) != hipSuccess ||
      hipEventElapsedTime(&ms, h->e0, h->e1) != hipSuccess)
    return finish(h, fail(CHASE_PH_ERR_HIP, "apply_h: kernel failed"));
  h->last_ms = ms;
  h->last_launches = 1;
  return CHASE_PH_OK;
}

chase_ph_status chase_ph_filter(chase_ph_t h, int32_t k, void* dW, int64_t ldw, const int32_t* degs, double mu1,
                                double mu_nevex, double mu_n, int32_t prec) {
  CHECK_PH_HANDLE(h);
  std::vector<int> d;
  Err e = check_filter_args(h, k, ldw, degs, mu1, mu_nevex, mu_n, d);
  if (!e && (prec != CHASE_PH_FP64 && prec != CHASE_PH_FP32)) e = fail(CHASE_PH_ERR_ARG, "filter: bad precision");
  if (!e && k > 0 && !dW) e = fail(CHASE_PH_ERR_ARG, "filter: null W");
  if (e) return finish(h, e);
  return finish(h, filter_any(h, k, dW, ldw, d, mu1, mu_nevex, mu_n, prec, nullptr));
}

chase_ph_status chase_ph_filter_refined(chase_ph_t h, int32_t k, void* dW, int64_t ldw, const void* dR, int64_t ldr,
                                        const double* hLam, const int32_t* degs, double mu1, double mu_nevex,
                                        double mu_n) {
  CHECK_PH_HANDLE(h);
  std::vector<int> d;
  Err e = check_filter_args(h, k, ldw, degs, mu1, mu_nevex, mu_n, d);
  if (!e && k > 0 && (!dW || !dR || !hLam || ldr < h->n)) e = fail(CHASE_PH_ERR_ARG, "filter_refined: bad arguments");
  if (e) return finish(h, e);
  if (k == 0) return CHASE_PH_OK;
  e = ensure_shadow(h);
  std::vector<double> lam(hLam, hLam + k);
  double fl = 0;
  if (!e) e = filter_correction(h, k, (c128*)dW, ldw, (const c128*)dR, ldr, lam, d, mu1, mu_nevex, mu_n, &fl);
  if (!e && hipStreamSynchronize(h->st) != hipSuccess) e = fail(CHASE_PH_ERR_HIP, "filter_refined: sync");
  return finish(h, e);
}

chase_ph_status chase_ph_qr(chase_ph_t h, int32_t k, void* dX, int64_t ldx, void* dR, int64_t ldr, int32_t* used_shift) {
  CHECK_PH_HANDLE(h);
  if (k < 0 || k > h->kmax || (k > 0 && !dX) || ldx < h->n || (dR && ldr < k))
    return finish(h, fail(CHASE_PH_ERR_ARG, "qr: bad arguments"));
  int us = 0;
  Err e = qr_impl(h, k, (c128*)dX, ldx, (c128*)dR, ldr, &us);
  if (!e) {
    if (hipStreamSynchronize(h->st) != hipSuccess) e = fail(CHASE_PH_ERR_HIP, "qr: sync");
  }
  if (used_shift) *used_shift = us;
  return finish(h, e);
}

chase_ph_status chase_ph_oblique_rr(chase_ph_t h, int32_t k, const void* dQ, int64_t ldq, double* hRitz, void* dZpos,
                                    int64_t ldz, void* dT, int64_t ldt) {
  CHECK_PH_HANDLE(h);
  if (k <= 0 || k % 2 != 0 || k > h->kmax || !dQ || !hRitz || !dZpos || !dT || ldq < h->n || ldz < k || ldt < h->n)
    return finish(h, fail(CHASE_PH_ERR_ARG, "oblique_rr: bad arguments"));
  return finish(h, rr_impl(h, k, (const c128*)dQ, ldq, hRitz, (c128*)dZpos, ldz, (c128*)dT, ldt));
}

chase_ph_status chase_ph_oblique_rr_backup(chase_ph_t h, int32_t k, const void* dQ, int64_t ldq, double* hRitz,
                                           void* dZpos, int64_t ldz, void* dT, int64_t ldt) {
  CHECK_PH_HANDLE(h);
  if (k <= 0 || k % 2 != 0 || k > h->kmax || !dQ || !hRitz || !dZpos || !dT || ldq < h->n || ldz < k || ldt < h->n)
    return finish(h, fail(CHASE_PH_ERR_ARG, "oblique_rr_backup: bad arguments"));
  return finish(h, rr_impl(h, k, (const c128*)dQ, ldq, hRitz, (c128*)dZpos, ldz, (c128*)dT, ldt, false, 1));
}

chase_ph_status chase_ph_oblique_rr_general(chase_ph_t h, int32_t k, const void* dQ, int64_t ldq, double* hRitz,
                                            void* dZpos, int64_t ldz, void* dT, int64_t ldt) {
  CHECK_PH_HANDLE(h);
  if (k <= 0 || k % 2 != 0 || k > h->kmax || !dQ || !hRitz || !dZpos || !dT || ldq < h->n || ldz < k || ldt < h->n)
    return finish(h, fail(CHASE_PH_ERR_ARG, "oblique_rr_general: bad arguments"));
  return finish(h, rr_impl(h, k, (const c128*)dQ, ldq, hRitz, (c128*)dZpos, ldz, (c128*)dT, ldt, false, 3));
}

chase_ph_status chase_ph_residuals(chase_ph_t h, int32_t k, int32_t kk, const void* dQ, int64_t ldq, const void* dT,
                                   int64_t ldt, const void* dZpos, int64_t ldz, const double* hRitz, void* dV,
                                   int64_t ldv, double* hResid) {
  CHECK_PH_HANDLE(h);
  if (k <= 0 || k > h->kmax || kk < 0 || kk > k / 2 || kk > h->nevex || !dQ || !dT || !dZpos || !hRitz || !dV ||
      !hResid || ldq < h->n || ldt < h->n || ldz < k || ldv < h->n)
    return finish(h, fail(CHASE_PH_ERR_ARG, "residuals: bad arguments"));
  return finish(h, resid_impl(h, k, kk, (const c128*)dQ, ldq, (const c128*)dT, ldt, (const c128*)dZpos, ldz, hRitz,
                              (c128*)dV, ldv, hResid));
}

chase_ph_status chase_ph_solve(chase_ph_t h, const void* dW0, int64_t ldw0, const void* dLz, int64_t ldlz,
                               double* hEvals, void* dV, int64_t ldv, double* hResid, chase_ph_info* info) {
  CHECK_HANDLE(h);
  const int64_t rows = h->p.tda ? h->m : h->n;
  if (!dW0 || !dLz || !hEvals || !dV || ldw0 < rows || ldlz < rows || ldv < rows)
    return finish(h, fail(CHASE_PH_ERR_ARG, "solve: bad arguments"));
  bool conv = false;
  Err e = h->p.tda ? solve_tda_impl(h, (const c128*)dW0, ldw0, (const c128*)dLz, ldlz, hEvals, (c128*)dV, ldv,
                                    hResid, info, &conv)
                   : solve_impl(h, (const c128*)dW0, ldw0, (const c128*)dLz, ldlz, hEvals, (c128*)dV, ldv, hResid,
                                info, &conv);
  if (e) return finish(h, e);
  if (!conv) return finish(h, fail(CHASE_PH_ERR_NO_CONVERGENCE, "max_iter reached before nev pairs converged"));
  return CHASE_PH_OK;
}

chase_ph_status chase_ph_eigval_backward(chase_ph_t h, int32_t nev, const void* dV, int64_t ldv, const double* hG,
                                         void* dGA, void* dGB, int64_t ldg) {
  CHECK_PH_HANDLE(h);
  if (nev <= 0 || !dV || !hG || !dGA || !dGB || ldv < h->n || ldg < h->m)
    return finish(h, fail(CHASE_PH_ERR_ARG, "eigval_backward: bad arguments"));
  return finish(h, backward_impl(h, nev, (const c128*)dV, ldv, hG, (c128*)dGA, (c128*)dGB, ldg));
}

chase_ph_status chase_ph_profile(chase_ph_t h, int32_t enable) {
  CHECK_HANDLE(h);
  h->prof = enable != 0;
  h->launches.clear();
  return CHASE_PH_OK;
}

chase_ph_status chase_ph_profile_read(chase_ph_t h, int32_t prec, double* total_ms, double* flops, double* bytes,
                                      int32_t* launches) {
  CHECK_HANDLE(h);
  if (hipStreamSynchronize(h->st) != hipSuccess) return finish(h, fail(CHASE_PH_ERR_HIP, "profile_read: sync"));
  double ms = 0, fl = 0, by = 0;
  int cnt = 0;
  // CHASE_PH_PROF_DUMP=1 lists every call (precision, columns, milliseconds) on stderr
  const char* dump = std::getenv("CHASE_PH_PROF_DUMP");
  const bool dump_calls = dump && dump[0] == '1';
  for (size_t i = 0; i < h->launches.size(); ++i) {
    if (h->launches[i].prec != prec) continue;
    float t = 0;
    if (hipEventElapsedTime(&t, h->evpool[2 * i], h->evpool[2 * i + 1]) != hipSuccess)
      return finish(h, fail(CHASE_PH_ERR_HIP, "profile_read: elapsed time"));
    if (dump_calls) std::fprintf(stderr, "[chase_ph] call prec=%d k=%d ms=%.4f\n", prec, h->launches[i].k, t);
    ms += t;
    fl += h->launches[i].flops;
    by += h->launches[i].bytes;
    ++cnt;
  }
  if (total_ms) *total_ms = ms;
  if (flops) *flops = fl;
  if (bytes) *bytes = by;
  if (launches) *launches = cnt;
  return CHASE_PH_OK;
}

chase_ph_status chase_ph_last_timing(chase_ph_t h, double* ms, int32_t* launches) {
  if (!h) return CHASE_PH_ERR_ARG;
  if (ms) *ms = h->last_ms;
  if (launches) *launches = h->last_launches;
  return CHASE_PH_OK;
}

}  // extern "C"
