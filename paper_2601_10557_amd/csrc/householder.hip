// Householder QR of a tall n x k c128 block: the last-resort orthonormalisation
// of Section 2, which pairs Cholesky QR with a Householder QR chosen by
// condition number.  It runs when CholeskyQR2 and its shifted CholeskyQR3
// fallback both break down (a numerically rank-deficient block), since it
// is unconditionally stable and yields an orthonormal basis whose leading
// columns span the leading columns of the block for any rank.
//  * Panels of HB = 32 columns.  Inside a panel each column takes three
//    launches over all rows: the partial sums of its squared norm below the
//    diagonal, the reflector (computed redundantly by every workgroup from
//    those sums, in the same fixed order) with the partial dot products of
//    the panel's later columns, and the rank-one update.  A zero column below
//    the diagonal with a real diagonal entry gets tau = 0 (H = I).
//  * Reflectors follow the usual complex convention H = I - tau v v^H with
//    v(0) = 1 and H^H [alpha; x] = [beta; 0], beta real.
//  * The panel's reflectors are applied to the trailing columns in compact
//    WY form, (I - V T V^H)^H C = C - V T^H (V^H C), with three complex GEMMs
//    on the FP64 MFMA; T comes from V^H V by the triangular recurrence
//    T(0:i, i) = -tau_i T(0:i, 0:i) (V(:, 0:i)^H v_i).
//  * Q = H_1 ... H_k [I; 0] is accumulated panel by panel from the last one,
//    and the signs of beta are moved from R into Q so that R has a real
//    non-negative diagonal (zero exactly where a column depends on the
//    previous ones).
#include <algorithm>
#include <cmath>

#include "common.h"
#include "dense.h"

namespace chase {
namespace {

constexpr int HB = HH_PANEL;  // panel width
constexpr int HP = HH_PARTS;  // workgroups of the row-parallel launches (one wave each)

__device__ __forceinline__ c128 hmul(c128 a, c128 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ c128 hconj(c128 a) { return {a.re, -a.im}; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

struct Refl {
  double beta;   // new diagonal entry (real)
  c128 tau;      // H = I - tau v v^H
  c128 scale;    // v(i) = x(i) * scale below the diagonal
  int ident;     // 1: H = I
};

// Sum of part[0 .. HP) in a fixed order, the same in every lane (called by
// the whole wave: lane l adds part[l + 64 q], then a butterfly of lane
// swaps, whose additions pair the same operands in every lane).
__device__ __forceinline__ double wave_total(const double* part) {
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < HP / 64; ++q) v += part[threadIdx.x + 64 * q];
  return wave_sum(v);
}

// Reflector of the column whose diagonal entry is alpha and whose squared
// norm below the diagonal is the sum of part[0 .. HP) (whole wave).
__device__ Refl reflector(const double* part, c128 alpha) {
  const double xs = wave_total(part);
  Refl r;
  if (xs == 0.0 && alpha.im == 0.0) {
    r.beta = alpha.re;
    r.tau = c128{0.0, 0.0};
    r.scale = c128{0.0, 0.0};
    r.ident = 1;
    return r;
  }
  const double nrm = std::sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xs);
  const double beta = alpha.re >= 0.0 ? -nrm : nrm;
  r.beta = beta;
  r.tau = c128{(beta - alpha.re) / beta, -alpha.im / beta};
  const c128 d{alpha.re - beta, alpha.im};            // 1 / (alpha - beta)
  const double dd = d.re * d.re + d.im * d.im;
  r.scale = c128{d.re / dd, -d.im / dd};
  r.ident = 0;
  return r;
}

// part[b] = sum of |X(i, col)|^2 over the rows i > r0 of workgroup b.
__global__ __launch_bounds__(64) void hh_colnorm_kernel(const c128* X, int64_t ldx, int64_t r0, int64_t n, int col,
                                                        double* part) {
  const c128* x = X + (int64_t)col * ldx;
  double s = 0.0;
  for (int64_t i = r0 + 1 + (int64_t)blockIdx.x * 64 + threadIdx.x; i < n; i += (int64_t)HP * 64)
    s += x[i].re * x[i].re + x[i].im * x[i].im;
  s = wave_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// dpart[b * HB + j] = sum over the rows i >= r0 of workgroup b of
// conj(v(i)) X(i, col + 1 + j), j < ncols.
__global__ __launch_bounds__(64) void hh_dot_kernel(const c128* X, int64_t ldx, int64_t r0, int64_t n, int col,
                                                    int ncols, const double* part, c128* dpart) {
  const Refl r = reflector(part, X[(int64_t)col * ldx + r0]);
  c128 acc[HB - 1];
#pragma unroll
  for (int j = 0; j < HB - 1; ++j) acc[j] = c128{0.0, 0.0};
  if (!r.ident) {
    for (int64_t i = r0 + (int64_t)blockIdx.x * 64 + threadIdx.x; i < n; i += (int64_t)HP * 64) {
      const c128 v = i == r0 ? c128{1.0, 0.0} : hmul(X[(int64_t)col * ldx + i], r.scale);
      const c128 vc = hconj(v);
#pragma unroll
      for (int j = 0; j < HB - 1; ++j)
        if (j < ncols) {
          const c128 y = hmul(vc, X[(int64_t)(col + 1 + j) * ldx + i]);
          acc[j].re += y.re;
          acc[j].im += y.im;
        }
    }
  }
#pragma unroll
  for (int j = 0; j < HB - 1; ++j) {
    if (j >= ncols) break;
    const double re = wave_sum(acc[j].re), im = wave_sum(acc[j].im);
    if (threadIdx.x == 0) dpart[(int64_t)blockIdx.x * HB + j] = c128{re, im};
  }
}

// X(:, col + 1 + j) -= conj(tau) v (v^H X(:, col + 1 + j)) on the rows
// i >= r0; then the column stores beta on the diagonal and v below it.
__global__ __launch_bounds__(64) void hh_update_kernel(c128* X, int64_t ldx, int64_t r0, int64_t n, int col,
                                                       int ncols, const double* part, const c128* dpart, c128* taus) {
  __shared__ c128 dsum[HB];
  const Refl r = reflector(part, X[(int64_t)col * ldx + r0]);
  for (int j = 0; j < ncols; ++j) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int q = 0; q < HP / 64; ++q) {
      const c128 z = dpart[(int64_t)(threadIdx.x + 64 * q) * HB + j];
      re += z.re;
      im += z.im;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (threadIdx.x == 0) dsum[j] = c128{re, im};
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) taus[col] = r.tau;
  const c128 tc = hconj(r.tau);
  for (int64_t i = r0 + (int64_t)blockIdx.x * 64 + threadIdx.x; i < n; i += (int64_t)HP * 64) {
    c128* xc = X + (int64_t)col * ldx + i;
    if (r.ident) {
      if (i == r0) *xc = c128{r.beta, 0.0};
      continue;
    }
    const c128 v = i == r0 ? c128{1.0, 0.0} : hmul(*xc, r.scale);
    const c128 tv = hmul(tc, v);
    for (int j = 0; j < ncols; ++j) {
      c128* y = X + (int64_t)(col + 1 + j) * ldx + i;
      const c128 u = hmul(tv, dsum[j]);
      y->re -= u.re;
      y->im -= u.im;
    }
    *xc = i == r0 ? c128{r.beta, 0.0} : v;
  }
}

// Explicit reflectors of the panel starting at column p (w columns): Vb
// (ld n, global row index) gets 0 above the diagonal, 1 on it and the
// stored v below it, on the rows p .. n - 1.
__global__ void hh_vcopy_kernel(const c128* X, int64_t ldx, int64_t n, int p, int w, c128* Vb) {
  const int64_t rows = n - p, total = rows * w;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t / rows);
    const int64_t i = p + t % rows;
    const int64_t dg = p + c;
    c128 v{0.0, 0.0};
    if (i == dg) v = c128{1.0, 0.0};
    else if (i > dg) v = X[dg * ldx + i];
    Vb[(int64_t)c * n + i] = v;
  }
}

// T (w x w upper triangular, ld HB) of the compact WY form from S = V^H V
// (ld HB) and the panel's taus; only the w x w block is written (the last
// panel's block ends at column k of the T buffer).
__global__ __launch_bounds__(64) void hh_tfactor_kernel(const c128* S, const c128* taus, int w, c128* T) {
  __shared__ c128 t[HB][HB + 1];
  const int r = threadIdx.x;
  if (r < HB)
    for (int c = 0; c < HB; ++c) t[r][c] = c128{0.0, 0.0};
  __syncthreads();
  for (int i = 0; i < w; ++i) {
    if (r < i) {
      c128 acc{0.0, 0.0};
      for (int c = r; c < i; ++c) {
        const c128 y = hmul(t[r][c], S[(int64_t)i * HB + c]);
        acc.re += y.re;
        acc.im += y.im;
      }
      const c128 y = hmul(taus[i], acc);
      t[r][i] = c128{-y.re, -y.im};
    } else if (r == i) {
      t[r][i] = taus[i];
    }
    __syncthreads();
  }
  if (r < w)
    for (int c = 0; c < w; ++c) T[(int64_t)c * HB + r] = t[r][c];
}

// Q = [I_k; 0] (n x k, ld n).
__global__ void hh_eye_kernel(c128* Q, int64_t n, int k) {
  const int64_t total = n * k;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / n, i = t % n;
    Q[t] = c128{i == j ? 1.0 : 0.0, 0.0};
  }
}

// R(i, j) = d_i X(i, j) for i <= j < k, 0 below (k x k, ld ldr), with
// d_i = -1 for a negative beta_i, else 1.
__global__ void hh_r_kernel(const c128* X, int64_t ldx, int k, const double* dsign, c128* R, int64_t ldr) {
  const int64_t total = (int64_t)k * k;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / k, i = t % k;
    const double d = dsign[i];
    const c128 x = X[j * ldx + i];
    R[j * ldr + i] = i <= j ? c128{d * x.re, d * x.im} : c128{0.0, 0.0};
  }
}

// X(:, j) = d_j Q(:, j) (the sign of beta_j moved into Q).
__global__ void hh_copy_q_kernel(c128* X, int64_t ldx, const c128* Q, int64_t n, int k, const double* dsign) {
  const int64_t total = n * k;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / n, i = t % n;
    const double d = dsign[j];
    const c128 q = Q[t];
    X[j * ldx + i] = c128{d * q.re, d * q.im};
  }
}

__global__ void hh_signs_kernel(const c128* X, int64_t ldx, int k, double* dsign) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < k; j += gridDim.x * blockDim.x)
    dsign[j] = X[(int64_t)j * ldx + j].re < 0.0 ? -1.0 : 1.0;
}

int grid_for(int64_t total) { return (int)std::min<int64_t>(std::max<int64_t>(ceil_div(total, 256), 1), 4096); }

Err gemm_hh(int ta, int tb, int64_t M, int64_t N, int64_t K, c128 alpha, const c128* A, int64_t lda, const c128* B,
            int64_t ldb, c128 beta, c128* C, int64_t ldc, const HouseholderWs& w, hipStream_t s) {
  ZgemmArgs g{};
  g.transA = ta; g.transB = tb;
  g.M = M; g.N = N; g.K = K;
  g.alpha = alpha; g.beta = beta;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.kneg = K;
  g.batch = 1;
  return zgemm(g, w.gemm_ws, w.gemm_ws_bytes, s);
}

}  // namespace

Err householder_qr(c128* X, int64_t ldx, int64_t n, int k, c128* R, int64_t ldr, const HouseholderWs& w,
                   hipStream_t s) {
  if (k <= 0) return ok();
  if (k > n || k > w.kmax) return fail(CHASE_PH_ERR_ARG, "householder_qr: k exceeds the workspace");
  // factorisation, panel by panel
  for (int p = 0; p < k; p += HB) {
    const int pw = std::min(HB, k - p);
    for (int c = 0; c < pw; ++c) {
      const int col = p + c;
      const int ncols = pw - 1 - c;
      hipLaunchKernelGGL(hh_colnorm_kernel, dim3(HP), dim3(64), 0, s, (const c128*)X, ldx, (int64_t)col, n, col,
                         w.part);
      CHASE_LAUNCH_CHECK();
      if (ncols > 0) {
        hipLaunchKernelGGL(hh_dot_kernel, dim3(HP), dim3(64), 0, s, (const c128*)X, ldx, (int64_t)col, n, col, ncols,
                           (const double*)w.part, w.dpart);
        CHASE_LAUNCH_CHECK();
      }
      hipLaunchKernelGGL(hh_update_kernel, dim3(HP), dim3(64), 0, s, X, ldx, (int64_t)col, n, col, ncols,
                         (const double*)w.part, (const c128*)w.dpart, w.taus);
      CHASE_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(hh_vcopy_kernel, dim3(grid_for((n - p) * pw)), dim3(256), 0, s, (const c128*)X, ldx, n, p, pw,
                       w.Vb);
    CHASE_LAUNCH_CHECK();
    // S = V^H V, then T of this panel
    CHASE_TRY(gemm_hh(1, 0, pw, pw, n - p, {1, 0}, w.Vb + p, n, w.Vb + p, n, {0, 0}, w.W1, HB, w, s));
    c128* Tp = w.Tb + (int64_t)p * HB;
    hipLaunchKernelGGL(hh_tfactor_kernel, dim3(1), dim3(64), 0, s, (const c128*)w.W1, (const c128*)(w.taus + p), pw,
                       Tp);
    CHASE_LAUNCH_CHECK();
    const int nt = k - p - pw;
    if (nt > 0) {
      c128* C = X + (int64_t)(p + pw) * ldx + p;
      CHASE_TRY(gemm_hh(1, 0, pw, nt, n - p, {1, 0}, w.Vb + p, n, C, ldx, {0, 0}, w.W1, HB, w, s));   // V^H C
      CHASE_TRY(gemm_hh(1, 0, pw, nt, pw, {1, 0}, Tp, HB, w.W1, HB, {0, 0}, w.W2, HB, w, s));        // T^H (V^H C)
      CHASE_TRY(gemm_hh(0, 0, n - p, nt, pw, {-1, 0}, w.Vb + p, n, w.W2, HB, {1, 0}, C, ldx, w, s)); // C -= V ...
    }
  }
  // Q = H_1 ... H_k [I; 0], from the last panel to the first
  hipLaunchKernelGGL(hh_eye_kernel, dim3(grid_for(n * k)), dim3(256), 0, s, w.Q, n, k);
  CHASE_LAUNCH_CHECK();
  const int last = (k - 1) / HB * HB;
  for (int p = last; p >= 0; p -= HB) {
    const int pw = std::min(HB, k - p);
    hipLaunchKernelGGL(hh_vcopy_kernel, dim3(grid_for((n - p) * pw)), dim3(256), 0, s, (const c128*)X, ldx, n, p, pw,
                       w.Vb);
    CHASE_LAUNCH_CHECK();
    c128* Qp = w.Q + (int64_t)p * n + p;
    const int nq = k - p;
    CHASE_TRY(gemm_hh(1, 0, pw, nq, n - p, {1, 0}, w.Vb + p, n, Qp, n, {0, 0}, w.W1, HB, w, s));            // V^H Q
    CHASE_TRY(gemm_hh(0, 0, pw, nq, pw, {1, 0}, w.Tb + (int64_t)p * HB, HB, w.W1, HB, {0, 0}, w.W2, HB, w, s));  // T (V^H Q)
    CHASE_TRY(gemm_hh(0, 0, n - p, nq, pw, {-1, 0}, w.Vb + p, n, w.W2, HB, {1, 0}, Qp, n, w, s));           // Q -= V ...
  }
  // signs of beta into Q, R from the upper triangle
  hipLaunchKernelGGL(hh_signs_kernel, dim3(grid_for(k)), dim3(256), 0, s, (const c128*)X, ldx, k, w.dsign);
  CHASE_LAUNCH_CHECK();
  if (R) {
    hipLaunchKernelGGL(hh_r_kernel, dim3(grid_for((int64_t)k * k)), dim3(256), 0, s, (const c128*)X, ldx, k,
                       (const double*)w.dsign, R, ldr);
    CHASE_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(hh_copy_q_kernel, dim3(grid_for(n * k)), dim3(256), 0, s, X, ldx, (const c128*)w.Q, n, k,
                     (const double*)w.dsign);
  CHASE_LAUNCH_CHECK();
  return ok();
}

}  // namespace chase
