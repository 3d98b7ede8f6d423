// Elementwise and column-reduction kernels of the solver loop: the real
// coordinates of the K-real pairs of the search block [S Y, S K conj(Y), W,
// K conj(W)] (Section 4.3, eq. 4.5; Thm 4.2) and their inverse, the pair
// recombination before the Rayleigh-Ritz quotient, c128 <-> c64 conversion
// of the filter block, the fused
// residual / normalisation of the half back-transform (Section 4.5),
// and the S-inner products of the Lanczos estimates (Section 4.1).
#include <algorithm>

#include "common.h"
#include "vec.h"

namespace chase {
namespace {

inline int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 8192)); }

__global__ void to_c64_kernel(const c128* src, int64_t lds, c64* dst, int64_t ldd, int64_t rows, int cols) {
  const int64_t total = rows * cols;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / rows, i = t % rows;
    const c128 z = src[j * lds + i];
    dst[j * ldd + i] = c64{(float)z.re, (float)z.im};
  }
}

__global__ void to_c128_kernel(const c64* src, int64_t lds, c128* dst, int64_t ldd, int64_t rows, int cols) {
  const int64_t total = rows * cols;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / rows, i = t % rows;
    const c64 z = src[j * lds + i];
    dst[j * ldd + i] = c128{(double)z.re, (double)z.im};
  }
}

__global__ void scale_lower_kernel(const c128* src, int64_t lds, c128* dst, int64_t ldd, int64_t m, int cols, double g) {
  const int64_t n = 2 * m;
  const int64_t total = n * cols;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / n, i = t % n;
    c128 z = src[j * lds + i];
    if (i >= m) { z.re *= g; z.im *= g; }
    dst[j * ldd + i] = z;
  }
}

__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Per column j: nu = ||V_j||, r_j = ||TZ_j - lam_j V_j|| / nu, V_j /= nu;
// optionally the residual vector of the unit Ritz vector, (TZ_j - lam_j V_j) / nu.
__global__ __launch_bounds__(256) void resid_kernel(c128* V, int64_t ldv, const c128* TZ, int64_t ldt, const double* lam,
                                                    int64_t n, double* resid, c128* R, int64_t ldr) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  c128* v = V + (int64_t)j * ldv;
  const c128* tz = TZ + (int64_t)j * ldt;
  const double l = lam[j];
  double s1 = 0, s2 = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const c128 a = v[i], b = tz[i];
    s1 += a.re * a.re + a.im * a.im;
    const double dr = b.re - l * a.re, di = b.im - l * a.im;
    s2 += dr * dr + di * di;
  }
  const double nu2 = block_sum(s1, red);
  const double rr2 = block_sum(s2, red);
  const double nu = sqrt(nu2);
  const double inv = nu > 0 ? 1.0 / nu : 0.0;
  c128* rv = R ? R + (int64_t)j * ldr : nullptr;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    c128 a = v[i];
    if (rv) {
      const c128 b = tz[i];
      rv[i] = c128{(b.re - l * a.re) * inv, (b.im - l * a.im) * inv};
    }
    v[i] = c128{a.re * inv, a.im * inv};
  }
  if (threadIdx.x == 0) resid[j] = sqrt(rr2) * inv;
}

// out[j] = Re(x_j^H y_j) over `rows` rows, rows from msplit on weighted by
// lsgn: lsgn = -1, msplit = m gives x^H S y on 2m rows, +1 the Euclidean
// product
__global__ __launch_bounds__(256) void sdot_kernel(const c128* X, int64_t ldx, const c128* Y, int64_t ldy, int64_t rows,
                                                   int64_t msplit, double lsgn, double* out) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  const c128* x = X + (int64_t)j * ldx;
  const c128* y = Y + (int64_t)j * ldy;
  double s = 0;
  for (int64_t i = threadIdx.x; i < rows; i += 256) {
    const double p = x[i].re * y[i].re + x[i].im * y[i].im;
    s += i < msplit ? p : lsgn * p;
  }
  const double r = block_sum(s, red);
  if (threadIdx.x == 0) out[j] = r;
}

// r = w - alpha v - beta v_prev  (per column scalars; beta_prev holds beta^2)
__global__ void lanczos_r_kernel(const c128* w, const c128* v, const c128* vp, c128* r, int64_t ld, int64_t n, int nv,
                                 const double* alpha, const double* beta_prev) {
  const int64_t total = n * nv;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / n);
    const int64_t o = (int64_t)j * ld + t % n;
    const double a = alpha[j], b = beta_prev ? sqrt(fmax(beta_prev[j], 0.0)) : 0.0;
    r[o] = c128{w[o].re - a * v[o].re - b * vp[o].re, w[o].im - a * v[o].im - b * vp[o].im};
  }
}

// vp <- v; v <- r / sqrt(bsq); w <- z / sqrt(bsq); beta <- sqrt(max(bsq, 0))
__global__ void lanczos_next_kernel(c128* vp, c128* v, c128* w, const c128* r, const c128* z, int64_t ld, int64_t n,
                                    int nv, const double* bsq, int shift_prev) {
  const int64_t total = n * nv;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / n);
    const int64_t o = (int64_t)j * ld + t % n;
    const double b = sqrt(fmax(bsq[j], 0.0));
    const double ib = b > 0 ? 1.0 / b : 0.0;
    if (shift_prev) vp[o] = v[o];
    v[o] = c128{r[o].re * ib, r[o].im * ib};
    w[o] = c128{z[o].re * ib, z[o].im * ib};
  }
}

// Adjoint operands from V (n x nev) and g: P = [x_i, conj(y_i)],
// P2 = [y_i, conj(x_i)], Pg = P * diag(gt, gt), gt_i = g_i / (|x_i|^2 - |y_i|^2).
__global__ void trace_kernel(const c128* G, int64_t ld, int k, double* out) {
  __shared__ double red[256];
  double s = 0;
  for (int i = threadIdx.x; i < k; i += 256) s += G[(int64_t)i * ld + i].re;
  const double r = block_sum(s, red);
  if (threadIdx.x == 0) *out = r;
}

// colmax[j] = max over i in [j, k) of |G_ij - delta_ij| (one workgroup per
// column j < k); then out = max_j colmax[j] (one workgroup).
__global__ __launch_bounds__(256) void gram_colmax_kernel(const c128* G, int64_t ld, int k, double* colmax) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double v = 0;
  for (int i = j + threadIdx.x; i < k; i += 256) {
    c128 g = G[(int64_t)j * ld + i];
    if (i == j) g.re -= 1.0;
    v = fmax(v, sqrt(g.re * g.re + g.im * g.im));
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) colmax[j] = red[0];
}

__global__ __launch_bounds__(256) void max_reduce_kernel(const double* x, int k, double* out) {
  __shared__ double red[256];
  double v = 0;
  for (int i = threadIdx.x; i < k; i += 256) v = fmax(v, x[i]);
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void diag_real_kernel(const c128* G, int64_t ld, int k, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) out[i] = G[(int64_t)i * ld + i].re;
}

__global__ void add_diag_kernel(c128* G, int64_t ld, int k, double s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) G[(int64_t)i * ld + i].re += s;
}

// dst[:, j] = src[:, perm[j]]
__global__ void gather_cols_kernel(const c128* src, int64_t lds, c128* dst, int64_t ldd, int64_t n, int k,
                                   const int* perm) {
  const int64_t total = n * k;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / n);
    const int64_t i = t % n;
    dst[(int64_t)j * ldd + i] = src[(int64_t)perm[j] * lds + i];
  }
}

// W[:, j] = pw[j] W[:, j] + ce D[:, j]   (W c128 in place, D c64)
__global__ void combine_kernel(c128* W, int64_t ldw, const c64* D, int64_t ldd, const double* pw, double ce, int64_t n,
                               int k) {
  const int64_t total = n * k;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / n);
    const int64_t i = t % n;
    const double p = pw[j];
    c128 w = W[(int64_t)j * ldw + i];
    const c64 d = D[(int64_t)j * ldd + i];
    W[(int64_t)j * ldw + i] = c128{p * w.re + ce * (double)d.re, p * w.im + ce * (double)d.im};
  }
}

__global__ void scale_c64_kernel(const c64* src, int64_t lds, c64* dst, int64_t ldd, int64_t rows, int cols, float a) {
  const int64_t total = rows * cols;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / rows, i = t % rows;
    const c64 z = src[j * lds + i];
    dst[j * ldd + i] = c64{a * z.re, a * z.im};
  }
}

// Real coordinates of the K-real parts of the search block's pairs.  For a
// vector x = [x1; x2] with J x = K conj(x) = [conj(x2); conj(x1)], the
// vectors u = (x + J x) / 2 and v = (x - J x) / (2i) satisfy J u = u,
// J v = v and span {x, J x} = span {u, v}.  A K-real vector [a; conj(a)] is
// stored by its real coordinates [Re a; Im a] (n reals, held in the real
// parts of a c128 column with zero imaginary parts); inner products of
// K-real vectors are twice the real inner products of their coordinates.
// Columns 2j, 2j + 1: u, v of S y_j (j < L), then u, v of w_j (j < kw).
__global__ void kreal_build_kernel(const c128* Y, int64_t ldy, int L, const c128* W, int64_t ldw, int kw, c128* X,
                                   int64_t ldx, int64_t m) {
  const int cols = 2 * L + 2 * kw;
  const int64_t total = m * cols;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t / m);
    const int64_t i = t % m;
    const int j = c / 2;
    const bool vpart = c & 1;
    c128 x1, x2;
    if (j < L) {
      x1 = Y[(int64_t)j * ldy + i];
      const c128 y2 = Y[(int64_t)j * ldy + m + i];
      x2 = c128{-y2.re, -y2.im};  // S y
    } else {
      x1 = W[(int64_t)(j - L) * ldw + i];
      x2 = W[(int64_t)(j - L) * ldw + m + i];
    }
    // top half a of u (x1 + conj(x2)) / 2 or of v (x1 - conj(x2)) / (2i)
    c128 a;
    if (!vpart) {
      a = c128{0.5 * (x1.re + x2.re), 0.5 * (x1.im - x2.im)};
    } else {
      const double dr = x1.re - x2.re, di = x1.im + x2.im;
      a = c128{0.5 * di, -0.5 * dr};
    }
    X[(int64_t)c * ldx + i] = c128{a.re, 0.0};
    X[(int64_t)c * ldx + m + i] = c128{a.im, 0.0};
  }
}

// In place, columns 2j and 2j + 1 (j < npair): (x, y) -> ((x + i y),
// (x - i y)) / sqrt(2), a unitary change of basis.
__global__ void pair_mix_kernel(c128* X, int64_t ldx, int64_t n, int npair) {
  const int64_t total = n * npair;
  const double h = 0.70710678118654752440;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / n, i = t % n;
    const c128 x = X[2 * j * ldx + i], y = X[(2 * j + 1) * ldx + i];
    X[2 * j * ldx + i] = c128{h * (x.re - y.im), h * (x.im + y.re)};
    X[(2 * j + 1) * ldx + i] = c128{h * (x.re + y.im), h * (x.im - y.re)};
  }
}

// Real coordinates sqrt(2) [Re a; Im a] of unit K-real columns [a; conj(a)]
// (the inverse of kreal_unpack).
__global__ void kreal_coords_kernel(const c128* Q, int64_t ldq, int64_t m, int k, c128* D, int64_t ldd) {
  const int64_t total = m * k;
  const double r2 = 1.41421356237309504880;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = t / m, i = t % m;
    const c128 a = Q[c * ldq + i];
    D[c * ldd + i] = c128{r2 * a.re, 0.0};
    D[c * ldd + m + i] = c128{r2 * a.im, 0.0};
  }
}

// x = e_r (n entries).
__global__ void unit_column_kernel(c128* x, int64_t n, int64_t r) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = c128{i == r ? 1.0 : 0.0, 0.0};
}

// In place: real coordinates [r1; r2] of unit length -> the unit K-real
// vector [a; conj(a)] / sqrt(2) with a = r1 + i r2.
__global__ void kreal_unpack_kernel(c128* X, int64_t ldx, int64_t m, int k) {
  const int64_t total = m * k;
  const double h = 0.70710678118654752440;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = t / m, i = t % m;
    const double r1 = X[c * ldx + i].re, r2 = X[c * ldx + m + i].re;
    X[c * ldx + i] = c128{h * r1, h * r2};
    X[c * ldx + m + i] = c128{h * r1, -h * r2};
  }
}

}  // namespace

Err kreal_build(const c128* Y, int64_t ldy, int L, const c128* W, int64_t ldw, int kw, c128* X, int64_t ldx, int64_t m,
                hipStream_t s) {
  const int64_t total = m * (2 * L + 2 * kw);
  if (total == 0) return ok();
  hipLaunchKernelGGL(kreal_build_kernel, dim3(grid_for(total)), dim3(256), 0, s, Y, ldy, L, W, ldw, kw, X, ldx, m);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err kreal_coords(const c128* Q, int64_t ldq, int64_t m, int k, c128* D, int64_t ldd, hipStream_t s) {
  if (m * k == 0) return ok();
  hipLaunchKernelGGL(kreal_coords_kernel, dim3(grid_for(m * k)), dim3(256), 0, s, Q, ldq, m, k, D, ldd);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err unit_column(c128* x, int64_t n, int64_t r, hipStream_t s) {
  hipLaunchKernelGGL(unit_column_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, r);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err pair_mix(c128* X, int64_t ldx, int64_t n, int npair, hipStream_t s) {
  if (n * npair == 0) return ok();
  hipLaunchKernelGGL(pair_mix_kernel, dim3(grid_for(n * npair)), dim3(256), 0, s, X, ldx, n, npair);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err kreal_unpack(c128* X, int64_t ldx, int64_t m, int k, hipStream_t s) {
  if (m * k == 0) return ok();
  hipLaunchKernelGGL(kreal_unpack_kernel, dim3(grid_for(m * k)), dim3(256), 0, s, X, ldx, m, k);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err scale_c64(const c64* src, int64_t lds, c64* dst, int64_t ldd, int64_t rows, int cols, float a, hipStream_t s) {
  if (rows * cols == 0) return ok();
  hipLaunchKernelGGL(scale_c64_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, s, src, lds, dst, ldd, rows, cols, a);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err combine_correction(c128* W, int64_t ldw, const c64* D, int64_t ldd, const double* dpw, double ce, int64_t n, int k,
                       hipStream_t s) {
  if (k == 0) return ok();
  hipLaunchKernelGGL(combine_kernel, dim3(grid_for(n * k)), dim3(256), 0, s, W, ldw, D, ldd, dpw, ce, n, k);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err convert_to_c64(const c128* src, int64_t lds, c64* dst, int64_t ldd, int64_t rows, int cols, hipStream_t s) {
  if (rows * cols == 0) return ok();
  hipLaunchKernelGGL(to_c64_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, s, src, lds, dst, ldd, rows, cols);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err convert_to_c128(const c64* src, int64_t lds, c128* dst, int64_t ldd, int64_t rows, int cols, hipStream_t s) {
  if (rows * cols == 0) return ok();
  hipLaunchKernelGGL(to_c128_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, s, src, lds, dst, ldd, rows, cols);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err scale_lower_half(const c128* src, int64_t lds, c128* dst, int64_t ldd, int64_t m, int cols, double g,
                     hipStream_t s) {
  if (cols == 0) return ok();
  hipLaunchKernelGGL(scale_lower_kernel, dim3(grid_for(2 * m * cols)), dim3(256), 0, s, src, lds, dst, ldd, m, cols, g);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err residual_norms(c128* V, int64_t ldv, const c128* TZ, int64_t ldt, const double* dlam, int64_t n, int kk,
                   double* dres, c128* R, int64_t ldr, hipStream_t s) {
  if (kk == 0) return ok();
  hipLaunchKernelGGL(resid_kernel, dim3(kk), dim3(256), 0, s, V, ldv, TZ, ldt, dlam, n, dres, R, ldr);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err s_dots(const c128* X, int64_t ldx, const c128* Y, int64_t ldy, int64_t m, int k, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sdot_kernel, dim3(k), dim3(256), 0, s, X, ldx, Y, ldy, 2 * m, m, -1.0, out);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err plain_dots(const c128* X, int64_t ldx, const c128* Y, int64_t ldy, int64_t m, int k, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sdot_kernel, dim3(k), dim3(256), 0, s, X, ldx, Y, ldy, 2 * m, 2 * m, 1.0, out);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err row_dots(const c128* X, int64_t ldx, const c128* Y, int64_t ldy, int64_t rows, int k, double* out,
             hipStream_t s) {
  hipLaunchKernelGGL(sdot_kernel, dim3(k), dim3(256), 0, s, X, ldx, Y, ldy, rows, rows, 1.0, out);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err lanczos_residual(const c128* w, const c128* v, const c128* vp, c128* r, int64_t ld, int64_t n, int nv,
                     const double* alpha, const double* beta_prev, hipStream_t s) {
  hipLaunchKernelGGL(lanczos_r_kernel, dim3(grid_for(n * nv)), dim3(256), 0, s, w, v, vp, r, ld, n, nv, alpha,
                     beta_prev);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err lanczos_advance(c128* vp, c128* v, c128* w, const c128* r, const c128* z, int64_t ld, int64_t n, int nv,
                    const double* bsq, bool shift_prev, hipStream_t s) {
  hipLaunchKernelGGL(lanczos_next_kernel, dim3(grid_for(n * nv)), dim3(256), 0, s, vp, v, w, r, z, ld, n, nv, bsq,
                     shift_prev ? 1 : 0);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err trace(const c128* G, int64_t ld, int k, double* dout, hipStream_t s) {
  hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(256), 0, s, G, ld, k, dout);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err gram_deviation(const c128* G, int64_t ld, int k, double* colmax, double* dout, hipStream_t s) {
  if (k <= 0) return ok();
  hipLaunchKernelGGL(gram_colmax_kernel, dim3(k), dim3(256), 0, s, G, ld, k, colmax);
  CHASE_LAUNCH_CHECK();
  hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(256), 0, s, (const double*)colmax, k, dout);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err diag_real(const c128* G, int64_t ld, int k, double* dout, hipStream_t s) {
  if (k == 0) return ok();
  hipLaunchKernelGGL(diag_real_kernel, dim3((unsigned)ceil_div(k, 256)), dim3(256), 0, s, G, ld, k, dout);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err add_diag(c128* G, int64_t ld, int k, double v, hipStream_t s) {
  hipLaunchKernelGGL(add_diag_kernel, dim3((unsigned)ceil_div(k, 256)), dim3(256), 0, s, G, ld, k, v);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err gather_columns(const c128* src, int64_t lds, c128* dst, int64_t ldd, int64_t n, int k, const int* dperm,
                   hipStream_t s) {
  if (k == 0) return ok();
  hipLaunchKernelGGL(gather_cols_kernel, dim3(grid_for(n * k)), dim3(256), 0, s, src, lds, dst, ldd, n, k, dperm);
  CHASE_LAUNCH_CHECK();
  return ok();
}

}  // namespace chase
