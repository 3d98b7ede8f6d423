// Eigenvalues and right eigenvectors of a small dense complex matrix, for
// the non-hermitian back-up Rayleigh quotient of Section 5.3 (whose Ritz
// values are complex).  Three phases, after Golub & Van Loan, Matrix
// Computations (4th ed.), Sections 7.4-7.6:
//   1. Householder reduction to upper Hessenberg form, G = Z H Z^H (one
//      reflector per column: a reflector launch, a left-application launch
//      with one workgroup per column and a right-application launch with
//      one workgroup per 64 rows of G and of Z);
//   2. the implicit single-shift complex QR algorithm on H with Wilkinson
//      shifts, exceptional shifts after 10 and 20 iterations without
//      deflation, and deflation of negligible subdiagonal entries, which
//      leaves the upper-triangular Schur factor T in place and accumulates
//      the rotations into Z.  One workgroup: every Givens step of a bulge
//      chase is one barrier; all threads derive the same rotation from the
//      same two entries (handed over in LDS by the step that produced
//      them), then update disjoint entries of the two rows, the two columns
//      and Z;
//   3. eigenvectors of T by back-substitution (one thread per eigenvector,
//      tiny pivots raised to ulp |lambda|), then V = Z Y by the c128 GEMM.
// The selection of the positive half runs on the device too.
#include <algorithm>
#include <cfloat>

#include "geev.h"

namespace chase {
namespace {

__device__ __forceinline__ c128 zadd(c128 a, c128 b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ c128 zsub(c128 a, c128 b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ c128 zmul(c128 a, c128 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ c128 zconj(c128 a) { return {a.re, -a.im}; }
__device__ __forceinline__ c128 zscale(double s, c128 a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ double zabs1(c128 a) { return fabs(a.re) + fabs(a.im); }

// a / b by Smith's scaling (no overflow for moderate quotients)
__device__ __forceinline__ c128 zdiv(c128 a, c128 b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const double r = b.re / b.im, d = b.re * r + b.im;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}

// principal square root
__device__ __forceinline__ c128 zsqrt(c128 a) {
  const double r = hypot(a.re, a.im);
  if (r == 0.0) return {0.0, 0.0};
  if (a.re >= 0.0) {
    const double t = sqrt(0.5 * (r + a.re));
    return {t, a.im / (2.0 * t)};
  }
  const double t = sqrt(0.5 * (r - a.re));
  return {fabs(a.im) / (2.0 * t), copysign(t, a.im)};
}

constexpr double ULP = 2.220446049250313e-16;
constexpr double SAFMIN = DBL_MIN;
constexpr int RT = 256;        // threads of the reflector / left-application workgroups
constexpr int QR_THREADS = 1024;

__device__ __forceinline__ double block_sum(double v, double* red) {
  // RT threads; red has RT / 64 slots
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < RT / 64; ++i) s += red[i];
  return s;
}

__device__ __forceinline__ c128 block_sum(c128 v, double* red) {
  const double re = block_sum(v.re, red);
  const double im = block_sum(v.im, red);
  return {re, im};
}

// Reflector for column j: x = G[j+1:k, j] -> beta e_1 with
// P = I - tau v v^H, v = x - beta e_1, beta = -(x_0 / |x_0|) ||x||,
// tau = 2 / (v^H v) (tau = 0 when x is already a multiple of e_1).
// Writes v (length k - j - 1) and tau, and the reduced column.
__global__ __launch_bounds__(RT) void hess_reflector_kernel(c128* G, int64_t ld, int k, int j, c128* v,
                                                            double* tau) {
  __shared__ double red[RT / 64];
  const int len = k - j - 1;
  c128* x = G + (int64_t)j * ld + j + 1;
  double s = 0.0;
  for (int r = 1 + threadIdx.x; r < len; r += RT) s += x[r].re * x[r].re + x[r].im * x[r].im;
  s = block_sum(s, red);
  const c128 x0 = x[0];
  const double a0 = hypot(x0.re, x0.im);
  if (s == 0.0) {
    if (threadIdx.x == 0) *tau = 0.0;
    return;
  }
  const double xn = sqrt(a0 * a0 + s);
  const c128 ph = a0 > 0.0 ? c128{x0.re / a0, x0.im / a0} : c128{1.0, 0.0};
  const c128 beta = zscale(-xn, ph);
  for (int r = threadIdx.x; r < len; r += RT) {
    v[r] = r == 0 ? zsub(x0, beta) : x[r];
  }
  __syncthreads();  // every v[r] is read from x before x is overwritten
  for (int r = threadIdx.x; r < len; r += RT) x[r] = r == 0 ? beta : c128{0.0, 0.0};
  if (threadIdx.x == 0) {
    const c128 v0 = zsub(x0, beta);
    *tau = 2.0 / (v0.re * v0.re + v0.im * v0.im + s);
  }
}

// G[j+1:k, c] -= tau v (v^H G[j+1:k, c]) for c = j+1 .. k-1 (one workgroup
// per column).
__global__ __launch_bounds__(RT) void hess_left_kernel(c128* G, int64_t ld, int k, int j, const c128* v,
                                                       const double* tau) {
  __shared__ double red[RT / 64];
  const double t = *tau;
  if (t == 0.0) return;
  const int len = k - j - 1;
  c128* col = G + (int64_t)(j + 1 + blockIdx.x) * ld + j + 1;
  c128 d{0.0, 0.0};
  for (int r = threadIdx.x; r < len; r += RT) d = zadd(d, zmul(zconj(v[r]), col[r]));
  d = zscale(t, block_sum(d, red));
  for (int r = threadIdx.x; r < len; r += RT) col[r] = zsub(col[r], zmul(v[r], d));
}

// M[r, j+1:k] -= tau (M[r, j+1:k] v) v^H for every row r of G (blockIdx.y
// = 0) and of Z (blockIdx.y = 1); 64 rows per workgroup, four column
// groups of 64 lanes.
__global__ __launch_bounds__(RT) void hess_right_kernel(c128* G, c128* Z, int64_t ld, int k, int j, const c128* v,
                                                        const double* tau) {
  __shared__ c128 part[RT];
  const double t = *tau;
  if (t == 0.0) return;
  c128* M = blockIdx.y == 0 ? G : Z;
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int r = blockIdx.x * 64 + lane;
  const int len = k - j - 1;
  c128* row0 = M + (int64_t)(j + 1) * ld;
  c128 u{0.0, 0.0};
  if (r < k)
    for (int c = grp; c < len; c += RT / 64) u = zadd(u, zmul(row0[(int64_t)c * ld + r], v[c]));
  part[threadIdx.x] = u;
  __syncthreads();
  u = c128{0.0, 0.0};
#pragma unroll
  for (int g = 0; g < RT / 64; ++g) u = zadd(u, part[g * 64 + lane]);
  u = zscale(t, u);
  if (r < k)
    for (int c = grp; c < len; c += RT / 64) {
      c128* p = row0 + (int64_t)c * ld + r;
      *p = zsub(*p, zmul(u, zconj(v[c])));
    }
}

// Rotation [[c, s], [-conj(s), c]] (c real) taking (x, y) to (r, 0).
__device__ __forceinline__ void givens(c128 x, c128 y, double& c, c128& s) {
  const double ax = hypot(x.re, x.im), ay = hypot(y.re, y.im);
  if (ay == 0.0) {
    c = 1.0;
    s = {0.0, 0.0};
  } else if (ax == 0.0) {
    c = 0.0;
    s = {1.0, 0.0};
  } else {
    const double rho = hypot(ax, ay);
    c = ax / rho;
    s = zscale(1.0 / (ax * rho), zmul(x, zconj(y)));
  }
}

// Wilkinson shift: the eigenvalue of [[a, b], [cc, d]] nearer to d,
// d - b cc / (p + sqrt(p^2 + b cc)), p = (a - d) / 2, root sign taken so
// that the denominator has the larger modulus.
__device__ __forceinline__ c128 wilkinson(c128 a, c128 b, c128 cc, c128 d) {
  const c128 p = zscale(0.5, zsub(a, d));
  const c128 bc = zmul(b, cc);
  c128 disc = zsqrt(zadd(zmul(p, p), bc));
  if (p.re * disc.re + p.im * disc.im < 0.0) disc = zscale(-1.0, disc);
  const c128 den = zadd(p, disc);
  if (den.re == 0.0 && den.im == 0.0) return d;
  return zsub(d, zdiv(bc, den));
}

// Schur form of the upper Hessenberg H (k x k, in place) with the rotations
// accumulated into Z; w gets the eigenvalues (diagonal of T).  *status = 1
// when a block does not deflate within 30 iterations or the total exceeds
// max_sweeps (T, Z then unspecified).  Every branch condition is uniform
// (derived from values read after a barrier), so all threads leave together.
__global__ __launch_bounds__(QR_THREADS) void hqr_kernel(c128* H, c128* Z, int64_t ld, int k, c128* w, int* status,
                                                         int max_sweeps) {
  __shared__ int s_l;
  __shared__ c128 s_xy[2][2];  // next rotation's inputs, by step parity
  const int tid = threadIdx.x;
  auto at = [&](int r, int c) -> c128& { return H[(int64_t)c * ld + r]; };
  int hi = k - 1, its = 0, total = 0;
  if (tid == 0) *status = 0;
  while (hi >= 0) {
    if (tid == 0) s_l = 0;
    __syncthreads();
    for (int l = hi - tid; l >= 1; l -= QR_THREADS) {
      const c128 sub = at(l, l - 1);
      double tst = zabs1(at(l - 1, l - 1)) + zabs1(at(l, l));
      if (tst == 0.0) tst = 1.0;
      if (zabs1(sub) <= fmax(ULP * tst, SAFMIN)) atomicMax(&s_l, l);
    }
    __syncthreads();
    const int l = s_l;
    __syncthreads();
    if (l > 0 && tid == 0) at(l, l - 1) = c128{0.0, 0.0};
    if (l == hi) {
      if (tid == 0) w[hi] = at(hi, hi);
      --hi;
      its = 0;
      __syncthreads();
      continue;
    }
    if (its >= 30 || total >= max_sweeps) {
      if (tid == 0) *status = 1;
      break;
    }
    c128 mu;
    if (its == 10 || its == 20) {
      mu = zadd(at(hi, hi), c128{0.75 * zabs1(at(hi, hi - 1)), 0.0});
    } else {
      mu = wilkinson(at(hi - 1, hi - 1), at(hi - 1, hi), at(hi, hi - 1), at(hi, hi));
    }
    // the first rotation's inputs, read by every thread before any update
    const c128 x0 = zsub(at(l, l), mu), y0 = at(l + 1, l);
    __syncthreads();
    for (int j = l; j < hi; ++j) {
      // later rotations take (H[j][j-1], H[j+1][j-1]) from the slot the
      // previous step filled, so that this step's updates of those entries
      // cannot race with their reads
      const c128 x = j == l ? x0 : s_xy[j & 1][0];
      const c128 y = j == l ? y0 : s_xy[j & 1][1];
      double c;
      c128 s;
      givens(x, y, c, s);
      const c128 sc = zconj(s);
      // rows j, j+1 (left rotation) over columns cs .. k-1 except j, j+1
      const int cs = j == l ? l : j - 1;
      const int rmax = min(j + 2, hi);
      const int nrow = k - cs;               // row-rotation items
      const int ncol = rmax + 1;             // column-rotation items (rows 0 .. rmax)
      for (int t = tid; t < nrow + ncol + k + 1; t += QR_THREADS) {
        if (t < nrow) {
          const int cc = cs + t;
          if (cc == j || cc == j + 1) continue;
          const c128 a = at(j, cc), b = at(j + 1, cc);
          at(j, cc) = zadd(zscale(c, a), zmul(s, b));
          at(j + 1, cc) = (j > l && cc == j - 1) ? c128{0.0, 0.0} : zsub(zscale(c, b), zmul(sc, a));
        } else if (t < nrow + ncol) {
          const int r = t - nrow;
          if (r == j || r == j + 1) continue;
          const c128 a = at(r, j), b = at(r, j + 1);
          const c128 rj = zadd(zscale(c, a), zmul(sc, b));
          at(r, j) = rj;
          at(r, j + 1) = zsub(zscale(c, b), zmul(s, a));
          if (r == j + 2) s_xy[(j + 1) & 1][1] = rj;  // the bulge, next step's y
        } else if (t < nrow + ncol + k) {
          const int r = t - nrow - ncol;
          c128* z0 = Z + (int64_t)j * ld + r;
          c128* z1 = z0 + ld;
          const c128 a = *z0, b = *z1;
          *z0 = zadd(zscale(c, a), zmul(sc, b));
          *z1 = zsub(zscale(c, b), zmul(s, a));
        } else {
          // the 2 x 2 block of rows and columns j, j+1: left then right
          c128 a00 = at(j, j), a01 = at(j, j + 1), a10 = at(j + 1, j), a11 = at(j + 1, j + 1);
          const c128 b00 = zadd(zscale(c, a00), zmul(s, a10)), b10 = zsub(zscale(c, a10), zmul(sc, a00));
          const c128 b01 = zadd(zscale(c, a01), zmul(s, a11)), b11 = zsub(zscale(c, a11), zmul(sc, a01));
          at(j, j) = zadd(zscale(c, b00), zmul(sc, b01));
          at(j, j + 1) = zsub(zscale(c, b01), zmul(s, b00));
          const c128 n10 = zadd(zscale(c, b10), zmul(sc, b11));
          at(j + 1, j) = n10;
          at(j + 1, j + 1) = zsub(zscale(c, b11), zmul(s, b10));
          s_xy[(j + 1) & 1][0] = n10;  // next step's x
        }
      }
      __syncthreads();
    }
    ++its;
    ++total;
  }
  __syncthreads();
}

// Eigenvectors of the upper-triangular T: thread i solves
// (T - t_ii I) y = 0 with y_i = 1, y_c = 0 for c > i, by back-substitution
// from row i - 1 up; a pivot |t_rr - t_ii| below smin = max(ulp |t_ii|,
// safmin) is replaced by smin.  The work vector is stored transposed
// (Yt[i + c k], coalesced across the threads of a block) and rescaled by
// 1e-150 when an entry exceeds 1e150; the column is
// finally written to Y (ld ldy).
__global__ __launch_bounds__(64) void trevc_kernel(const c128* T, int64_t ld, int k, c128* Yt, c128* Y,
                                                   int64_t ldy) {
  const int i0 = blockIdx.x * 64, i = i0 + threadIdx.x;
  const int imax = min(i0 + 63, k - 1);
  const bool act = i < k;
  const c128 lam = act ? T[(int64_t)i * ld + i] : c128{0.0, 0.0};
  const double smin = fmax(ULP * zabs1(lam), SAFMIN);
  if (act)
    for (int c = i0; c <= imax; ++c) Yt[(int64_t)c * k + i] = c == i ? c128{1.0, 0.0} : c128{0.0, 0.0};
  for (int r = imax - 1; r >= 0; --r) {
    if (!act || r >= i) continue;
    c128 acc{0.0, 0.0};
    for (int c = r + 1; c <= i; ++c) acc = zadd(acc, zmul(T[(int64_t)c * ld + r], Yt[(int64_t)c * k + i]));
    c128 d = zsub(T[(int64_t)r * ld + r], lam);
    if (zabs1(d) < smin) d = c128{smin, 0.0};
    const c128 yr = zscale(-1.0, zdiv(acc, d));
    Yt[(int64_t)r * k + i] = yr;
    // repeated tiny pivots (equal eigenvalues) make y grow geometrically:
    // scale the entries found so far down before they can overflow (the
    // eigenvector is defined up to scale)
    if (zabs1(yr) > 1e150)
      for (int c = r; c <= i; ++c) Yt[(int64_t)c * k + i] = zscale(1e-150, Yt[(int64_t)c * k + i]);
  }
  if (act)
    for (int c = 0; c < k; ++c) Y[(int64_t)i * ldy + c] = c <= i ? Yt[(int64_t)c * k + i] : c128{0.0, 0.0};
}

__global__ void eye_kernel(c128* Z, int64_t ld, int k) {
  const int64_t total = (int64_t)k * k;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t / k), r = (int)(t % k);
    Z[(int64_t)c * ld + r] = c128{r == c ? 1.0 : 0.0, 0.0};
  }
}

// Rank of each eigenvalue by real part (ties by index) and the count p of
// non-positive real parts.  Slots 0 .. np - 1 (np = min(k/2, k - p)) take
// the smallest positive real parts ascending (rank p + slot); the remaining
// k/2 - np slots take the largest non-positive ones, descending (rank
// p - 1 - (slot - np)).  sel[slot] = i, lam[slot] = Re w_i.
__global__ void rank_select_kernel(const c128* w, int k, int* sel, double* lam) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const double wi = w[i].re;
  int rank = 0, p = 0;
  for (int j = 0; j < k; ++j) {
    const double wj = w[j].re;
    rank += (wj < wi || (wj == wi && j < i)) ? 1 : 0;
    p += wj <= 0.0 ? 1 : 0;
  }
  const int half = k / 2, np = min(half, k - p);
  int pos = -1;
  if (rank >= p && rank - p < np) pos = rank - p;
  else if (rank < p && p - 1 - rank < half - np) pos = np + (p - 1 - rank);
  if (pos >= 0) {
    sel[pos] = i;
    lam[pos] = wi;
  }
}

__global__ void gather_cols_kernel(const c128* V, int64_t ldv, int k, const int* sel, int nsel, c128* out,
                                   int64_t ldo) {
  const int64_t total = (int64_t)k * nsel;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t / k), r = (int)(t % k);
    int j = sel[c];
    if (j < 0 || j >= k) j = 0;  // non-finite eigenvalues leave gaps in the ranking
    out[(int64_t)c * ldo + r] = V[(int64_t)j * ldv + r];
  }
}

__global__ void backup_diag_kernel(c128* N, int64_t ld, int k, double dmin, double* d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  c128* p = N + (int64_t)i * ld + i;
  double di = p->re;
  if (fabs(di) < dmin) di = 1.0;
  d[i] = di;
  p->re -= di;
}

__global__ void scale_rows_inv_kernel(c128* G, int64_t ld, int k, const double* d) {
  const int64_t total = (int64_t)k * k;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t / k), r = (int)(t % k);
    c128* p = G + (int64_t)c * ld + r;
    *p = zscale(1.0 / d[r], *p);
  }
}

}  // namespace

__global__ void conj_transpose_kernel(const c128* src, int64_t lds, c128* dst, int64_t ldd, int k) {
  const int64_t total = (int64_t)k * k;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / k, i = t % k;  // dst(i, j) = conj(src(j, i))
    const c128 z = src[i * lds + j];
    dst[j * ldd + i] = c128{z.re, -z.im};
  }
}

Err conj_transpose(const c128* src, int64_t lds, c128* dst, int64_t ldd, int k, hipStream_t s) {
  if (k <= 0) return ok();
  const int64_t total = (int64_t)k * k;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(conj_transpose_kernel, dim3(blocks), dim3(256), 0, s, src, lds, dst, ldd, k);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err backup_diag(c128* N, int64_t ld, int k, double dmin, double* d, hipStream_t s) {
  if (k <= 0) return ok();
  hipLaunchKernelGGL(backup_diag_kernel, dim3((unsigned)ceil_div(k, 256)), dim3(256), 0, s, N, ld, k, dmin, d);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err scale_rows_inv(c128* G, int64_t ld, int k, const double* d, hipStream_t s) {
  if (k <= 0) return ok();
  const int nb = (int)std::min<int64_t>(1024, ceil_div((int64_t)k * k, 256));
  hipLaunchKernelGGL(scale_rows_inv_kernel, dim3(nb), dim3(256), 0, s, G, ld, k, d);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err nonsym_eig(c128* G, c128* Z, int64_t ld, int k, c128* w, c128* Yt, c128* Y, const GeevWs& ws, hipStream_t s,
               int* qr_status) {
  if (k <= 0) return ok();
  const int eb = (int)std::min<int64_t>(1024, ceil_div((int64_t)k * k, 256));
  hipLaunchKernelGGL(eye_kernel, dim3(eb), dim3(256), 0, s, Z, ld, k);
  CHASE_LAUNCH_CHECK();
  for (int j = 0; j + 2 < k; ++j) {
    hipLaunchKernelGGL(hess_reflector_kernel, dim3(1), dim3(RT), 0, s, G, ld, k, j, ws.v, ws.tau);
    CHASE_LAUNCH_CHECK();
    hipLaunchKernelGGL(hess_left_kernel, dim3(k - j - 1), dim3(RT), 0, s, G, ld, k, j, (const c128*)ws.v,
                       (const double*)ws.tau);
    CHASE_LAUNCH_CHECK();
    hipLaunchKernelGGL(hess_right_kernel, dim3((unsigned)ceil_div(k, 64), 2), dim3(RT), 0, s, G, Z, ld, k, j,
                       (const c128*)ws.v, (const double*)ws.tau);
    CHASE_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(hqr_kernel, dim3(1), dim3(QR_THREADS), 0, s, G, Z, ld, k, w, ws.status,
                     std::max(100, 10 * k));
  CHASE_LAUNCH_CHECK();
  CHASE_HIP(hipMemcpyAsync(qr_status, ws.status, sizeof(int), hipMemcpyDeviceToHost, s));
  CHASE_HIP(hipStreamSynchronize(s));
  if (*qr_status != 0) return ok();
  hipLaunchKernelGGL(trevc_kernel, dim3((unsigned)ceil_div(k, 64)), dim3(64), 0, s, (const c128*)G, ld, k, Yt, Y,
                     ld);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err select_by_real_part(const c128* w, int k, const c128* V, int64_t ldv, int* sel, double* lam, c128* out,
                        int64_t ldo, hipStream_t s) {
  if (k < 2) return ok();
  hipLaunchKernelGGL(rank_select_kernel, dim3((unsigned)ceil_div(k, 256)), dim3(256), 0, s, w, k, sel, lam);
  CHASE_LAUNCH_CHECK();
  const int nb = (int)std::min<int64_t>(1024, ceil_div((int64_t)k * (k / 2), 256));
  hipLaunchKernelGGL(gather_cols_kernel, dim3(nb), dim3(256), 0, s, V, ldv, k, (const int*)sel, k / 2, out, ldo);
  CHASE_LAUNCH_CHECK();
  return ok();
}

}  // namespace chase
