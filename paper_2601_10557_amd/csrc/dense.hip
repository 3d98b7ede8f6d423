// Small dense FP64 kernels of the QR and Rayleigh-Ritz steps (Section 2:
// Cholesky QR; Alg. 2: POTRF, TRSM, HEEVD).  All operate on k x k Hermitian
// or triangular matrices stored in a padded kp x kp buffer (kp a multiple of
// 64, leading dimension kp) so that every blocked step has uniform sizes:
//  * Cholesky  M = L L^H, right-looking, 64-column panels;
//  * triangular inverse L^{-1}, by block diagonals of batched GEMMs;
//  * Hermitian eigensolver: block Jacobi with 16-column blocks; each pair of
//    blocks (a 32 x 32 subproblem) gets one cyclic Jacobi sweep in LDS and
//    the block rotations are applied to the matrix and the eigenvectors with
//    32 x 32 complex products.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "common.h"
#include "dense.h"

namespace chase {
namespace {

constexpr int NB = 64;   // panel / padding granularity
constexpr int JB = 16;   // Jacobi block (subproblem is 2*JB)
constexpr int SP = 2 * JB;

__device__ __forceinline__ c128 cmul(c128 a, c128 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ c128 cconj(c128 a) { return {a.re, -a.im}; }
__device__ __forceinline__ c128 cadd(c128 a, c128 b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ c128 csub(c128 a, c128 b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ c128 cscale(double s, c128 a) { return {s * a.re, s * a.im}; }
// r - a b and r - a conj(b), as four fused multiply-adds each
__device__ __forceinline__ c128 cfms(c128 r, c128 a, c128 b) {
  return {fma(-a.re, b.re, fma(a.im, b.im, r.re)), fma(-a.re, b.im, fma(-a.im, b.re, r.im))};
}
__device__ __forceinline__ c128 cfms_conj(c128 r, c128 a, c128 b) {
  return {fma(-a.re, b.re, fma(-a.im, b.im, r.re)), fma(a.re, b.im, fma(-a.im, b.re, r.im))};
}

// ---------------------------------------------------------------- fills
__global__ void fill_diag_kernel(c128* M, int64_t ld, int kp, int k, double inner, double pad, int zero_all) {
  const int64_t total = (int64_t)kp * kp;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / kp), i = (int)(t % kp);
    c128* p = M + (int64_t)j * ld + i;
    if (i == j) {
      *p = c128{i < k ? inner : pad, 0.0};
    } else if (zero_all || i >= k || j >= k) {
      *p = c128{0.0, 0.0};
    }
  }
}

// Zero the strict upper triangle (used after the blocked Cholesky, whose
// trailing updates also touch the upper part).
__global__ void zero_upper_kernel(c128* M, int64_t ld, int kp) {
  const int64_t total = (int64_t)kp * kp;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / kp), i = (int)(t % kp);
    if (i < j) M[(int64_t)j * ld + i] = c128{0.0, 0.0};
  }
}

// ------------------------------------------------------- Cholesky block
// 64 x 64 diagonal blocks, 256 threads.  Lane i of every wave holds row i
// (Cholesky) or column i (inverse), and wave w the 16 columns (rows)
// w, w + 4, ..., w + 60 in registers: interleaved, so that the four waves
// share the shrinking trailing part evenly.  A step publishes one column
// (row) through LDS, on rotating buffers, so it takes one barrier, and
// every other operand of the step is a broadcast LDS read.
constexpr int CT = 256;     // threads of the block kernels
constexpr int CW = NB / 4;  // columns (rows) per wave

// Lane exchange inside a row of 16 lanes by DPP (no LDS round trip).
template <int CTRL>
__device__ __forceinline__ double dpp_swap(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lane l of each row of 16 lanes takes the value of lane (l + 1) mod 16
// (DPP row_ror:15).
__device__ __forceinline__ double row_next(double x) { return dpp_swap<0x12F>(x); }

// f(std::integral_constant<int, B>), ..., f(std::integral_constant<int, E - 1>)
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// 1 / sqrt(y) and 1 / d for normal positive y and nonzero d: hardware
// estimates refined by two Newton steps each (r <- r (3 - y r^2) / 2 and
// q <- q (2 - d q)), which take the estimate to within about an ulp.
__device__ __forceinline__ double rsqrt_nr(double y) {
  double r = __builtin_amdgcn_rsq(y);
  r = r * (1.5 - 0.5 * y * r * r);
  r = r * (1.5 - 0.5 * y * r * r);
  return r;
}

__device__ __forceinline__ double rcp_nr(double d) {
  double q = __builtin_amdgcn_rcp(d);
  q = q * (2.0 - d * q);
  q = q * (2.0 - d * q);
  return q;
}

// Lower Cholesky A = L L^H of the block and its inverse X = L^{-1}, run as
// one sweep of 64 column steps with one barrier each.
//  * Cholesky, right-looking in LDL^H form: step j takes the pivot
//    d_j = A[j][j] and applies A[i][l] -= A[i][j] conj(A[l][j]) / d_j for
//    j < l <= i; thread (w, i) holds A[i][4 t + w] in r[t], and the columns
//    are scaled by 1 / sqrt(d_j) at the end.
//  * Inverse, forward substitution on the 64 unit right-hand sides one step
//    behind: step j finishes row j - 1 of X (x = b / L[j-1][j-1], on wave
//    (j - 1) mod 4) and every wave updates its rows r > j - 1 by
//    b_r -= L[r][j-1] x with column j - 1 of L (published the step before);
//    thread (w, c) holds X[4 t + w][c] in b[t].
// A step publishes column j (and row j - 1 of X) through LDS, the columns
// triple-buffered since a step reads the last two.  A non-positive or
// non-finite pivot is replaced by 1 so that the block stays finite (the
// caller flags it and discards the result).  On return r holds the
// unscaled columns, b the inverse, dpiv the raw pivots and rsq[j] =
// 1 / sqrt(d_j) (1 for a replaced pivot).
__device__ __forceinline__ void chol_inv64(c128 (&r)[CW], c128 (&b)[CW], c128 (*colb)[NB], c128 (*xb)[NB],
                                           double* dpiv, double* rsq) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
  for (int t = 0; t < CW; ++t) b[t] = (4 * t + w == lane) ? c128{1.0, 0.0} : c128{0.0, 0.0};
  double rs_prev = 1.0;  // 1 / sqrt(d_{j-1})
  // slot tj unrolled (register indices stay static), owner wave wj not
#pragma unroll
  for (int tj = 0; tj < CW; ++tj) {
#pragma unroll 1
    for (int wj = 0; wj < 4; ++wj) {
      const int j = 4 * tj + wj;
      const int k = j - 1;                  // row of X finished in this step
      const int tk0 = tj > 0 ? tj - 1 : 0;  // its slot: tk0 (wj = 0) or tj
      c128* col = colb[j % 3];
      if (w == wj) col[lane] = r[tj];  // column j, final since step j - 1
      if (k >= 0 && w == (k & 3)) {
        if (wj == 0) {
          b[tk0] = cscale(rs_prev, b[tk0]);
          xb[k & 1][lane] = b[tk0];
        } else {
          b[tj] = cscale(rs_prev, b[tj]);
          xb[k & 1][lane] = b[tj];
        }
      }
      __syncthreads();
      const double draw = col[j].re;
      const double d = (draw > 0.0 && isfinite(draw)) ? draw : 1.0;
      if (threadIdx.x == 0) {
        dpiv[j] = draw;
        rsq[j] = rsqrt_nr(d);
      }
      const c128 s = cscale(rcp_nr(d), col[lane]);
      // all reads of the step first, so that their latencies overlap
      c128 c[CW], l[CW];
#pragma unroll
      for (int t = tj; t < CW; ++t) c[t] = col[4 * t + w];
      c128 x{0.0, 0.0};
      if (k >= 0) {
        // x_{j-1} times the column scale of L[:, j-1]
        x = cscale(rs_prev, xb[k & 1][lane]);
        const c128* colk = colb[(j + 2) % 3];
#pragma unroll
        for (int t = tk0; t < CW; ++t) l[t] = colk[4 * t + w];
      }
      // columns l > j, all rows: the entries above the diagonal (l > i) take
      // updates too but are never read for an entry on or below it
#pragma unroll
      for (int t = tj; t < CW; ++t)
        if (t > tj || w > wj) r[t] = cfms_conj(r[t], s, c[t]);
      if (k >= 0) {
#pragma unroll
        for (int t = tk0; t < CW; ++t)
          if (4 * t + w > k) b[t] = cfms(b[t], l[t], x);
      }
      rs_prev = rsqrt_nr(d);
    }
  }
  // row 63 of X: its last update came with step 63
  if (w == 3) b[CW - 1] = cscale(rs_prev, b[CW - 1]);
}

// X = L^{-1} by forward substitution on the 64 unit right-hand sides at
// once: thread (w, c) holds X[4 t + w][c] in b[t]; step k finishes row k
// (x_k = b_k / L[k][k]) on wave k mod 4, which publishes it, and every
// wave updates its rows r > k by b_r -= L[r][k] x_k.  L (lower) is read
// from S, its reciprocal diagonal from rpiv.
__device__ __forceinline__ void trinv64(const c128 (*S)[NB + 1], const double* rpiv, c128 (*xb)[NB],
                                        c128 (&b)[CW]) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
  for (int t = 0; t < CW; ++t) b[t] = (4 * t + w == lane) ? c128{1.0, 0.0} : c128{0.0, 0.0};
#pragma unroll
  for (int tk = 0; tk < CW; ++tk) {
#pragma unroll 1
    for (int wk = 0; wk < 4; ++wk) {
      const int k = 4 * tk + wk;
      c128* xr = xb[k & 1];
      if (w == wk) {
        b[tk] = cscale(rpiv[k], b[tk]);
        xr[lane] = b[tk];
      }
      __syncthreads();
      const c128 x = xr[lane];
      c128 l[CW];
#pragma unroll
      for (int t = tk; t < CW; ++t) l[t] = S[4 * t + w][k];
#pragma unroll
      for (int t = tk; t < CW; ++t)
        if (t > tk || w > wk) b[t] = cfms(b[t], l[t], x);
    }
  }
}

// Factor the 64 x 64 diagonal block at (p, p): writes L_pp (lower, upper
// zeroed) in place and L_pp^{-1} into inv (64 x 64, ld 64).
__global__ __launch_bounds__(CT) void potrf_diag_kernel(c128* M, int64_t ld, int p, c128* inv, int* fail) {
  __shared__ c128 S[NB][NB + 1];
  __shared__ c128 colb[3][NB];
  __shared__ c128 xb[2][NB];
  __shared__ double dpiv[NB];
  __shared__ double rsq[NB];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  c128 r[CW], b[CW];
#pragma unroll
  for (int t = 0; t < CW; ++t) r[t] = M[(int64_t)(p + 4 * t + w) * ld + p + lane];
  chol_inv64(r, b, colb, xb, dpiv, rsq);
  __syncthreads();
#pragma unroll
  for (int t = 0; t < CW; ++t) {
    const int l = 4 * t + w;
    const double dl = dpiv[l];
    const bool ok = dl > 0.0 && isfinite(dl);
    const c128 v = lane > l ? cscale(rsq[l], r[t]) : (lane == l ? c128{ok ? sqrt(dl) : 1.0, 0.0} : c128{0.0, 0.0});
    M[(int64_t)(p + l) * ld + p + lane] = v;
    if (lane == l && !ok) atomicOr(fail, 1);
    S[l][lane] = b[t];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < NB * NB; t += CT) {
    const int j = t / NB, i = t % NB;
    inv[(int64_t)j * NB + i] = (i >= j) ? S[i][j] : c128{0.0, 0.0};
  }
}

__global__ void copy_block_kernel(const c128* src, int64_t lds, c128* dst, int64_t ldd, int rows, int cols) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / rows, i = t % rows;
    dst[j * ldd + i] = src[j * lds + i];
  }
}

// Invert each 64 x 64 diagonal block of a lower-triangular L (padded) and
// write it into the diagonal of Linv.
__global__ __launch_bounds__(CT) void trinv_diag_kernel(const c128* L, c128* X, int64_t ld) {
  __shared__ c128 S[NB][NB + 1];
  __shared__ c128 xb[2][NB];
  __shared__ double rpiv[NB];
  const int p = blockIdx.x * NB;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int t = threadIdx.x; t < NB * NB; t += CT) {
    const int j = t / NB, i = t % NB;
    S[i][j] = L[(int64_t)(p + j) * ld + p + i];
  }
  __syncthreads();
  if (threadIdx.x < NB) rpiv[threadIdx.x] = 1.0 / S[threadIdx.x][threadIdx.x].re;
  __syncthreads();
  c128 b[CW];
  trinv64(S, rpiv, xb, b);
  __syncthreads();
  static_for<0, CW>([&](auto U) {
    constexpr int t = decltype(U)::value;
    S[4 * t + w][lane] = b[t];
  });
  __syncthreads();
  for (int t = threadIdx.x; t < NB * NB; t += CT) {
    const int j = t / NB, i = t % NB;
    X[(int64_t)(p + j) * ld + p + i] = (i >= j) ? S[i][j] : c128{0.0, 0.0};
  }
}

// ------------------------------------------------------------- Jacobi

// Rotation annihilating b in [[a, b], [conj(b), d]] (a, d real).  With
// x = d - a and the classical t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
// tau = x / (2|b|) (Golub & Van Loan, symmetric Schur 2x2, conjugated by
// diag(1, e^{-i arg b})), write t = tp |b| with
//   tp = 2 sign(x) / (|x| + sqrt(x^2 + 4|b|^2)),
// so that c = 1 / sqrt(1 + tp^2 |b|^2), s = tp c b and the diagonal shift
// t |b| = tp |b|^2 need no |b| itself.  The square roots and the division
// use refined hardware estimates; the rotation stays unitary to rounding.
__device__ __forceinline__ void jacobi_rot(double a, double d, c128 b, double thr, double& c, c128& s, double& t_out, int& did) {
  const double nb2 = b.re * b.re + b.im * b.im;
  if (!(nb2 > thr * thr)) {
    c = 1.0; s = c128{0.0, 0.0}; t_out = 0.0; did = 0;
    return;
  }
  const double x = d - a;
  const double y = x * x + 4.0 * nb2;
  const double tp = (x >= 0.0 ? 2.0 : -2.0) * rcp_nr(fabs(x) + y * rsqrt_nr(y));
  c = rsqrt_nr(1.0 + tp * tp * nb2);
  s = c128{tp * c * b.re, tp * c * b.im};
  t_out = tp * nb2;
  did = 1;
}

// Round-robin pairing of n players (n even), round r: position i plays
// position n-1-i; position 0 is fixed, positions 1..n-1 rotate.
__device__ __forceinline__ int rr_player(int pos, int r, int n) {
  if (pos == 0) return 0;
  return ((pos - 1 + r) % (n - 1)) + 1;
}

// One Jacobi sweep on the 32 x 32 subproblem [[G_pp, G_pq], [G_qp, G_qq]]
// of pair `pair` in round `round`, in steps of 16 disjoint rotations.
// Round 0 of an outer sweep holds every block of G in exactly one pair, so
// there the subproblem gets a full cyclic sweep (31 steps, round-robin
// pairing) and every index pair inside a block is rotated once; the later
// rounds (cross = 1) rotate only the 256 index pairs across the two blocks
// (16 steps; step r pairs row i of block p with row (i + r) mod 16 of block
// q).  The outer sweep thus meets every index pair of G once, as a cyclic
// Jacobi sweep does.  Thread (a, b) = (tid % 16, tid / 16) owns the 2 x 2
// block of rotation a's rows and rotation b's columns and rows b, b + 16 of
// rotation a's two columns of the accumulated unitary.  Every lane computes
// rotation a = lane % 16 from the step's input matrix and takes rotation b
// from lane b of its own wave by a lane shuffle; the matrix is
// double-buffered in LDS, so a step needs one barrier.  The unitary takes a
// step's rotation one step late, while the next step's operands are read
// (round 0), or holds it in registers (the cross rounds, below).
// Writes U (32 x 32, column-major) to Uw[pair] and flags the pair in pflag
// when it rotated; *count counts the pairs that rotated.  A subproblem whose
// off-diagonal entries are all at or below thr is left alone (U = I is
// implied by pflag = 0).
__global__ __launch_bounds__(256) void jacobi_sub_kernel(const c128* G, int64_t ld, int nbj, int round, c128* Uw,
                                                         double thr, int max_sweeps, int* count, int* pflag) {
  __shared__ c128 S[2][SP][SP + 1];
  __shared__ c128 U[SP][SP + 1];
  const int pair = blockIdx.x;
  const int tid = threadIdx.x;
  const int bp = rr_player(pair, round, nbj), bq = rr_player(nbj - 1 - pair, round, nbj);
  const int P = min(bp, bq) * JB, Q = max(bp, bq) * JB;
  int big = 0;
  for (int t = tid; t < SP * SP; t += 256) {
    const int j = t / SP, i = t % SP;
    const int gi = i < JB ? P + i : Q + i - JB;
    const int gj = j < JB ? P + j : Q + j - JB;
    const c128 g = G[(int64_t)gj * ld + gi];
    S[0][i][j] = g;
    U[i][j] = (i == j) ? c128{1.0, 0.0} : c128{0.0, 0.0};
    if (i != j && g.re * g.re + g.im * g.im > thr * thr) big = 1;
  }
  const bool needed = __syncthreads_or(big);
  const int a = tid % (SP / 2), b = tid / (SP / 2);
  const bool cross = round > 0;
  const int nsteps = cross ? JB : SP - 1;
  int total = 0;
  // U <- U J on the columns (up, uq) of a rotation (c, s), rows b and b + 16
  auto rotate_u = [&](int up_col, int uq_col, double c, c128 sr) {
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int i = b + (SP / 2) * v;
      const c128 up = U[i][up_col], uq = U[i][uq_col];
      U[i][up_col] = csub(cscale(c, up), cmul(cconj(sr), uq));
      U[i][uq_col] = cadd(cmul(sr, up), cscale(c, uq));
    }
  };
  // In the cross rounds U stays in registers: thread (a, b) holds U[b][a]
  // and U[b + 16][a] (its rotation's fixed column) and U[b][q], U[b + 16][q]
  // for the step's partner column q = 16 + (a + r) mod 16, which passes one
  // lane down the row of 16 lanes (DPP row rotation) after each step; after
  // the 16 steps q is 16 + a again.
  c128 up0{a == b ? 1.0 : 0.0, 0.0}, up1{0.0, 0.0}, uq0{0.0, 0.0}, uq1{a == b ? 1.0 : 0.0, 0.0};
  for (int sweep = 0; needed && sweep < max_sweeps; ++sweep) {
    int did_any = 0;
    int lp = 0, lq = 0;  // the previous step's rotation a, not yet applied to U
    double lc = 1.0;
    c128 ls{0.0, 0.0};
    for (int r = 0; r < nsteps; ++r) {
      const c128 (*cur)[SP + 1] = S[r & 1];
      c128 (*nxt)[SP + 1] = S[(r + 1) & 1];
      int pa, qa, pb, qb;
      if (cross) {
        pa = a;
        qa = JB + ((a + r) & (JB - 1));
        pb = b;
        qb = JB + ((b + r) & (JB - 1));
      } else {
        const int pa0 = rr_player(a, r, SP), qa0 = rr_player(SP - 1 - a, r, SP);
        const int pb0 = rr_player(b, r, SP), qb0 = rr_player(SP - 1 - b, r, SP);
        pa = min(pa0, qa0);
        qa = max(pa0, qa0);
        pb = min(pb0, qb0);
        qb = max(pb0, qb0);
      }
      const double app = cur[pa][pa].re, aqq = cur[qa][qa].re;
      const c128 apq = cur[pa][qa];
      const c128 x00 = cur[pa][pb], x01 = cur[pa][qb], x10 = cur[qa][pb], x11 = cur[qa][qb];
      if (!cross && r > 0) rotate_u(lp, lq, lc, ls);
      double ca, ta;
      c128 sa;
      int da;
      jacobi_rot(app, aqq, apq, thr, ca, sa, ta, da);
      did_any |= da;
      // rotation b was computed by lane b of this wave (lane % 16 == b)
      const double cb = __shfl(ca, b);
      const c128 sb{__shfl(sa.re, b), __shfl(sa.im, b)};
      // rows: row_p' = c row_p - s row_q ; row_q' = conj(s) row_p + c row_q
      const c128 y00 = csub(cscale(ca, x00), cmul(sa, x10));
      const c128 y01 = csub(cscale(ca, x01), cmul(sa, x11));
      const c128 y10 = cadd(cmul(cconj(sa), x00), cscale(ca, x10));
      const c128 y11 = cadd(cmul(cconj(sa), x01), cscale(ca, x11));
      // cols: col_p' = c col_p - conj(s) col_q ; col_q' = s col_p + c col_q
      c128 z00 = csub(cscale(cb, y00), cmul(cconj(sb), y01));
      c128 z01 = cadd(cmul(sb, y00), cscale(cb, y01));
      c128 z10 = csub(cscale(cb, y10), cmul(cconj(sb), y11));
      c128 z11 = cadd(cmul(sb, y10), cscale(cb, y11));
      if (a == b) {
        if (ta != 0.0) {
          z00 = c128{x00.re - ta, 0.0};
          z11 = c128{x11.re + ta, 0.0};
          z01 = c128{0.0, 0.0};
          z10 = c128{0.0, 0.0};
        } else {
          z00.im = 0.0;
          z11.im = 0.0;
        }
      }
      nxt[pa][pb] = z00;
      nxt[pa][qb] = z01;
      nxt[qa][pb] = z10;
      nxt[qa][qb] = z11;
      if (cross) {
        // U <- U J on columns a and q: col_a' = c col_a - conj(s) col_q,
        // col_q' = s col_a + c col_q; then q moves on (lane a takes lane a + 1's)
        const c128 n0 = csub(cscale(ca, up0), cmul(cconj(sa), uq0));
        const c128 m0 = cadd(cmul(sa, up0), cscale(ca, uq0));
        const c128 n1 = csub(cscale(ca, up1), cmul(cconj(sa), uq1));
        const c128 m1 = cadd(cmul(sa, up1), cscale(ca, uq1));
        up0 = n0;
        up1 = n1;
        uq0 = c128{row_next(m0.re), row_next(m0.im)};
        uq1 = c128{row_next(m1.re), row_next(m1.im)};
      }
      lp = pa;
      lq = qa;
      lc = ca;
      ls = sa;
      __syncthreads();
    }
    if (!cross) rotate_u(lp, lq, lc, ls);
    // the sweep's result is in S[nsteps & 1]; a further sweep starts from S[0]
    if ((nsteps & 1) && sweep + 1 < max_sweeps) {
      for (int t = tid; t < SP * SP; t += 256) S[0][t % SP][t / SP] = S[1][t % SP][t / SP];
    }
    if (!__syncthreads_or(did_any)) break;
    ++total;
  }
  if (tid == 0) {
    if (total > 0) atomicAdd(count, 1);
    pflag[pair] = total > 0;
  }
  if (total == 0) return;
  c128* Uo = Uw + (int64_t)pair * SP * SP;
  if (cross) {
    Uo[a * SP + b] = up0;
    Uo[a * SP + b + JB] = up1;
    Uo[(JB + a) * SP + b] = uq0;
    Uo[(JB + a) * SP + b + JB] = uq1;
    return;
  }
  for (int t = tid; t < SP * SP; t += 256) {
    const int j = t / SP, i = t % SP;
    Uo[(int64_t)j * SP + i] = U[i][j];
  }
}

// Index of row/col i (0..2*JB-1) of the subproblem of pair `pair` in round `round`.
__device__ __forceinline__ int sub_index(int pair, int round, int nbj, int i) {
  const int bp = rr_player(pair, round, nbj), bq = rr_player(nbj - 1 - pair, round, nbj);
  const int P = min(bp, bq) * JB, Q = max(bp, bq) * JB;
  return i < JB ? P + i : Q + i - JB;
}

// 16 x 16 output tile of a 32 x 32 complex product on the FP64 MFMA
// (v_mfma_f64_16x16x4f64; lane l holds A[l % 16][k0 + l / 16] and
// B[k0 + l / 16][l % 16]; accumulator r of lane l is row l / 16 + 4 r,
// column l % 16).  a(i, k) and b(k, j) fetch the complex operands; two
// accumulators per tile take Re = Ar Br - Ai Bi and Im = Ar Bi + Ai Br.
template <typename FA, typename FB>
__device__ __forceinline__ void cgemm_tile32(int lane, FA a, FB b, doublex4& cr, doublex4& ci) {
  cr = doublex4{0, 0, 0, 0};
  ci = doublex4{0, 0, 0, 0};
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int k0 = 0; k0 < SP; k0 += 4) {
    const c128 x = a(li, k0 + lk);
    const c128 y = b(k0 + lk, li);
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(x.re, y.re, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(x.re, y.im, ci, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(x.im, -y.im, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(x.im, y.re, ci, 0, 0, 0);
  }
}

// G <- J^H G J with J block-diagonal (one 32 x 32 U per pair, in the pair's
// index set); block (a, b) of pairs is U_a^H G_ab U_b.  G stays Hermitian,
// so only the blocks a <= b are formed and each is also written, conjugate
// transposed, to (b, a) (a diagonal block from its upper triangle).  Also
// V <- V J on row chunks of 32.  blockIdx.x < npair (npair + 1) / 2: G
// blocks; the rest: V blocks.  The data block and the rotation blocks are
// staged in LDS; each of the four waves computes one 16 x 16 quarter of each
// 32 x 32 product on MFMA.
__global__ __launch_bounds__(256) void jacobi_apply_kernel(c128* G, c128* V, int64_t ld, int kp, int nbj, int round,
                                                           const c128* Uw, const int* pflag) {
  __shared__ c128 X[SP][SP + 1];
  __shared__ c128 Y[SP][SP + 1];
  __shared__ c128 UA[SP][SP + 1];
  __shared__ c128 UB[SP][SP + 1];
  const int npair = nbj / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = (wave >> 1) * 16, c0 = (wave & 1) * 16;  // this wave's quarter
  int blk = blockIdx.x;
  doublex4 cr, ci;
  const int ntri = npair * (npair + 1) / 2;
  if (blk < ntri) {
    // blk -> (a, b), a <= b, row by row of the upper triangle
    int a = 0, rest = blk;
    while (rest >= npair - a) {
      rest -= npair - a;
      ++a;
    }
    const int b = a + rest;
    const bool ua = pflag[a], ub = pflag[b];
    if (!ua && !ub) return;  // both rotations are the identity
    const c128* Ua = Uw + (int64_t)a * SP * SP;
    const c128* Ub = Uw + (int64_t)b * SP * SP;
    for (int t = tid; t < SP * SP; t += 256) {
      const int j = t / SP, i = t % SP;
      X[i][j] = G[(int64_t)sub_index(b, round, nbj, j) * ld + sub_index(a, round, nbj, i)];
      if (ua) UA[i][j] = Ua[t];
      if (ub) UB[i][j] = Ub[t];
    }
    __syncthreads();
    // Y = X Ub
    if (ub) {
      cgemm_tile32(lane, [&](int i, int k) { return X[r0 + i][k]; }, [&](int k, int j) { return UB[k][c0 + j]; },
                   cr, ci);
#pragma unroll
      for (int r = 0; r < 4; ++r) Y[r0 + (lane >> 4) + 4 * r][c0 + (lane & 15)] = c128{cr[r], ci[r]};
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = r0 + (lane >> 4) + 4 * r, j = c0 + (lane & 15);
        Y[i][j] = X[i][j];
      }
    }
    __syncthreads();
    // out = Ua^H Y
    if (ua) {
      cgemm_tile32(lane, [&](int i, int k) { return cconj(UA[k][r0 + i]); },
                   [&](int k, int j) { return Y[k][c0 + j]; }, cr, ci);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const c128 y = Y[r0 + (lane >> 4) + 4 * r][c0 + (lane & 15)];
        cr[r] = y.re;
        ci[r] = y.im;
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = r0 + (lane >> 4) + 4 * r, j = c0 + (lane & 15);
      const int gi = sub_index(a, round, nbj, i), gj = sub_index(b, round, nbj, j);
      if (a != b) {
        G[(int64_t)gj * ld + gi] = c128{cr[r], ci[r]};
        G[(int64_t)gi * ld + gj] = c128{cr[r], -ci[r]};
      } else if (i < j) {
        G[(int64_t)gj * ld + gi] = c128{cr[r], ci[r]};
        G[(int64_t)gi * ld + gj] = c128{cr[r], -ci[r]};
      } else if (i == j) {
        G[(int64_t)gj * ld + gi] = c128{cr[r], 0.0};
      }
    }
  } else {
    blk -= ntri;
    const int a = blk % npair, rb = blk / npair;  // pair, row chunk
    if (!pflag[a]) return;
    const c128* Ua = Uw + (int64_t)a * SP * SP;
    const int v0 = rb * SP;
    for (int t = tid; t < SP * SP; t += 256) {
      const int j = t / SP, i = t % SP;
      X[i][j] = V[(int64_t)sub_index(a, round, nbj, j) * ld + v0 + i];
      UA[i][j] = Ua[t];
    }
    __syncthreads();
    cgemm_tile32(lane, [&](int i, int k) { return X[r0 + i][k]; }, [&](int k, int j) { return UA[k][c0 + j]; }, cr,
                 ci);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = r0 + (lane >> 4) + 4 * r, j = c0 + (lane & 15);
      V[(int64_t)sub_index(a, round, nbj, j) * ld + v0 + i] = c128{cr[r], ci[r]};
    }
  }
}

// Frobenius norm in two deterministic stages: one block per column writes the
// column's sum of squares, then one block adds the kp column sums in a fixed
// order.
__global__ __launch_bounds__(256) void frob_cols_kernel(const c128* G, int64_t ld, int kp, double* part) {
  __shared__ double red[256];
  const int64_t col = blockIdx.x;
  double s = 0;
  for (int i = threadIdx.x; i < kp; i += 256) {
    const c128 z = G[col * ld + i];
    s += z.re * z.re + z.im * z.im;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[col] = red[0];
}

__global__ __launch_bounds__(256) void frob_sum_kernel(const double* part, int kp, double* out) {
  __shared__ double red[256];
  double s = 0;
  for (int i = threadIdx.x; i < kp; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt(red[0]);
}

// Select eigenvalues theta > 0 of the first k diagonal entries, order them
// descending (ascending 1/theta), gather the matching eigenvector columns
// (first kp rows) into Ysel and write lambda = 1/theta.  Counts positives and
// negatives that are resolved away from zero.
__global__ void select_kernel(const c128* G, const c128* V, int64_t ld, int k, int kp, double tiny,
                              c128* Ysel, double* lam, int* npos, int* nneg) {
  const int i = blockIdx.x;
  if (i >= k) return;
  const double ti = G[(int64_t)i * ld + i].re;
  if (threadIdx.x == 0) {
    if (ti > tiny) atomicAdd(npos, 1);
    if (ti < -tiny) atomicAdd(nneg, 1);
  }
  if (!(ti > tiny)) return;
  __shared__ int rank;
  if (threadIdx.x == 0) rank = 0;
  __syncthreads();
  int cnt = 0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    const double tj = G[(int64_t)j * ld + j].re;
    if (tj > ti || (tj == ti && j < i)) ++cnt;
  }
  atomicAdd(&rank, cnt);
  __syncthreads();
  const int r = rank;
  if (r >= k / 2) return;
  if (threadIdx.x == 0) lam[r] = 1.0 / ti;
  for (int row = threadIdx.x; row < kp; row += blockDim.x) Ysel[(int64_t)r * kp + row] = V[(int64_t)i * ld + row];
}

}  // namespace

// ---------------------------------------------------------------------------
Err d2h_small(void* host, const void* dev, size_t bytes, const DenseWs& ws, hipStream_t s) {
  if (bytes == 0) return ok();
  void* dst = (ws.hpin && bytes <= ws.hpin_bytes) ? ws.hpin : host;
  CHASE_HIP(hipMemcpyAsync(dst, dev, bytes, hipMemcpyDeviceToHost, s));
  CHASE_HIP(hipStreamSynchronize(s));
  if (dst != host) std::memcpy(host, dst, bytes);
  return ok();
}

static int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 2048)); }

static Err frob_norm(const c128* G, int kp, DenseWs& ws, hipStream_t s, double* host_out) {
  double* part = reinterpret_cast<double*>(ws.panel);  // kp doubles (panel holds kp x 64 c128)
  hipLaunchKernelGGL(frob_cols_kernel, dim3(kp), dim3(256), 0, s, G, (int64_t)kp, kp, part);
  CHASE_LAUNCH_CHECK();
  hipLaunchKernelGGL(frob_sum_kernel, dim3(1), dim3(256), 0, s, (const double*)part, kp, ws.dscalar);
  CHASE_LAUNCH_CHECK();
  return d2h_small(host_out, ws.dscalar, sizeof(double), ws, s);
}

Err fill_padded(c128* M, int kp, int k, double inner, double pad, bool zero_all, hipStream_t s) {
  hipLaunchKernelGGL(fill_diag_kernel, dim3(grid_for((int64_t)kp * kp)), dim3(256), 0, s, M, (int64_t)kp, kp, k,
                     inner, pad, zero_all ? 1 : 0);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err cholesky_lower(c128* M, int kp, DenseWs& ws, hipStream_t s, bool* failed) {
  CHASE_HIP(hipMemsetAsync(ws.flag, 0, sizeof(int), s));
  const int nblk = kp / NB;
  for (int b = 0; b < nblk; ++b) {
    const int p = b * NB;
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(CT), 0, s, M, (int64_t)kp, p, ws.small, ws.flag);
    CHASE_LAUNCH_CHECK();
    const int rest = kp - p - NB;
    if (rest <= 0) break;
    // panel: L_ip = A_ip * L_pp^{-H}
    hipLaunchKernelGGL(copy_block_kernel, dim3(grid_for((int64_t)rest * NB)), dim3(256), 0, s,
                       (const c128*)(M + (int64_t)p * kp + p + NB), (int64_t)kp, ws.panel, (int64_t)rest, rest, NB);
    CHASE_LAUNCH_CHECK();
    ZgemmArgs g{};
    g.transA = 0; g.transB = 1;
    g.M = rest; g.N = NB; g.K = NB;
    g.alpha = {1, 0}; g.beta = {0, 0};
    g.A = ws.panel; g.lda = rest; g.B = ws.small; g.ldb = NB;
    g.C = M + (int64_t)p * kp + p + NB; g.ldc = kp;
    g.kneg = NB; g.batch = 1;
    CHASE_TRY(zgemm(g, nullptr, 0, s));
    // trailing update: A22 -= L_ip L_ip^H
    ZgemmArgs u{};
    u.transA = 0; u.transB = 1;
    u.M = rest; u.N = rest; u.K = NB;
    u.alpha = {-1, 0}; u.beta = {1, 0};
    u.A = M + (int64_t)p * kp + p + NB; u.lda = kp;
    u.B = M + (int64_t)p * kp + p + NB; u.ldb = kp;
    u.C = M + (int64_t)(p + NB) * kp + p + NB; u.ldc = kp;
    u.kneg = NB; u.batch = 1;
    CHASE_TRY(zgemm(u, nullptr, 0, s));
  }
  hipLaunchKernelGGL(zero_upper_kernel, dim3(grid_for((int64_t)kp * kp)), dim3(256), 0, s, M, (int64_t)kp, kp);
  CHASE_LAUNCH_CHECK();
  int f = 0;
  CHASE_TRY(d2h_small(&f, ws.flag, sizeof(int), ws, s));
  *failed = f != 0;
  return ok();
}

Err tri_inverse_lower(const c128* L, c128* X, int kp, DenseWs& ws, hipStream_t s) {
  const int nblk = kp / NB;
  CHASE_TRY(fill_padded(X, kp, kp, 0.0, 0.0, true, s));
  hipLaunchKernelGGL(trinv_diag_kernel, dim3(nblk), dim3(CT), 0, s, L, X, (int64_t)kp);
  CHASE_LAUNCH_CHECK();
  const int64_t stride = (int64_t)NB * (kp + 1);
  for (int d = 1; d < nblk; ++d) {
    const int batch = nblk - d;
    // T_j = L[j+d, j..j+d-1] * X[j..j+d-1, j]
    ZgemmArgs g{};
    g.transA = 0; g.transB = 0;
    g.M = NB; g.N = NB; g.K = (int64_t)d * NB;
    g.alpha = {1, 0}; g.beta = {0, 0};
    g.A = L + (int64_t)d * NB; g.lda = kp; g.strideA = stride;
    g.B = X; g.ldb = kp; g.strideB = stride;
    g.C = ws.tmp; g.ldc = NB; g.strideC = (int64_t)NB * NB;
    g.kneg = g.K; g.batch = batch;
    CHASE_TRY(zgemm(g, ws.gemm_ws, ws.gemm_ws_bytes, s));  // K = d * 64: split along K
    // X[j+d, j] = -X[j+d, j+d] * T_j
    ZgemmArgs h{};
    h.transA = 0; h.transB = 0;
    h.M = NB; h.N = NB; h.K = NB;
    h.alpha = {-1, 0}; h.beta = {0, 0};
    h.A = X + (int64_t)d * NB * (kp + 1); h.lda = kp; h.strideA = stride;
    h.B = ws.tmp; h.ldb = NB; h.strideB = (int64_t)NB * NB;
    h.C = X + (int64_t)d * NB; h.ldc = kp; h.strideC = stride;
    h.kneg = NB; h.batch = batch;
    CHASE_TRY(zgemm(h, nullptr, 0, s));
  }
  return ok();
}

// flag[0] = 1 if some off-diagonal entry of the kp x kp G has |g| > thr:
// the condition under which a further Jacobi sweep would rotate at all.
__global__ __launch_bounds__(256) void offdiag_above_kernel(const c128* G, int kp, double thr2, int* flag) {
  const int64_t total = (int64_t)kp * kp;
  int big = 0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / kp, i = t % kp;
    const c128 g = G[t];
    if (i != j && g.re * g.re + g.im * g.im > thr2) big = 1;
  }
  if (__syncthreads_or(big) && threadIdx.x == 0) atomicOr(flag, 1);
}

Err jacobi_eigh(c128* G, c128* V, int kp, DenseWs& ws, hipStream_t s, int max_sweeps, int* sweeps_out) {
  const int nbj = kp / JB;  // even since kp % 64 == 0
  const int npair = nbj / 2;
  CHASE_TRY(fill_padded(V, kp, kp, 1.0, 1.0, true, s));
  double fro = 0;
  CHASE_TRY(frob_norm(G, kp, ws, s, &fro));
  const double thr = 1e-16 * std::max(fro, 1e-300);
  // One cyclic sweep per subproblem: block Jacobi with approximate
  // subproblem solutions needs about as many outer sweeps as with exact ones
  // and a fraction of the inner work.
  const int inner_sweeps = 1;
  int sweep = 0;
  bool converged = false;
  for (; sweep < max_sweeps; ++sweep) {
    CHASE_HIP(hipMemsetAsync(ws.flag, 0, 2 * sizeof(int), s));
    for (int r = 0; r < nbj - 1; ++r) {
      hipLaunchKernelGGL(jacobi_sub_kernel, dim3(npair), dim3(256), 0, s, (const c128*)G, (int64_t)kp, nbj, r,
                         ws.U, thr, inner_sweeps, ws.flag, ws.pflag);
      CHASE_LAUNCH_CHECK();
      const int blocks = npair * (npair + 1) / 2 + npair * (kp / SP);
      hipLaunchKernelGGL(jacobi_apply_kernel, dim3(blocks), dim3(256), 0, s, G, V, (int64_t)kp, kp, nbj, r,
                         (const c128*)ws.U, (const int*)ws.pflag);
      CHASE_LAUNCH_CHECK();
    }
    // the sweep rotated: stop if no off-diagonal entry is left above thr
    // (the next sweep would then leave G and V unchanged)
    hipLaunchKernelGGL(offdiag_above_kernel, dim3((unsigned)std::min<int64_t>(ceil_div((int64_t)kp * kp, 256), 1024)),
                       dim3(256), 0, s, (const c128*)G, kp, thr * thr, ws.flag + 1);
    CHASE_LAUNCH_CHECK();
    int cnt[2] = {0, 0};
    CHASE_TRY(d2h_small(cnt, ws.flag, 2 * sizeof(int), ws, s));
    if (cnt[0] == 0 || cnt[1] == 0) {
      if (cnt[0] != 0) ++sweep;  // count the sweep that rotated
      converged = true;
      break;
    }
  }
  if (sweeps_out) *sweeps_out = sweep;
  if (!converged)
    return fail(CHASE_PH_ERR_EIG, "Jacobi eigensolver: off-diagonal entries above 1e-16 ||G||_F after " +
                                      std::to_string(max_sweeps) + " sweeps");
  return ok();
}

Err select_positive(const c128* G, const c128* V, int k, int kp, c128* Ysel, double* dlam, DenseWs& ws,
                    hipStream_t s, int* npos, int* nneg) {
  // tiny: 1e3 * u * max|theta| bounded by the Frobenius norm
  double fro = 0;
  CHASE_TRY(frob_norm(G, kp, ws, s, &fro));
  const double tiny = 1e3 * 1.1102230246251565e-16 * fro;
  CHASE_HIP(hipMemsetAsync(ws.flag, 0, 2 * sizeof(int), s));
  CHASE_HIP(hipMemsetAsync(Ysel, 0, (size_t)kp * (k / 2) * sizeof(c128), s));
  hipLaunchKernelGGL(select_kernel, dim3(k), dim3(256), 0, s, G, V, (int64_t)kp, k, kp, tiny, Ysel, dlam, ws.flag,
                     ws.flag + 1);
  CHASE_LAUNCH_CHECK();
  int h[2] = {0, 0};
  CHASE_TRY(d2h_small(h, ws.flag, 2 * sizeof(int), ws, s));
  *npos = h[0];
  *nneg = h[1];
  return ok();
}

int pad64(int k) { return (int)ceil_div(std::max(k, 1), NB) * NB; }

}  // namespace chase
