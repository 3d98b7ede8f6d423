// Complex FP64 GEMM on v_mfma_f64_16x16x4_f64:
//   C = alpha * op(A) * diag(s) * op(B) + beta * C,   s_k = -1 for k >= kneg
// op(X) in {X, X^H}.  Used for the Gram matrices of CholeskyQR2 (X^H X), the
// Rayleigh quotient pieces of Alg. 2 (Q^H S T folds S through kneg = m,
// Q2^H Q2), the back-transforms Q Z and T Z, the triangular products of the
// Cholesky / inverse / Jacobi kernels (batched) and the adjoint contraction.
// Tall-skinny inner products (K >> M, N) are split along K into a workspace
// and reduced in a fixed order (deterministic).  Real matrices held in c128
// (real_data) take only the real-by-real MFMA of each step.
#include "common.h"

namespace chase {
namespace {

constexpr int BK = 16, NT = 256;

typedef double doublex2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ doublex4 mfma64(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct ZgemmDev {
  int transA, transB;
  int64_t M, N, K;
  double ar, ai, br, bi;  // alpha, beta
  const c128* A;
  int64_t lda, strideA;
  const c128* B;
  int64_t ldb, strideB;
  c128* C;
  int64_t ldc, strideC;
  int64_t kneg;
  int lower_only, a_lower, b_upper;
  int real_data;
  int splits;
  int tb;          // square tile of the launch (64 or 32)
  int64_t kchunk;  // K range per split (multiple of BK)
  c128* ws;        // splits * batch * M * N partials (split-K only)
};

// TB x TB output tiles (64, or 32 for products too small to fill the CUs
// with 64 x 64 tiles); each of the four waves owns a TB/2 x TB/2 quarter of
// FR x FR MFMA tiles of 16 x 16.
template <bool REAL, int TB>
__global__ __launch_bounds__(NT) void zgemm_kernel(const ZgemmDev g) {
  constexpr int BM = TB, BN = TB, FR = TB / 32;
  constexpr int LDS_A = BM + 2, LDS_B = BN + 2;
  __shared__ double As[2][2][BK][LDS_A];
  __shared__ double Bs[2][2][BK][LDS_B];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int TN = (int)((g.N + BN - 1) / BN);
  const int64_t m0 = (int64_t)(blockIdx.x / TN) * BM;
  const int64_t n0 = (int64_t)(blockIdx.x % TN) * BN;
  const int bt = blockIdx.y, sp = blockIdx.z;
  if (g.lower_only && m0 + BM <= n0) return;  // strictly above the diagonal
  const c128* A = g.A + (int64_t)bt * g.strideA;
  const c128* B = g.B + (int64_t)bt * g.strideB;
  // triangular operands: products with k beyond the last row of this tile
  // (lower op(A)) or the last column (upper op(B)) vanish
  int64_t klim = g.K;
  if (g.a_lower) klim = min(klim, m0 + BM);
  if (g.b_upper) klim = min(klim, n0 + BN);
  const int64_t kbeg = (int64_t)sp * g.kchunk;
  const int64_t kend = min(klim, kbeg + g.kchunk);
  const int KT = (int)((kend - kbeg + BK - 1) / BK);
  const int wm0 = (wave >> 1) * (TB / 2), wn0 = (wave & 1) * (TB / 2);

  constexpr int PER = BM * BK / NT;  // 4 (TB 64) or 2 elements of each operand per thread
  // raw loads (clamped addresses) plus validity bits; conj / sign are applied
  // when the tile is written to LDS, after the MFMAs of the previous slab
  doublex2 ra[PER], rb[PER];
  unsigned okA = 0, okB = 0, negB = 0;

  auto load = [&](int kt) {
    const int64_t k0 = kbeg + (int64_t)kt * BK;
    okA = okB = negB = 0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int el = tid + e * NT;
      int i, kk;
      if (g.transA == 0) { kk = el / BM; i = el % BM; } else { i = el / BK; kk = el % BK; }
      const int64_t gi = m0 + i, gk = k0 + kk;
      const bool ok = gi < g.M && gk < kend;
      const int64_t idx = ok ? (g.transA == 0 ? gk * g.lda + gi : gi * g.lda + gk) : 0;
      ra[e] = *reinterpret_cast<const doublex2*>(A + idx);
      if (ok) okA |= 1u << e;
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int el = tid + e * NT;
      int j, kk;
      if (g.transB == 0) { j = el / BK; kk = el % BK; } else { kk = el / BN; j = el % BN; }
      const int64_t gj = n0 + j, gk = k0 + kk;
      const bool ok = gj < g.N && gk < kend;
      const int64_t idx = ok ? (g.transB == 0 ? gj * g.ldb + gk : gk * g.ldb + gj) : 0;
      rb[e] = *reinterpret_cast<const doublex2*>(B + idx);
      if (ok) okB |= 1u << e;
      if (gk >= g.kneg) negB |= 1u << e;
    }
  };
  auto store = [&](int buf) {
    const double ca = g.transA ? -1.0 : 1.0, cb = g.transB ? -1.0 : 1.0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int el = tid + e * NT;
      int i, kk;
      if (g.transA == 0) { kk = el / BM; i = el % BM; } else { i = el / BK; kk = el % BK; }
      const bool ok = (okA >> e) & 1u;
      As[buf][0][kk][i] = ok ? ra[e][0] : 0.0;
      As[buf][1][kk][i] = ok ? ra[e][1] * ca : 0.0;
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int el = tid + e * NT;
      int j, kk;
      if (g.transB == 0) { j = el / BK; kk = el % BK; } else { kk = el / BN; j = el % BN; }
      const bool ok = (okB >> e) & 1u;
      const double sg = ((negB >> e) & 1u) ? -1.0 : 1.0;
      Bs[buf][0][kk][j] = ok ? rb[e][0] * sg : 0.0;
      Bs[buf][1][kk][j] = ok ? rb[e][1] * cb * sg : 0.0;
    }
  };

  doublex4 cr[FR][FR], ci[FR][FR];
#pragma unroll
  for (int i = 0; i < FR; ++i)
#pragma unroll
    for (int j = 0; j < FR; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) { cr[i][j][r] = 0; ci[i][j][r] = 0; }

  if (KT > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (int kt = 0; kt < KT; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < KT) load(kt + 1);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double fa_r[FR], fa_i[FR], fb_r[FR], fb_i[FR], fb_n[FR];
#pragma unroll
      for (int i = 0; i < FR; ++i) {
        fa_r[i] = As[buf][0][ks + lk][wm0 + 16 * i + lr];
        fa_i[i] = As[buf][1][ks + lk][wm0 + 16 * i + lr];
      }
#pragma unroll
      for (int j = 0; j < FR; ++j) {
        fb_r[j] = Bs[buf][0][ks + lk][wn0 + 16 * j + lr];
        fb_i[j] = Bs[buf][1][ks + lk][wn0 + 16 * j + lr];
        fb_n[j] = -fb_i[j];
      }
      if constexpr (REAL) {
#pragma unroll
        for (int i = 0; i < FR; ++i)
#pragma unroll
          for (int j = 0; j < FR; ++j) cr[i][j] = mfma64(fa_r[i], fb_r[j], cr[i][j]);
      } else {
#pragma unroll
        for (int i = 0; i < FR; ++i)
#pragma unroll
          for (int j = 0; j < FR; ++j) {
            cr[i][j] = mfma64(fa_r[i], fb_r[j], cr[i][j]);
            ci[i][j] = mfma64(fa_r[i], fb_i[j], ci[i][j]);
          }
#pragma unroll
        for (int i = 0; i < FR; ++i)
#pragma unroll
          for (int j = 0; j < FR; ++j) {
            cr[i][j] = mfma64(fa_i[i], fb_n[j], cr[i][j]);
            ci[i][j] = mfma64(fa_i[i], fb_r[j], ci[i][j]);
          }
      }
    }
    if (kt + 1 < KT) store(buf ^ 1);
    __syncthreads();
  }

  const int batch = gridDim.y;
#pragma unroll
  for (int i = 0; i < FR; ++i)
#pragma unroll
    for (int j = 0; j < FR; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = m0 + wm0 + 16 * i + (lane >> 4) + 4 * r;
        const int64_t gj = n0 + wn0 + 16 * j + (lane & 15);
        if (gi < g.M && gj < g.N) {
          const double xr = cr[i][j][r], xi = ci[i][j][r];
          const double yr = g.ar * xr - g.ai * xi, yi = g.ar * xi + g.ai * xr;
          if (g.splits > 1) {
            c128* w = g.ws + ((int64_t)sp * batch + bt) * g.M * g.N;
            w[gj * g.M + gi] = c128{yr, yi};
          } else {
            c128* Cp = g.C + (int64_t)bt * g.strideC + gj * g.ldc + gi;
            double outr = yr, outi = yi;
            if (g.br != 0.0 || g.bi != 0.0) {
              c128 c = *Cp;
              outr += g.br * c.re - g.bi * c.im;
              outi += g.br * c.im + g.bi * c.re;
            }
            *Cp = c128{outr, outi};
          }
        }
      }
}

__global__ void zgemm_reduce(const ZgemmDev g, int batch) {
  const int64_t total = (int64_t)batch * g.M * g.N;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t bt = t / (g.M * g.N), rem = t % (g.M * g.N);
    const int64_t gj = rem / g.M, gi = rem % g.M;
    if (g.lower_only && gi / g.tb < gj / g.tb) continue;  // tile not computed
    double sr = 0, si = 0;
    for (int s = 0; s < g.splits; ++s) {
      c128 w = g.ws[((int64_t)s * batch + bt) * g.M * g.N + rem];
      sr += w.re;
      si += w.im;
    }
    c128* Cp = g.C + bt * g.strideC + gj * g.ldc + gi;
    if (g.br != 0.0 || g.bi != 0.0) {
      c128 c = *Cp;
      sr += g.br * c.re - g.bi * c.im;
      si += g.br * c.im + g.bi * c.re;
    }
    *Cp = c128{sr, si};
  }
}

}  // namespace

Err zgemm(const ZgemmArgs& a, void* ws, size_t ws_bytes, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0 || a.batch <= 0) return ok();
  ZgemmDev g;
  g.transA = a.transA; g.transB = a.transB;
  g.M = a.M; g.N = a.N; g.K = a.K;
  g.ar = a.alpha.re; g.ai = a.alpha.im; g.br = a.beta.re; g.bi = a.beta.im;
  g.A = a.A; g.lda = a.lda; g.strideA = a.strideA;
  g.B = a.B; g.ldb = a.ldb; g.strideB = a.strideB;
  g.C = a.C; g.ldc = a.ldc; g.strideC = a.strideC;
  g.kneg = a.kneg;
  g.lower_only = a.lower_only; g.a_lower = a.a_lower; g.b_upper = a.b_upper;
  g.real_data = a.real_data;
  // 32 x 32 tiles when 64 x 64 ones would leave most CUs idle and K is too
  // short for a split: a 64 x 64 x 64 complex tile is about 7 us of one CU's
  // FP64 MFMA, a 32 x 32 one a quarter of that
  const int64_t t64 = ceil_div(a.M, (int64_t)64) * ceil_div(a.N, (int64_t)64) * a.batch;
  const int tb = (t64 < 128 && a.K <= 256) ? 32 : 64;
  g.tb = tb;
  const int64_t tiles = ceil_div(a.M, (int64_t)tb) * ceil_div(a.N, (int64_t)tb);
  const int64_t tm = ceil_div(a.M, (int64_t)tb);
  const int64_t work_tiles = a.lower_only ? tm * (tm + 1) / 2 : tiles;  // tiles that compute
  int splits = 1;
  if (a.K > 0 && ws && work_tiles * a.batch < 512) {
    const int64_t want = ceil_div(1024, work_tiles * a.batch);
    const int64_t maxk = std::max<int64_t>(1, a.K / (4 * BK));  // at least 4 K slabs per split
    int64_t sp = std::min(want, maxk);
    const int64_t per = a.M * a.N * a.batch * (int64_t)sizeof(c128);
    sp = std::min<int64_t>(sp, (int64_t)(ws_bytes / per));
    splits = (int)std::max<int64_t>(1, std::min<int64_t>(sp, 64));
  }
  g.splits = splits;
  g.kchunk = ceil_div(ceil_div(std::max<int64_t>(a.K, 1), splits), BK) * BK;
  splits = (int)ceil_div(std::max<int64_t>(a.K, 1), g.kchunk);
  g.splits = splits;
  g.ws = (c128*)ws;
  const dim3 grid((unsigned)tiles, (unsigned)a.batch, (unsigned)splits);
  if (a.real_data) {
    if (tb == 32) hipLaunchKernelGGL((zgemm_kernel<true, 32>), grid, dim3(NT), 0, s, g);
    else hipLaunchKernelGGL((zgemm_kernel<true, 64>), grid, dim3(NT), 0, s, g);
  } else {
    if (tb == 32) hipLaunchKernelGGL((zgemm_kernel<false, 32>), grid, dim3(NT), 0, s, g);
    else hipLaunchKernelGGL((zgemm_kernel<false, 64>), grid, dim3(NT), 0, s, g);
  }
  CHASE_LAUNCH_CHECK();
  if (splits > 1) {
    const int64_t total = (int64_t)a.batch * a.M * a.N;
    const int blocks = (int)std::min<int64_t>(ceil_div(total, 256), 4096);
    hipLaunchKernelGGL(zgemm_reduce, dim3(blocks), dim3(256), 0, s, g, a.batch);
    CHASE_LAUNCH_CHECK();
  }
  return ok();
}

}  // namespace chase
