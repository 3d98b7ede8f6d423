// Block-structured complex GEMM that applies H = [[A, B], [-conj(B), -conj(A)]]
// (Section 1, eq. 1.1) to a tall block X without ever forming H or H^2.
//
// Identity used: with X = [X1; X2] (m rows each),
//   H X = [A X1 + B X2; -conj(A conj(X2) + B conj(X1))]
// so one GEMM  R = [A B] * [X, K conj(X)]  (M = m, N = 2k, K-dim = 2m) gives
//   (H X)_top = R[:, :k]   and   (H X)_bot = -conj(R[:, k:]).
// The big operand [A B] is streamed unmodified (optionally conjugated when the
// buffer holds conj(A)); the conjugation and half swap K conj(X) are folded
// into the loads of the small operand, and the sign/conj of the bottom half
// into the epilogue, which also fuses the Chebyshev three-term update
//   Y = alpha (H X) + beta P + gamma Q.
//
// Complex products run on real MFMA tiles: Re += Ar Br - Ai Bi,
// Im += Ar Bi + Ai Br (four MFMAs per complex k-slice, two accumulators).
//   c64 : v_mfma_f32_32x32x2_f32, block tile 128 x 128, 4 waves of 64 x 64
//   c128: v_mfma_f64_16x16x4_f64, block tile 128 x 64,  4 waves of 64 x 32
// Tiles of the operand strip are staged through LDS (double buffered, split
// real/imaginary planes, k-major so MFMA fragment reads are unit-stride).
// Tile order is XCD-aware: workgroups dispatched to the same XCD take
// consecutive tiles along N, i.e. they share one row strip of [A B] in that
// XCD's L2.
#include "common.h"

namespace chase {
namespace {

struct TF32 {
  using R = float;
  using C = c64;
  using Acc = floatx16;
  static constexpr int MB = 32, NB = 32, KB = 2, NACC = 16;
  __device__ static int a_row(int l) { return l & 31; }
  __device__ static int a_k(int l) { return l >> 5; }
  __device__ static int acc_row(int r, int l) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }
  __device__ static int acc_col(int l) { return l & 31; }
  __device__ static Acc mfma(R a, R b, Acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};

struct TF64 {
  using R = double;
  using C = c128;
  using Acc = doublex4;
  static constexpr int MB = 16, NB = 16, KB = 4, NACC = 4;
  __device__ static int a_row(int l) { return l & 15; }
  __device__ static int a_k(int l) { return l >> 4; }
  __device__ static int acc_row(int r, int l) { return (l >> 4) + 4 * r; }
  __device__ static int acc_col(int l) { return l & 15; }
  __device__ static Acc mfma(R a, R b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// 16-byte vector of the complex type: two c64 or one c128.
template <typename R>
struct Vec16;
template <>
struct Vec16<float> {
  static constexpr int N = 2;
  using T = floatx4;
};
template <>
struct Vec16<double> {
  static constexpr int N = 1;
  using T = doublex4;  // unused for loads; c128 is itself 16 bytes
};

template <typename Tr, int BM, int BN, int BK, int WGM, int WGN>
struct Cfg {
  using R = typename Tr::R;
  using C = typename Tr::C;
  static constexpr int NT = 64 * WGM * WGN;
  static constexpr int WTM = BM / WGM, WTN = BN / WGN;
  static constexpr int FM = WTM / Tr::MB, FN = WTN / Tr::NB;
  static constexpr int VEC = Vec16<R>::N;            // complex per 16-byte A load
  static constexpr int ACHUNK = BM * BK / VEC / NT;  // A loads per thread
  static constexpr int BELEM = BK * BN / NT;         // B loads per thread
  static constexpr int PADA = 4, PADB = 4;
  static constexpr int LDA_S = BM + PADA, LDB_S = BN + PADB;
  static_assert(BM * BK % (VEC * NT) == 0, "A tile split");
  static_assert(BK * BN % NT == 0, "B tile split");
  static_assert(BK % Tr::KB == 0, "BK");
  static_assert(WTM % Tr::MB == 0 && WTN % Tr::NB == 0, "wave tile");
};

__device__ __forceinline__ int xcd_remap(int w, int T) {
  // Workgroup w runs on XCD w % 8.  Give each XCD a contiguous range of
  // tile ids so that tiles sharing a row strip stay in one L2.
  const int xcd = w & 7, slot = w >> 3;
  const int q = T >> 3, r = T & 7;
  return xcd * q + (xcd < r ? xcd : r) + slot;
}

template <typename Tr, int BM, int BN, int BK, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM* WGN) void apply_h_kernel(const ApplyHArgs<typename Tr::R> a) {
  using CF = Cfg<Tr, BM, BN, BK, WGM, WGN>;
  using R = typename Tr::R;
  using C = typename Tr::C;
  constexpr int NT = CF::NT;

  __shared__ R As[2][2][BK][CF::LDA_S];
  __shared__ R Bs[2][2][BK][CF::LDB_S];

  const int m = (int)a.m;
  const int kc = a.k;
  const int N2 = 2 * kc;
  const int TM = (m + BM - 1) / BM;
  const int TN = (N2 + BN - 1) / BN;
  const int tid = threadIdx.x;
  const int nid = xcd_remap(blockIdx.x, TM * TN);
  const int m0 = (nid / TN) * BM;
  const int n0 = (nid % TN) * BN;
  const int nkt = (m + BK - 1) / BK;
  const int KT = 2 * nkt;

  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / WGN) * CF::WTM;
  const int wn0 = (wave % WGN) * CF::WTN;

  // prefetch registers
  R ar[CF::ACHUNK][CF::VEC], ai[CF::ACHUNK][CF::VEC];
  R br[CF::BELEM], bi[CF::BELEM];

  auto load_tiles = [&](int kt) {
    const int phase = kt >= nkt;
    const int kk0 = (kt - phase * nkt) * BK;
    const C* Mat = phase ? a.B : a.A;
    const R csgn = (!phase && a.a_conj) ? R(-1) : R(1);
#pragma unroll
    for (int c = 0; c < CF::ACHUNK; ++c) {
      const int ch = tid + c * NT;
      const int kk = ch / (BM / CF::VEC);
      const int r = (ch % (BM / CF::VEC)) * CF::VEC;
      const int gr = m0 + r, gk = kk0 + kk;
      const C* src = Mat + (int64_t)gk * a.lda + gr;
      if (gk < m && gr + CF::VEC <= m) {
        if constexpr (CF::VEC == 2) {
          floatx4 v = *reinterpret_cast<const floatx4*>(src);
          ar[c][0] = v[0];
          ai[c][0] = v[1] * csgn;
          ar[c][1] = v[2];
          ai[c][1] = v[3] * csgn;
        } else {
          C v = src[0];
          ar[c][0] = v.re;
          ai[c][0] = v.im * csgn;
        }
      } else {
#pragma unroll
        for (int v = 0; v < CF::VEC; ++v) {
          if (gk < m && gr + v < m) {
            C z = src[v];
            ar[c][v] = z.re;
            ai[c][v] = z.im * csgn;
          } else {
            ar[c][v] = R(0);
            ai[c][v] = R(0);
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < CF::BELEM; ++e) {
      const int el = tid + e * NT;
      const int j = el / BK, kk = el % BK;
      const int gj = n0 + j, gk = kk0 + kk;
      R vr = R(0), vi = R(0);
      if (gj < N2 && gk < m) {
        if (gj < kc) {
          C z = a.X[(int64_t)gj * a.ldx + (int64_t)phase * m + gk];
          vr = z.re;
          vi = z.im;
        } else {
          C z = a.X[(int64_t)(gj - kc) * a.ldx + (int64_t)(1 - phase) * m + gk];
          vr = z.re;
          vi = -z.im;
        }
      }
      br[e] = vr;
      bi[e] = vi;
    }
  };

  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int c = 0; c < CF::ACHUNK; ++c) {
      const int ch = tid + c * NT;
      const int kk = ch / (BM / CF::VEC);
      const int r = (ch % (BM / CF::VEC)) * CF::VEC;
#pragma unroll
      for (int v = 0; v < CF::VEC; ++v) {
        As[buf][0][kk][r + v] = ar[c][v];
        As[buf][1][kk][r + v] = ai[c][v];
      }
    }
#pragma unroll
    for (int e = 0; e < CF::BELEM; ++e) {
      const int el = tid + e * NT;
      const int j = el / BK, kk = el % BK;
      Bs[buf][0][kk][j] = br[e];
      Bs[buf][1][kk][j] = bi[e];
    }
  };

  typename Tr::Acc accr[CF::FM][CF::FN], acci[CF::FM][CF::FN];
#pragma unroll
  for (int i = 0; i < CF::FM; ++i)
#pragma unroll
    for (int j = 0; j < CF::FN; ++j)
#pragma unroll
      for (int r = 0; r < Tr::NACC; ++r) {
        accr[i][j][r] = R(0);
        acci[i][j][r] = R(0);
      }

  load_tiles(0);
  store_tiles(0);
  __syncthreads();

  const int ak = Tr::a_k(lane), arow = Tr::a_row(lane);
  for (int kt = 0; kt < KT; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < KT) load_tiles(kt + 1);
#pragma unroll
    for (int ks = 0; ks < BK; ks += Tr::KB) {
      R fa_r[CF::FM], fa_i[CF::FM], fb_r[CF::FN], fb_i[CF::FN], fb_n[CF::FN];
#pragma unroll
      for (int i = 0; i < CF::FM; ++i) {
        fa_r[i] = As[buf][0][ks + ak][wm0 + i * Tr::MB + arow];
        fa_i[i] = As[buf][1][ks + ak][wm0 + i * Tr::MB + arow];
      }
#pragma unroll
      for (int j = 0; j < CF::FN; ++j) {
        fb_r[j] = Bs[buf][0][ks + ak][wn0 + j * Tr::NB + arow];
        fb_i[j] = Bs[buf][1][ks + ak][wn0 + j * Tr::NB + arow];
        fb_n[j] = -fb_i[j];
      }
#pragma unroll
      for (int i = 0; i < CF::FM; ++i)
#pragma unroll
        for (int j = 0; j < CF::FN; ++j) {
          accr[i][j] = Tr::mfma(fa_r[i], fb_r[j], accr[i][j]);
          acci[i][j] = Tr::mfma(fa_r[i], fb_i[j], acci[i][j]);
        }
#pragma unroll
      for (int i = 0; i < CF::FM; ++i)
#pragma unroll
        for (int j = 0; j < CF::FN; ++j) {
          accr[i][j] = Tr::mfma(fa_i[i], fb_n[j], accr[i][j]);
          acci[i][j] = Tr::mfma(fa_i[i], fb_r[j], acci[i][j]);
        }
    }
    if (kt + 1 < KT) store_tiles(buf ^ 1);
    __syncthreads();
  }

  // epilogue: Y = alpha (H X) + beta P + gamma Q
  const int ccol = Tr::acc_col(lane);
#pragma unroll
  for (int i = 0; i < CF::FM; ++i)
#pragma unroll
    for (int j = 0; j < CF::FN; ++j)
#pragma unroll
      for (int r = 0; r < Tr::NACC; ++r) {
        const int gr = m0 + wm0 + i * Tr::MB + Tr::acc_row(r, lane);
        const int gc = n0 + wn0 + j * Tr::NB + ccol;
        if (gr < m && gc < N2) {
          R hr = accr[i][j][r], hi = acci[i][j][r];
          int64_t orow = gr;
          int ocol = gc;
          if (gc >= kc) {  // bottom half: -conj(R)
            hr = -hr;
            orow += m;
            ocol -= kc;
          }
          R yr = a.alpha * hr, yi = a.alpha * hi;
          if (a.P) {
            C p = a.P[(int64_t)ocol * a.ldp + orow];
            yr += a.beta * p.re;
            yi += a.beta * p.im;
          }
          if (a.Q) {
            C q = a.Q[(int64_t)ocol * a.ldq + orow];
            yr += a.gamma * q.re;
            yi += a.gamma * q.im;
          }
          C out;
          out.re = yr;
          out.im = yi;
          a.Y[(int64_t)ocol * a.ldy + orow] = out;
        }
      }
}

}  // namespace

Err launch_apply_h_f32(const ApplyHArgs<float>& a, hipStream_t s) {
  if (a.k <= 0 || a.m <= 0) return ok();
  constexpr int BM = 128, BN = 128, BK = 16;
  const int64_t tiles = ceil_div(a.m, BM) * ceil_div(2 * (int64_t)a.k, BN);
  hipLaunchKernelGGL((apply_h_kernel<TF32, BM, BN, BK, 2, 2>), dim3((unsigned)tiles), dim3(256), 0, s, a);
  CHASE_LAUNCH_CHECK();
  return ok();
}

Err launch_apply_h_f64(const ApplyHArgs<double>& a, hipStream_t s) {
  if (a.k <= 0 || a.m <= 0) return ok();
  constexpr int BM = 128, BN = 64, BK = 16;
  const int64_t tiles = ceil_div(a.m, BM) * ceil_div(2 * (int64_t)a.k, BN);
  hipLaunchKernelGGL((apply_h_kernel<TF64, BM, BN, BK, 2, 2>), dim3((unsigned)tiles), dim3(256), 0, s, a);
  CHASE_LAUNCH_CHECK();
  return ok();
}

}  // namespace chase
