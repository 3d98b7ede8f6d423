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
//   Y = alpha (H X) + beta P + gamma Q + diag(dcol) S.
//
// Complex products run on real MFMA tiles: Re += Ar Br - Ai Bi,
// Im += Ar Bi + Ai Br (four MFMAs per complex k-slice, two accumulators).
//   c64 : v_mfma_f32_32x32x2_f32, waves of 64 x 64 outputs
//   c128: v_mfma_f64_16x16x4_f64, waves of 64 x 32 outputs
// Operand tiles are staged through LDS (double buffered, split real and
// imaginary planes, k-major so MFMA fragment reads are unit-stride).  Global
// loads are branch-free (clamped address + select) so that a whole tile is in
// flight at once while the MFMAs of the previous tile run.
//
// Tile order is XCD-aware: workgroups dispatched to the same XCD take
// consecutive tiles along N of one K range, i.e. they share one row strip of
// [A B] in that XCD's L2.  When the tile grid alone cannot fill the 256 CUs
// the K range is split; partial products go to a workspace and a second
// kernel sums them in a fixed order and applies the fused epilogue.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <type_traits>

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

// Same FP32 rate on 16 x 16 output blocks (k = 4 per MFMA): lets the N tile
// follow 2k in steps of 16 columns instead of 32 or 64.
struct TF32S {
  using R = float;
  using C = c64;
  using Acc = floatx4;
  static constexpr int MB = 16, NB = 16, KB = 4, NACC = 4;
  __device__ static int a_row(int l) { return l & 15; }
  __device__ static int a_k(int l) { return l >> 4; }
  __device__ static int acc_row(int r, int l) { return 4 * (l >> 4) + r; }
  __device__ static int acc_col(int l) { return l & 15; }
  __device__ static Acc mfma(R a, R b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
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

// Raw 16- or 8-byte vectors of V consecutive complex elements: loaded in
// one instruction, consumed only when the tile is written to LDS (after the
// MFMAs of the previous tile), so the loads stay in flight meanwhile.
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef double doublex2 __attribute__((ext_vector_type(2)));
template <typename R, int V>
struct Raw;
template <>
struct Raw<float, 2> {
  using T = floatx4;
};
template <>
struct Raw<float, 1> {
  using T = floatx2;
};
template <>
struct Raw<double, 1> {
  using T = doublex2;
};

template <typename Tr, int BM, int BN, int BK, int WGM, int WGN, int VB>
struct Cfg {
  using R = typename Tr::R;
  static constexpr int NT = 64 * WGM * WGN;
  static constexpr int WTM = BM / WGM, WTN = BN / WGN;
  static constexpr int FM = WTM / Tr::MB, FN = WTN / Tr::NB;
  static constexpr int VEC = sizeof(R) == 4 ? 2 : 1;   // complex per A load
  static constexpr int ACHUNK = BM * BK / VEC / NT;     // A loads per thread
  static constexpr int BCHUNK = BK * BN / VB / NT;      // B loads per thread
  // LDS row pitch: fragment reads of the FP32 16-row MFMA take four k rows
  // of 16 words, conflict-free when the pitch is 16 mod 32 words; those of
  // the FP32 32-row MFMA take two half-waves of 32 consecutive words, so no
  // pad is needed (which keeps the 256 x 64 tile at 80 KB, two workgroups
  // per CU); the FP64 shapes keep a pad of 4 elements.
  static constexpr bool kF32x16 = sizeof(R) == 4 && Tr::MB == 16;
  static constexpr int pitch(int x) {
    return kF32x16 ? x + ((16 - x % 32) + 32) % 32 : (sizeof(R) == 4 ? x : x + 4);
  }
  static constexpr int LDA_S = pitch(BM), LDB_S = pitch(BN);
  static_assert(BM * BK % (VEC * NT) == 0, "A tile split");
  static_assert(BK * BN % (VB * NT) == 0, "B tile split");
  static_assert(BK % Tr::KB == 0, "BK");
  static_assert(WTM % Tr::MB == 0 && WTN % Tr::NB == 0, "wave tile");
};

// f(integral_constant<B>) ... f(integral_constant<E - 1>)
template <int B, int E, typename F>
__device__ __forceinline__ void static_for_n(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for_n<B + 1, E>(f);
  }
}

__device__ __forceinline__ int xcd_remap(int w, int T) {
  // Workgroup w runs on XCD w % 8.  Give each XCD a contiguous range of
  // tile ids so that tiles sharing a row strip stay in one L2.
  const int xcd = w & 7, slot = w >> 3;
  const int q = T >> 3, r = T & 7;
  return xcd * q + (xcd < r ? xcd : r) + slot;
}

template <typename R, typename C>
__device__ __forceinline__ void epilogue_store(const ApplyHArgs<R>& a, int gr, int gc, R hr, R hi) {
  int64_t orow = gr;
  int ocol = gc;
  if (gc >= a.k) {  // bottom half: -conj(R)
    hr = -hr;
    orow += a.m;
    ocol -= a.k;
  }
  R yr = a.alpha * hr, yi = a.alpha * hi;
  if (a.P) {
    const C p = a.P[(int64_t)ocol * a.ldp + orow];
    yr += a.beta * p.re;
    yi += a.beta * p.im;
  }
  if (a.Q) {
    const C q = a.Q[(int64_t)ocol * a.ldq + orow];
    yr += a.gamma * q.re;
    yi += a.gamma * q.im;
  }
  if (a.S) {
    const C z = a.S[(int64_t)ocol * a.lds + orow];
    const R d = a.dcol[ocol];
    yr += d * z.re;
    yi += d * z.im;
  }
  C out;
  out.re = yr;
  out.im = yi;
  a.Y[(int64_t)ocol * a.ldy + orow] = out;
}

// Two waves per SIMD where registers and LDS allow (the 256-row FP32 tiles
// use at most 80 KB of LDS): while one workgroup waits at a tile boundary
// the other keeps the matrix cores busy.
template <typename Tr, int BM, int BN, int BK, int WGM, int WGN, int VB>
__global__ __launch_bounds__(64 * WGM* WGN) __attribute__((amdgpu_waves_per_eu(2, 2))) void apply_h_kernel(const ApplyHArgs<typename Tr::R> a, int splits,
                                                                 int kps, typename Tr::C* ws) {
  using CF = Cfg<Tr, BM, BN, BK, WGM, WGN, VB>;
  using R = typename Tr::R;
  using C = typename Tr::C;
  constexpr int NT = CF::NT;
  constexpr int VEC = CF::VEC;

  __shared__ R As[2][2][BK][CF::LDA_S];
  __shared__ R Bs[2][2][BK][CF::LDB_S];

  const int m = (int)a.m;
  const int kc = a.k;
  const int N2 = a.kreal ? kc : 2 * kc;
  const int TM = (m + BM - 1) / BM;
  const int TN = (N2 + BN - 1) / BN;
  const int T = TM * TN;
  const int tid = threadIdx.x;
  const int nid = xcd_remap(blockIdx.x, T * splits);
  const int sp = nid / T;
  const int t = nid - sp * T;
  const int m0 = (t / TN) * BM;
  const int n0 = (t % TN) * BN;
  const int nkt = (m + BK - 1) / BK;
  const int kt_beg = sp * kps;
  const int kt_end = min(2 * nkt, kt_beg + kps);

  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / WGN) * CF::WTM;
  const int wn0 = (wave % WGN) * CF::WTN;

  // prefetch registers: raw vectors plus validity bits
  using RawA = typename Raw<R, VEC>::T;
  using RawB = typename Raw<R, VB>::T;
  RawA ra[CF::ACHUNK];
  RawB rb[CF::BCHUNK];
  unsigned mask_a = 0, mask_b = 0, bot_b = 0;  // bit per (chunk, element)
  static_assert(CF::ACHUNK * VEC <= 32 && CF::BCHUNK * VB <= 32, "mask width");

  auto load_tiles = [&](int kt) {
    const int phase = kt >= nkt;
    const int kk0 = (kt - phase * nkt) * BK;
    const C* Mat = phase ? a.B : a.A;
    mask_a = 0;
    mask_b = 0;
    bot_b = 0;
#pragma unroll
    for (int c = 0; c < CF::ACHUNK; ++c) {
      const int ch = tid + c * NT;
      const int kk = ch / (BM / VEC);
      const int r = (ch % (BM / VEC)) * VEC;
      const int gr = m0 + r, gk = kk0 + kk;
      const bool okk = gk < m;
      const int64_t idx = (okk && gr < m) ? (int64_t)gk * a.lda + gr : 0;
      ra[c] = *reinterpret_cast<const RawA*>(Mat + idx);
#pragma unroll
      for (int v = 0; v < VEC; ++v)
        if (okk && gr + v < m) mask_a |= 1u << (c * VEC + v);
    }
#pragma unroll
    for (int e = 0; e < CF::BCHUNK; ++e) {
      const int el = tid + e * NT;
      const int j = el / (BK / VB);
      const int kk = (el % (BK / VB)) * VB;
      const int gj = n0 + j, gk = kk0 + kk;
      const bool ok = gj < N2 && gk < m;
      const bool bot = !a.kreal && gj >= kc;
      const int64_t col = bot ? gj - kc : gj;
      const int64_t row = (int64_t)(bot ? 1 - phase : phase) * m + gk;
      const int64_t idx = ok ? col * a.ldx + row : 0;
      rb[e] = *reinterpret_cast<const RawB*>(a.X + idx);
#pragma unroll
      for (int v = 0; v < VB; ++v)
        if (ok && gk + v < m) mask_b |= 1u << (e * VB + v);
      if (bot) bot_b |= 1u << e;
    }
  };

  auto store_tiles = [&](int buf, int kt) {
    const int phase = kt >= nkt;
    const R csgn = (!phase && a.a_conj) ? R(-1) : R(1);
#pragma unroll
    for (int c = 0; c < CF::ACHUNK; ++c) {
      const int ch = tid + c * NT;
      const int kk = ch / (BM / VEC);
      const int r = (ch % (BM / VEC)) * VEC;
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const bool okv = (mask_a >> (c * VEC + v)) & 1u;
        As[buf][0][kk][r + v] = okv ? ra[c][2 * v] : R(0);
        As[buf][1][kk][r + v] = okv ? ra[c][2 * v + 1] * csgn : R(0);
      }
    }
#pragma unroll
    for (int e = 0; e < CF::BCHUNK; ++e) {
      const int el = tid + e * NT;
      const int j = el / (BK / VB);
      const int kk = (el % (BK / VB)) * VB;
      const R isgn = ((bot_b >> e) & 1u) ? R(-1) : R(1);
#pragma unroll
      for (int v = 0; v < VB; ++v) {
        const bool okv = (mask_b >> (e * VB + v)) & 1u;
        Bs[buf][0][kk + v][j] = okv ? rb[e][2 * v] : R(0);
        Bs[buf][1][kk + v][j] = okv ? rb[e][2 * v + 1] * isgn : R(0);
      }
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

  if (kt_beg < kt_end) {
    load_tiles(kt_beg);
    store_tiles(0, kt_beg);
  }
  __syncthreads();

  const int ak = Tr::a_k(lane), arow = Tr::a_row(lane);
  // The K loop, compiled for NL = 0 .. FN live column fragments of this
  // wave: in the last tile column only the fragments that hold columns
  // < 2k do MFMAs (the others stay zero and are never stored), so a ragged
  // 2k (e.g. 520 = 8 x 64 + 8) wastes at most one fragment per wave.
  auto kloop = [&](auto NLc) {
    constexpr int NL = decltype(NLc)::value;
    for (int kt = kt_beg; kt < kt_end; ++kt) {
      const int buf = (kt - kt_beg) & 1;
      if (kt + 1 < kt_end) load_tiles(kt + 1);
      if constexpr (NL > 0) {
#pragma unroll
        for (int ks = 0; ks < BK; ks += Tr::KB) {
          R fa_r[CF::FM], fa_i[CF::FM], fb_r[NL], fb_i[NL], fb_n[NL];
#pragma unroll
          for (int i = 0; i < CF::FM; ++i) {
            fa_r[i] = As[buf][0][ks + ak][wm0 + i * Tr::MB + arow];
            fa_i[i] = As[buf][1][ks + ak][wm0 + i * Tr::MB + arow];
          }
#pragma unroll
          for (int j = 0; j < NL; ++j) {
            fb_r[j] = Bs[buf][0][ks + ak][wn0 + j * Tr::NB + arow];
            fb_i[j] = Bs[buf][1][ks + ak][wn0 + j * Tr::NB + arow];
            fb_n[j] = -fb_i[j];
          }
#pragma unroll
          for (int i = 0; i < CF::FM; ++i)
#pragma unroll
            for (int j = 0; j < NL; ++j) {
              accr[i][j] = Tr::mfma(fa_r[i], fb_r[j], accr[i][j]);
              acci[i][j] = Tr::mfma(fa_r[i], fb_i[j], acci[i][j]);
            }
#pragma unroll
          for (int i = 0; i < CF::FM; ++i)
#pragma unroll
            for (int j = 0; j < NL; ++j) {
              accr[i][j] = Tr::mfma(fa_i[i], fb_n[j], accr[i][j]);
              acci[i][j] = Tr::mfma(fa_i[i], fb_r[j], acci[i][j]);
            }
        }
      }
      if (kt + 1 < kt_end) store_tiles(buf ^ 1, kt + 1);
      __syncthreads();
    }
  };
  const int live = (N2 - (n0 + wn0) + Tr::NB - 1) / Tr::NB;  // wave-uniform
  if (live >= CF::FN) {
    kloop(std::integral_constant<int, CF::FN>{});
  } else if (live <= 0) {
    kloop(std::integral_constant<int, 0>{});
  } else {
    static_for_n<1, CF::FN>([&](auto L) {
      if (live == decltype(L)::value) kloop(L);
    });
  }

  const int ccol = Tr::acc_col(lane);
  C* wsp = ws + (int64_t)sp * m * N2;
#pragma unroll
  for (int i = 0; i < CF::FM; ++i)
#pragma unroll
    for (int j = 0; j < CF::FN; ++j)
#pragma unroll
      for (int r = 0; r < Tr::NACC; ++r) {
        const int gr = m0 + wm0 + i * Tr::MB + Tr::acc_row(r, lane);
        const int gc = n0 + wn0 + j * Tr::NB + ccol;
        if (gr < m && gc < N2) {
          if (splits > 1) {
            C z;
            z.re = accr[i][j][r];
            z.im = acci[i][j][r];
            wsp[(int64_t)gc * m + gr] = z;
          } else {
            epilogue_store<R, C>(a, gr, gc, accr[i][j][r], acci[i][j][r]);
            if (a.kreal) epilogue_store<R, C>(a, gr, gc + kc, accr[i][j][r], acci[i][j][r]);
          }
        }
      }
}

// c64 H X with both operand tiles copied HBM -> LDS by the gfx950
// direct-to-LDS load (global_load_lds_dwordx4: lane l's 16 bytes land at
// the wave's LDS base + 16 l), so nothing is staged through registers.
//  * Tile 256 x BN (BN = 64 on the 32 x 32 MFMA, the main tile; BN = 32 on
//    the 16 x 16 MFMA, for narrow launches), K slabs of 8, a ring of 4 LDS
//    stages: slabs s + 1 .. s + 3 are in flight while slab s is multiplied.
//  * A side ([A B] columns): k-major, interleaved complex, 2 KB per k; one
//    8-byte LDS read gives the real and imaginary fragment.
//  * X side: slot (k pair p, column c) holds X[2p], X[2p + 1] of column c
//    (16 bytes; one copy per k pair fills 64 column slots, of which a
//    32-wide tile reads the first 32).  The K conj of the bottom-half
//    columns is a sign on the fragment's imaginary part, the half swap an
//    address offset.
//  * Rows of A past m and columns past 2k are read from clamped addresses
//    (their outputs are never stored); in a slab that crosses m the X
//    fragment of k >= m is replaced by 0.
//  * The copies are issued from inline assembly, so the compiler neither
//    waits on them nor counts them: every wave issues the same 5 copies per
//    slab (the last slabs repeat the final one into stages that are not read
//    again) and waits with vmcnt(10) for slab s + 1 before the barrier.
//    Nothing else in the K loop reads global memory.
// Needs m even, 16-byte aligned A, B and X, and even lda, ldx.
constexpr int DMA_BM = 256, DMA_XP = 64, DMA_BK = 8, DMA_NST = 4;

__device__ __forceinline__ void vm_wait10() { __builtin_amdgcn_s_waitcnt(0xF7A); }  // vmcnt(10)
__device__ __forceinline__ void vm_wait0() { __builtin_amdgcn_s_waitcnt(0xF70); }   // vmcnt(0)

// One direct-to-LDS copy of 16 bytes per lane to lds_base + 16 lane (M0 is
// saved and restored around it).
__device__ __forceinline__ void lds_copy16(const void* src, unsigned lds_base) {
  unsigned keep;
  __asm__ __volatile__(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %2\n\t"
      "global_load_lds_dwordx4 %1, off\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(keep)
      : "v"(src), "s"(lds_base)
      : "memory");
}

// Workgroup barrier for the DMA ring: this wave's LDS reads are complete
// (lgkmcnt 0) and the copies it must wait for have been waited for
// explicitly (a fenced __syncthreads would also drain every copy still in
// flight).  The empty asm statements keep the compiler from moving memory
// accesses across the barrier.
__device__ __forceinline__ void ring_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), vmcnt / expcnt unchanged
  __asm__ __volatile__("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __asm__ __volatile__("" ::: "memory");
}

template <typename Tr, int BN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void apply_h_dma_kernel(
    const ApplyHArgs<float> a, int splits, int kps, c64* ws) {
  using R = float;
  using C = c64;
  constexpr int BM = DMA_BM, BK = DMA_BK, NST = DMA_NST, XP = DMA_XP, WTM = 64;
  constexpr int FM = WTM / Tr::MB, FN = BN / Tr::NB;
  constexpr int ASTAGE = BK * BM;        // complex per A stage
  constexpr int BSTAGE = (BK / 2) * XP;  // 16-byte slots per X stage
  static_assert(BN <= XP && BN % Tr::NB == 0 && BK % Tr::KB == 0, "DMA tile");
  __shared__ __attribute__((aligned(16))) C As[NST][ASTAGE];
  __shared__ __attribute__((aligned(16))) floatx4 Bs[NST][BSTAGE];

  const int m = (int)a.m;
  const int kc = a.k;
  const int N2 = 2 * kc;
  const int TM = (m + BM - 1) / BM;
  const int TN = (N2 + BN - 1) / BN;
  const int T = TM * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nid = xcd_remap(blockIdx.x, T * splits);
  const int sp = nid / T;
  const int t = nid - sp * T;
  const int m0 = (t / TN) * BM;
  const int n0 = (t % TN) * BN;
  const int nkt = (m + BK - 1) / BK;
  const int kt_beg = sp * kps;
  const int nsl = max(0, min(2 * nkt, kt_beg + kps) - kt_beg);
  const int wm0 = wave * WTM;
  const int64_t rmax = a.lda - 2;  // last valid start of a row pair

  // this lane's X column for the copies (clamped) and its bottom-half flag
  const int gjc = min(n0 + lane, N2 - 1);
  const bool cbot = gjc >= kc;
  const int64_t xcol = cbot ? gjc - kc : gjc;
  const unsigned as_base = (unsigned)(uintptr_t)&As[0][0];
  const unsigned bs_base = (unsigned)(uintptr_t)&Bs[0][0];

  // copies of slab kt into ring stage st: wave w takes the A k-columns
  // 2w, 2w + 1 (two halves of 128 rows each) and the X k pair w
  auto copy_slab = [&](int kt, int st) {
    const int phase = kt >= nkt;
    const int kk0 = (kt - phase * nkt) * BK;
    const C* Mat = phase ? a.B : a.A;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kk = wave * 2 + (q >> 1), half = q & 1;
      const int64_t gk = min(kk0 + kk, m - 1);
      const int64_t r = min((int64_t)(m0 + half * 128 + lane * 2), rmax);
      const unsigned dst = __builtin_amdgcn_readfirstlane(
          as_base + (unsigned)(((st * BK + kk) * BM + half * 128) * sizeof(C)));
      lds_copy16(Mat + gk * a.lda + r, dst);
    }
    const int krow = min(kk0 + 2 * wave, m - 2);
    const int64_t row = (int64_t)(cbot ? 1 - phase : phase) * m + krow;
    const unsigned dstb = __builtin_amdgcn_readfirstlane(
        bs_base + (unsigned)((st * BSTAGE + wave * XP) * sizeof(floatx4)));
    lds_copy16(a.X + xcol * a.ldx + row, dstb);
  };

  typename Tr::Acc accr[FM][FN], acci[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < Tr::NACC; ++r) {
        accr[i][j][r] = R(0);
        acci[i][j][r] = R(0);
      }
  const int ak = Tr::a_k(lane), arow = Tr::a_row(lane);
  const int live = (N2 - n0 + Tr::NB - 1) / Tr::NB;
  // sign of the imaginary part of this lane's X fragments (K conj of the
  // bottom-half columns)
  R bsgn[FN];
#pragma unroll
  for (int j = 0; j < FN; ++j) bsgn[j] = (n0 + j * Tr::NB + arow >= kc) ? R(-1) : R(1);

  if (nsl > 0) {
    copy_slab(kt_beg, 0);
    copy_slab(kt_beg + min(1, nsl - 1), 1);
    copy_slab(kt_beg + min(2, nsl - 1), 2);
    vm_wait10();  // slab 0 landed (slabs 1 and 2 may still be in flight)
  }
  ring_barrier();

  auto kloop = [&](auto NLc) {
    constexpr int NL = decltype(NLc)::value;
    for (int s = 0; s < nsl; ++s) {
      const int st = s & (NST - 1);
      copy_slab(kt_beg + min(s + 3, nsl - 1), (s + 3) & (NST - 1));
      if constexpr (NL > 0) {
        const int kt = kt_beg + s;
        const int phase = kt >= nkt;
        const int kk0 = (kt - phase * nkt) * BK;
        const bool ragged = kk0 + BK > m;  // slab crosses m: zero X for k >= m
        const C* Ast = &As[st][0];
        const floatx4* Bst = &Bs[st][0];
#pragma unroll
        for (int ks = 0; ks < BK; ks += Tr::KB) {
          const int k = ks + ak;
          R fa_r[FM], fa_i[FM], fb_r[NL], fb_i[NL], fb_n[NL];
#pragma unroll
          for (int i = 0; i < FM; ++i) {
            const C z = Ast[k * BM + wm0 + i * Tr::MB + arow];
            fa_r[i] = z.re;
            fa_i[i] = z.im;
          }
          const R kmask = (ragged && kk0 + k >= m) ? R(0) : R(1);
#pragma unroll
          for (int j = 0; j < NL; ++j) {
            const C* slot = reinterpret_cast<const C*>(&Bst[(k >> 1) * XP + j * Tr::NB + arow]);
            const C z = slot[k & 1];
            fb_r[j] = z.re * kmask;
            fb_i[j] = z.im * bsgn[j] * kmask;
            fb_n[j] = -fb_i[j];
          }
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < NL; ++j) {
              accr[i][j] = Tr::mfma(fa_r[i], fb_r[j], accr[i][j]);
              acci[i][j] = Tr::mfma(fa_r[i], fb_i[j], acci[i][j]);
            }
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < NL; ++j) {
              accr[i][j] = Tr::mfma(fa_i[i], fb_n[j], accr[i][j]);
              acci[i][j] = Tr::mfma(fa_i[i], fb_r[j], acci[i][j]);
            }
        }
      }
      // slab s + 1 landed for this wave: at most the copies of slabs s + 2
      // and s + 3 (10) are still in flight
      vm_wait10();
      ring_barrier();
    }
  };
  // K loop compiled for the number of live column fragments (at most FN)
  const int nl = min(live, FN);
  static_for_n<0, FN + 1>([&](auto NLc) {
    if (nl == decltype(NLc)::value) kloop(NLc);
  });
  vm_wait0();  // the trailing repeat copies

  const int ccol = Tr::acc_col(lane);
  C* wsp = ws + (int64_t)sp * m * N2;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < Tr::NACC; ++r) {
        const int gr = m0 + wm0 + i * Tr::MB + Tr::acc_row(r, lane);
        const int gc = n0 + j * Tr::NB + ccol;
        if (gr < m && gc < N2) {
          if (splits > 1) {
            C z;
            z.re = accr[i][j][r];
            z.im = acci[i][j][r];
            wsp[(int64_t)gc * m + gr] = z;
          } else {
            epilogue_store<R, C>(a, gr, gc, accr[i][j][r], acci[i][j][r]);
          }
        }
      }
}

// Sum the split-K partials in a fixed order and apply the epilogue.
template <typename R, typename C>
__global__ void apply_h_reduce(const ApplyHArgs<R> a, int splits, const C* ws) {
  const int m = (int)a.m;
  const int64_t total = (int64_t)m * (a.kreal ? 1 : 2) * a.k;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int gc = (int)(t / m), gr = (int)(t % m);
    R sr = 0, si = 0;
    for (int s = 0; s < splits; ++s) {
      const C z = ws[(int64_t)s * total + t];
      sr += z.re;
      si += z.im;
    }
    epilogue_store<R, C>(a, gr, gc, sr, si);
    if (a.kreal) epilogue_store<R, C>(a, gr, gc + a.k, sr, si);
  }
}

struct Plan {
  int cfg, splits, kps;
  int64_t tiles;
};

// Largest K split of one launch: narrow launches (2k <= 32) need 32 splits
// of the m / 256 row tiles to give every CU two workgroups.
constexpr int MAX_SPLITS = 32;

// Pick the tile shape and K split that minimise (rounds of 256 x occ
// workgroups, occ sharing a CU) x occ x (K slabs per workgroup) x (outputs
// per tile) / (relative MFMA efficiency of the shape) x (1 + split_penalty
// per extra split: each split costs a partial-sum write and read).  The
// efficiencies of the c64 shapes were fitted to a sweep of every shape and
// split over 2k = 32 ... 520 on the m = 4000 workload (the fitted plans came
// within 1% of the fastest ones in total time).
template <int NCFG>
Plan make_plan(int64_t m, int64_t n2, const int (&bm)[NCFG], const int (&bn)[NCFG], const int (&bk)[NCFG],
               const double (&eff)[NCFG], const int (&occ)[NCFG], double split_penalty, size_t elem,
               size_t ws_bytes, int ncfg = NCFG) {
  Plan best{0, 1, 1, 0};
  double best_cost = 1e300;
  for (int c = 0; c < ncfg; ++c) {
    const int64_t kt = 2 * ceil_div(m, bk[c]);
    const int64_t tiles = ceil_div(m, bm[c]) * ceil_div(n2, bn[c]);
    for (int s = 1; s <= MAX_SPLITS; ++s) {
      if (s > 1 && (size_t)s * m * n2 * elem > ws_bytes) break;
      const int64_t kps = ceil_div(kt, s);
      const int64_t real_s = ceil_div(kt, kps);
      // occ[c] workgroups share a CU, each at 1 / occ[c] of its speed
      const int64_t rounds = ceil_div(tiles * real_s, (int64_t)256 * occ[c]) * occ[c];
      const double cost = (double)rounds * kps * bk[c] * bm[c] * bn[c] * (1.0 + split_penalty * (real_s - 1)) / eff[c];
      if (cost < best_cost * 0.999) {
        best_cost = cost;
        best = Plan{c, (int)real_s, (int)kps, tiles};
      }
    }
  }
  return best;
}

template <typename Tr, int BM, int BN, int BK, int WGM, int WGN, int VB>
Err launch_cfg(const ApplyHArgs<typename Tr::R>& a, const Plan& p, void* ws, hipStream_t s) {
  using C = typename Tr::C;
  const int64_t grid = p.tiles * p.splits;
  hipLaunchKernelGGL((apply_h_kernel<Tr, BM, BN, BK, WGM, WGN, VB>), dim3((unsigned)grid), dim3(64 * WGM * WGN), 0,
                     s, a, p.splits, p.kps, (C*)ws);
  CHASE_LAUNCH_CHECK();
  if (p.splits > 1) {
    const int64_t total = a.m * (a.kreal ? 1 : 2) * (int64_t)a.k;
    const int blocks = (int)std::min<int64_t>(ceil_div(total, 256), 8192);
    hipLaunchKernelGGL((apply_h_reduce<typename Tr::R, C>), dim3(blocks), dim3(256), 0, s, a, p.splits, (const C*)ws);
    CHASE_LAUNCH_CHECK();
  }
  return ok();
}

template <typename Tr, int BN>
Err launch_dma(const ApplyHArgs<float>& a, const Plan& p, void* ws, hipStream_t s) {
  const int64_t grid = p.tiles * p.splits;
  hipLaunchKernelGGL((apply_h_dma_kernel<Tr, BN>), dim3((unsigned)grid), dim3(256), 0, s, a, p.splits, p.kps,
                     (c64*)ws);
  CHASE_LAUNCH_CHECK();
  if (p.splits > 1) {
    const int64_t total = a.m * 2 * (int64_t)a.k;
    const int blocks = (int)std::min<int64_t>(ceil_div(total, 256), 8192);
    hipLaunchKernelGGL((apply_h_reduce<float, c64>), dim3(blocks), dim3(256), 0, s, a, p.splits, (const c64*)ws);
    CHASE_LAUNCH_CHECK();
  }
  return ok();
}

// CHASE_PH_APPLY_PLAN="cfg,splits" forces a tile shape and K split, so that
// every tile shape and split can be checked for parity on one problem.
template <int NCFG>
void plan_override(Plan& p, int64_t m, int64_t n2, const int (&bm)[NCFG], const int (&bn)[NCFG],
                   const int (&bk)[NCFG], size_t elem, size_t ws_bytes) {
  const char* e = std::getenv("CHASE_PH_APPLY_PLAN");
  if (!e) return;
  int c = 0, s = 1;
  if (std::sscanf(e, "%d,%d", &c, &s) != 2 || c < 0 || c >= NCFG || s < 1) return;
  const int64_t kt = 2 * ceil_div(m, bk[c]);
  if (s > 1 && (size_t)s * m * n2 * elem > ws_bytes) return;
  p.cfg = c;
  p.kps = (int)ceil_div(kt, s);
  p.splits = (int)ceil_div(kt, p.kps);
  p.tiles = ceil_div(m, bm[c]) * ceil_div(n2, bn[c]);
}

}  // namespace

static Err launch_one_f32(const ApplyHArgs<float>& a, void* ws, size_t ws_bytes, hipStream_t s) {
  if (a.k <= 0 || a.m <= 0) return ok();
  if (a.kreal) return fail(CHASE_PH_ERR_ARG, "apply_h: K-real columns are a c128 mode");
  // 32 x 32 MFMA tiles: 0 (256 x 64), 3 (128 x 64), 4 (128 x 128); 16 x 16
  // MFMA tiles, whose widths cover N = 2k with less padding: 1 (256 x 32),
  // 2 (256 x 48), 5 (128 x 32), 6 (128 x 48).  All fit two workgroups per
  // CU, 5 and 6 three (LDS bound).  Wider 16 x 16 tiles need more
  // accumulators than one wave holds without extra register moves.
  // eff / occ fitted as described at make_plan.
  // Direct-to-LDS tiles (apply_h_dma_kernel): 7 (256 x 64, 32 x 32 MFMA),
  // 8 (256 x 32, 16 x 16 MFMA, for narrow launches; a 256 x 64 tile on the
  // 16 x 16 MFMA would spill).
  static const int bm[9] = {256, 256, 256, 128, 128, 128, 128, 256, 256};
  static const int bn[9] = {64, 32, 48, 64, 128, 32, 48, 64, 32};
  static const int bk[9] = {16, 16, 16, 16, 16, 16, 16, 8, 8};
  static const double eff[9] = {1.0, 0.9, 0.95, 0.95, 0.9, 0.85, 0.9, 1.1, 1.0};
  static const int occ[9] = {2, 2, 2, 2, 2, 3, 3, 2, 2};
  const bool vb2 = (a.m % 2 == 0) && (a.ldx % 2 == 0) && ((reinterpret_cast<uintptr_t>(a.X) & 15) == 0);
  const bool dma_ok = vb2 && !a.a_conj && a.m >= 2 && (a.lda % 2 == 0) &&
                      ((reinterpret_cast<uintptr_t>(a.A) & 15) == 0) && ((reinterpret_cast<uintptr_t>(a.B) & 15) == 0);
  const size_t wsb = ws ? ws_bytes : 0;
  Plan p = make_plan<9>(a.m, 2 * (int64_t)a.k, bm, bn, bk, eff, occ, 0.01, sizeof(c64), wsb, dma_ok ? 9 : 7);
  plan_override<9>(p, a.m, 2 * (int64_t)a.k, bm, bn, bk, sizeof(c64), wsb);
  if (p.cfg >= 7 && !dma_ok) p.cfg = p.cfg == 8 ? 1 : 0;
  switch (p.cfg) {
    case 0:
      return vb2 ? launch_cfg<TF32, 256, 64, 16, 4, 1, 2>(a, p, ws, s)
                 : launch_cfg<TF32, 256, 64, 16, 4, 1, 1>(a, p, ws, s);
    case 1: return launch_cfg<TF32S, 256, 32, 16, 4, 1, 1>(a, p, ws, s);
    case 2: return launch_cfg<TF32S, 256, 48, 16, 4, 1, 1>(a, p, ws, s);
    case 3:
      return vb2 ? launch_cfg<TF32, 128, 64, 16, 2, 2, 2>(a, p, ws, s)
                 : launch_cfg<TF32, 128, 64, 16, 2, 2, 1>(a, p, ws, s);
    case 4:
      return vb2 ? launch_cfg<TF32, 128, 128, 16, 2, 2, 2>(a, p, ws, s)
                 : launch_cfg<TF32, 128, 128, 16, 2, 2, 1>(a, p, ws, s);
    case 5: return launch_cfg<TF32S, 128, 32, 16, 2, 2, 1>(a, p, ws, s);
    case 6: return launch_cfg<TF32S, 128, 48, 16, 4, 1, 1>(a, p, ws, s);
    case 7: return launch_dma<TF32, 64>(a, p, ws, s);
    default: return launch_dma<TF32S, 32>(a, p, ws, s);
  }
}

static Err launch_one_f64(const ApplyHArgs<double>& a, void* ws, size_t ws_bytes, hipStream_t s) {
  if (a.k <= 0 || a.m <= 0) return ok();
  // 0, 1: one workgroup per CU; 2, 3: smaller K slab or tile, two per CU
  // (2 reaches 70-77% of the FP64 peak on the m = 4000 shapes); eff fitted to
  // a sweep of every shape and split over 2k = 32 ... 1040
  static const int bm[4] = {128, 256, 128, 64}, bn[4] = {64, 32, 64, 64}, bk[4] = {16, 16, 8, 16};
  static const double eff[4] = {1.0, 0.8, 1.2, 0.8};
  static const int occ[4] = {1, 1, 2, 2};
  const size_t wsb = ws ? ws_bytes : 0;
  const int64_t n2 = (a.kreal ? 1 : 2) * (int64_t)a.k;
  Plan p = make_plan<4>(a.m, n2, bm, bn, bk, eff, occ, 0.02, sizeof(c128), wsb);
  plan_override<4>(p, a.m, n2, bm, bn, bk, sizeof(c128), wsb);
  switch (p.cfg) {
    case 0: return launch_cfg<TF64, 128, 64, 16, 2, 2, 1>(a, p, ws, s);
    case 1: return launch_cfg<TF64, 256, 32, 16, 4, 1, 1>(a, p, ws, s);
    case 2: return launch_cfg<TF64, 128, 64, 8, 2, 2, 1>(a, p, ws, s);
    default: return launch_cfg<TF64, 64, 64, 16, 2, 2, 1>(a, p, ws, s);
  }
}

// When 2k is a few columns past a multiple of 64 (e.g. k = 260 or k = 73;
// k >= 64), the 64-wide tiles of the last tile column are mostly padding.
// The launch is then split by columns (H X is column-wise, and so is the
// fused epilogue): the first k - r columns, 2(k - r) a multiple of 64, on the
// caller's stream, and the last r <= 20 (c64; c128: 16) on the side stream, queued after the main
// launch, so that its workgroups take the CU slots the main launch frees in
// its last round and during its split-K reduction.  Event fork / join keep
// the pair ordered with the caller's stream.
template <typename R>
Err launch_split(const ApplyHArgs<R>& a, void* ws, size_t ws_bytes, hipStream_t s, const SideStream* side,
                 Err (*one)(const ApplyHArgs<R>&, void*, size_t, hipStream_t)) {
  constexpr int gran = 32;
  const int krem = a.k % gran;
  // c64: split when the last r = k mod 32 columns (2r of the 2k) fit in at
  // most three 16-column fragments of the narrow tile (measured inside the
  // filter on m = 4000, r = 17 and 20 gain 3-5% over the whole launch, r = 22
  // and 26 lose 7-20%); c128: r <= 16.
  constexpr int rmax = sizeof(R) == 4 ? 20 : 16;
  if (!side || !side->st || !ws || krem == 0 || krem > rmax || a.k < 2 * gran || a.kreal)
    return one(a, ws, ws_bytes, s);
  using C = typename ApplyHArgs<R>::C;
  ApplyHArgs<R> am = a, ar = a;
  am.k = a.k - krem;
  ar.k = krem;
  const int64_t c0 = am.k;
  ar.X = a.X + c0 * a.ldx;
  ar.Y = a.Y + c0 * a.ldy;
  if (a.P) ar.P = a.P + c0 * a.ldp;
  if (a.Q) ar.Q = a.Q + c0 * a.ldq;
  if (a.S) ar.S = a.S + c0 * a.lds;
  if (a.dcol) ar.dcol = a.dcol + c0;
  // the remainder's split-K partials (up to MAX_SPLITS) at the top of ws
  size_t rem_bytes = (size_t)MAX_SPLITS * a.m * 2 * krem * sizeof(C);
  rem_bytes = std::min(ceil_div((int64_t)rem_bytes, (int64_t)256) * 256, (int64_t)(ws_bytes / 4));
  const size_t main_bytes = (ws_bytes - rem_bytes) / 256 * 256;
  CHASE_HIP(hipEventRecord(side->fork, s));
  CHASE_HIP(hipStreamWaitEvent(side->st, side->fork, 0));
  CHASE_TRY(one(am, ws, main_bytes, s));
  CHASE_TRY(one(ar, static_cast<char*>(ws) + main_bytes, rem_bytes, side->st));
  CHASE_HIP(hipEventRecord(side->join, side->st));
  CHASE_HIP(hipStreamWaitEvent(s, side->join, 0));
  return ok();
}

Err launch_apply_h_f32(const ApplyHArgs<float>& a, void* ws, size_t ws_bytes, hipStream_t s, const SideStream* side) {
  if (a.k <= 0 || a.m <= 0) return ok();
  return launch_split<float>(a, ws, ws_bytes, s, side, launch_one_f32);
}

Err launch_apply_h_f64(const ApplyHArgs<double>& a, void* ws, size_t ws_bytes, hipStream_t s, const SideStream* side) {
  if (a.k <= 0 || a.m <= 0) return ok();
  return launch_split<double>(a, ws, ws_bytes, s, side, launch_one_f64);
}

}  // namespace chase
