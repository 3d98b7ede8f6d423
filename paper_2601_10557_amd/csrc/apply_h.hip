// Block-structured product H X, H = [[A, B], [-conj(B), -conj(A)]]
// (Section 1, eq. 1.1), as one real GEMM over the real structure of H.
//
// H is real-linear on K-real vectors (Thm 3.1: H K conj = -K conj H): for
// u = [a; conj(a)],
//   H u = [t; -conj(t)],   t = A a + B conj(a) = (A + B) Re(a) + i (A - B) Im(a).
// Every column x = [x1; x2] splits into K-real parts, x = u + i v, with
//   a_u = (x1 + conj(x2)) / 2,   a_v = (x1 - conj(x2)) / (2 i),
// so that  H x = [t_u + i t_v; -conj(t_u) - i conj(t_v)].
// With D = [A+B, i(A-B)] column-interleaved (m x 2m complex: column 2p is
// A[:, p] + B[:, p], column 2p + 1 is i (A[:, p] - B[:, p])) read as a real
// 2m x 2m matrix M (real row 2i + s = component s of complex row i), the
// real coordinates [Re t_0, Im t_0, Re t_1, ...] of t are M y for
// y = [Re a_0, Im a_0, Re a_1, ...].  So, for k columns of X,
//   Out = M Y,   Y = 2m x 2k real (column 2j: y of a_u of x_j; 2j + 1: of a_v),
// is one real GEMM of 2m x 2m by 2m x 2k: 16 m^2 k = 4 n^2 k real flops,
// half of the complex GEMM [A B] [X, K conj(X)] (32 m^2 k).  For K-real
// columns (x = u) it is 2m x 2m by 2m x k, 2 n^2 k flops.
//
// Pipeline of one product:
//  * pack: X (complex n x k) -> Y in k-pair layout: row pair (2p, 2p + 1)
//    of real column c at Yp[p * ldyr + 2 c + (0, 1)] (complex row p of the
//    operand), row pairs past m zero;
//  * GEMM: both operand tiles copied HBM -> LDS by the gfx950
//    direct-to-LDS load (global_load_lds_dwordx4: lane l's 16 bytes land at
//    the wave's LDS base + 16 l) into a ring of LDS stages, NST - 1 slabs
//    ahead; real MFMAs (f32 32x32x2 or 16x16x4, f64 16x16x4);
//  * epilogue: a lane holds the real and imaginary part of t for one
//    column of the pair (u_j or v_j) and takes the other from its
//    neighbour lane (l ^ 1); the u lane writes row i of H x_j, the v lane
//    row m + i, each fused with the Chebyshev three-term update
//      Y = alpha (H X) + beta P + gamma Q + diag(dcol) S.
// When the tile grid alone cannot fill the 256 CUs the K range is split;
// the real partial products go to a workspace and a second kernel sums them
// in a fixed order and applies the same epilogue.
//
// Tile order is XCD-aware: workgroups dispatched to the same XCD take
// consecutive tiles along N of one K range, i.e. they share one row strip of
// M in that XCD's L2.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "common.h"

namespace chase {
namespace {

// MFMA shapes.  phys_row(r, l): the real row (within a fragment of MB rows)
// of accumulator r of lane l; the accumulators 2t, 2t + 1 hold the real rows
// 2i, 2i + 1 of one complex row i.  a_row(l): the fragment row whose A
// operand lane l supplies (a permutation for the f64 shape, so that the
// output rows land as stated).
struct TF32 {  // v_mfma_f32_32x32x2f32
  using R = float;
  using C = c64;
  using Acc = floatx16;
  static constexpr int MB = 32, NB = 32, KB = 2, NACC = 16;
  __device__ static int a_row(int l) { return l & 31; }
  __device__ static int a_k(int l) { return l >> 5; }
  __device__ static int phys_row(int r, int l) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }
  __device__ static int acc_col(int l) { return l & 31; }
  __device__ static Acc mfma(R a, R b, Acc c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
};

struct TF32S {  // v_mfma_f32_16x16x4f32: narrow launches
  using R = float;
  using C = c64;
  using Acc = floatx4;
  static constexpr int MB = 16, NB = 16, KB = 4, NACC = 4;
  __device__ static int a_row(int l) { return l & 15; }
  __device__ static int a_k(int l) { return l >> 4; }
  __device__ static int phys_row(int r, int l) { return 4 * (l >> 4) + r; }
  __device__ static int acc_col(int l) { return l & 15; }
  __device__ static Acc mfma(R a, R b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

struct TF64 {  // v_mfma_f64_16x16x4f64
  using R = double;
  using C = c128;
  using Acc = doublex4;
  static constexpr int MB = 16, NB = 16, KB = 4, NACC = 4;
  // output row rho = (l >> 4) + 4 r of the MFMA is fed from real row
  // pi(rho) = 8 (r >> 1) + 2 (l >> 4) + (r & 1), so accumulators 0, 1 and 2, 3
  // of a lane are the real rows 2q, 2q + 1 and 8 + 2q, 9 + 2q (q = l >> 4)
  __device__ static int pi(int rho) { return 8 * ((rho >> 2) >> 1) + 2 * (rho & 3) + ((rho >> 2) & 1); }
  __device__ static int a_row(int l) { return pi(l & 15); }
  __device__ static int a_k(int l) { return l >> 4; }
  __device__ static int phys_row(int r, int l) { return pi((l >> 4) + 4 * r); }
  __device__ static int acc_col(int l) { return l & 15; }
  __device__ static Acc mfma(R a, R b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
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

// Y[orow, ocol] = alpha h + beta P + gamma Q + dcol S (each read before the
// write, so Y may alias P or Q)
template <typename R, typename C>
__device__ __forceinline__ void store_hx(const ApplyHArgs<R>& a, int64_t orow, int ocol, R hr, R hi) {
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

// Epilogue of complex row ci for real column col: (tr, ti) is t of this
// column (K-real: column col of X; otherwise u_j for even col, v_j for odd)
// and (pr, pi_) t of the other column of the pair.
template <typename R, typename C>
__device__ __forceinline__ void finish_pair(const ApplyHArgs<R>& a, int64_t ci, int col, R tr, R ti, R pr, R pi_) {
  const int64_t m = a.m;
  if (a.tda) {
    store_hx<R, C>(a, ci, col, tr, ti);        // A x
    return;
  }
  if (a.kreal) {
    store_hx<R, C>(a, ci, col, tr, ti);        // t
    store_hx<R, C>(a, ci + m, col, -tr, ti);   // -conj(t)
    return;
  }
  const int odd = col & 1;
  const R ur = odd ? pr : tr, ui = odd ? pi_ : ti, vr = odd ? tr : pr, vi = odd ? ti : pi_;
  if (!odd)
    store_hx<R, C>(a, ci, col >> 1, ur - vi, ui + vr);        // t_u + i t_v
  else
    store_hx<R, C>(a, ci + m, col >> 1, -ur - vi, ui - vr);   // -conj(t_u) - i conj(t_v)
}

__device__ __forceinline__ float shfl1(float v) { return __shfl_xor(v, 1); }
__device__ __forceinline__ double shfl1(double v) { return __shfl_xor(v, 1); }

// ---------------------------------------------------------------- pack
// Yp (k-pair layout, ldyr reals per row pair, rows >= m zero):
//  general: real columns 2j, 2j + 1 = coordinates of a_u, a_v of x_j (one
//           16-byte group [Re a_u, Im a_u, Re a_v, Im a_v] per row pair);
//  K-real:  real column j = coordinates of the top half of x_j (column k,
//           when k is odd, is zero); the same for the m-row x_j of a TDA
//           product.
template <typename R, typename C>
__global__ __launch_bounds__(256) void pack_kernel(const C* X, int64_t ldx, int64_t m, int k, int kreal, R* Y,
                                                   int64_t ldyr, int64_t rows) {
  // A tile of 64 row pairs p and TJ columns j goes through LDS: the reads
  // of X run along rows (coalesced), the writes along the row pair's
  // CW * TJ = 64 contiguous reals of Y.
  constexpr int TP = 64, NR = 64;
  __shared__ R s[TP][NR + 1];
  const int cw = kreal ? 2 : 4;          // reals per (row pair, column)
  const int tj = NR / cw;                // columns per tile
  const int kc = kreal ? (k + 1) / 2 * 2 : k;
  const int64_t p0 = (int64_t)blockIdx.x * TP;
  const int j0 = blockIdx.y * tj;
  const int tid = threadIdx.x;
  for (int t = tid; t < TP * tj; t += 256) {
    const int pp = t % TP, jj = t / TP;
    const int64_t p = p0 + pp;
    const int j = j0 + jj;
    R q0 = 0, q1 = 0, q2 = 0, q3 = 0;
    if (p < m && j < k) {
      const C x1 = X[(int64_t)j * ldx + p];
      if (kreal) {
        q0 = x1.re;
        q1 = x1.im;
      } else {
        const C x2 = X[(int64_t)j * ldx + m + p];
        q0 = R(0.5) * (x1.re + x2.re);   // Re a_u
        q1 = R(0.5) * (x1.im - x2.im);   // Im a_u
        q2 = R(0.5) * (x1.im + x2.im);   // Re a_v
        q3 = R(0.5) * (x2.re - x1.re);   // Im a_v
      }
    }
    s[pp][cw * jj] = q0;
    s[pp][cw * jj + 1] = q1;
    if (!kreal) {
      s[pp][cw * jj + 2] = q2;
      s[pp][cw * jj + 3] = q3;
    }
  }
  __syncthreads();
  const int nreal = cw * (min(kc, j0 + tj) - j0);  // reals of this tile in one row pair
  for (int t = tid; t < TP * NR; t += 256) {
    const int pp = t / NR, c = t % NR;
    const int64_t p = p0 + pp;
    if (p < rows && c < nreal) Y[p * ldyr + (int64_t)cw * j0 + c] = s[pp][c];
  }
}

// -------------------------------------------------------------- GEMM
// Direct-to-LDS copy of 16 bytes per lane to lds_base + 16 lane (M0 is
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

// s_waitcnt vmcnt(N) with expcnt and lgkmcnt left alone (gfx9 encoding:
// vmcnt[3:0] in bits 3:0, vmcnt[5:4] in bits 15:14)
template <int N>
__device__ __forceinline__ void vm_wait() {
  static_assert(N >= 0 && N < 64, "vmcnt");
  __builtin_amdgcn_s_waitcnt((N & 15) | (0x7 << 4) | (0xF << 8) | ((N >> 4) << 14));
}

// Workgroup barrier for the ring: this wave's LDS reads are complete
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

template <typename Tr, int BM, int BN, int BK, int NST, int WGM, int WGN>
struct Cfg {
  using R = typename Tr::R;
  static constexpr int V = 16 / (int)sizeof(R);          // reals per 16-byte copy
  static constexpr int WTM = BM / WGM, WTN = BN / WGN;   // wave tile
  static constexpr int FM = WTM / Tr::MB, FN = WTN / Tr::NB;
  static constexpr int CW = 64 * V / 2;                  // Y columns per copy (one row pair)
  static constexpr int BNP = (BN + CW - 1) / CW * CW;     // Y columns per LDS row pair
  // k-row pitch of the M stage: a 32-lane half of a wave reads 32 words of
  // one k row and the other half the next k row (f32); half a pitch of 32
  // words puts the two halves on disjoint banks (f64: 16 doubles)
  static constexpr int SA = BM + (sizeof(R) == 4 ? 32 : 16);
  static constexpr int PARTS = BM / (64 * V);             // copies per k column of M
  static constexpr int ACOP = BK * PARTS;                 // copies of the M tile per slab
  static constexpr int BCOP = (BK / 2) * (BNP / CW);     // copies of the Y tile per slab
  static constexpr int NCOP = ACOP + BCOP;
  static constexpr int NCW = NCOP / 4;                    // per wave
  static constexpr int ASTAGE = BK * SA;                  // reals
  static constexpr int BSTAGE = (BK / 2) * BNP * 2;       // reals
  static_assert(WGM * WGN == 4, "four waves");
  static_assert(BM % (64 * V) == 0, "tile rows");
  static_assert(BK % 2 == 0 && BK % Tr::KB == 0, "slab");
  static_assert(NCOP % 4 == 0, "equal copies per wave");
  static_assert(WTM % Tr::MB == 0 && WTN % Tr::NB == 0, "wave tile");
  static_assert((NST - 2) * NCW < 64, "vmcnt");
  static constexpr size_t LDS = (size_t)NST * (ASTAGE + BSTAGE) * sizeof(R);
  static_assert(LDS <= 80 * 1024, "two workgroups per CU");
};

// Out = M Y over K-slabs [kt_beg, kt_beg + kps) of BK reals; M from D
// (complex m x 2m, ldd, read as real 2m x 2m with ld 2 ldd), Y from a.yr
// (k-pair layout).  Needs 16-byte aligned D and yr, ldd a multiple of 8,
// ldyr >= 2 N rounded up to 2 columns, and row pairs of yr up to 2m rounded
// up to BK.
// Scheduling of one K step (measured on the m = 4000 shapes): SCHED 1 lets
// the compiler interleave the fragment reads of the slab with its MFMAs
// (iglp_opt(0): 72-77% of the FP32 peak on the 256 x 128 tile against
// 69-73% without); SCHED 3 places one read after every two MFMAs (c128
// 128 x 128 tile: 76% against 74%).
template <int SCHED>
__device__ __forceinline__ void step_schedule() {
  if constexpr (SCHED == 1) __builtin_amdgcn_iglp_opt(0);
  if constexpr (SCHED == 3) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // 2 MFMA
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // 1 DS read
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);
  }
}

// One tile of the GEMM: workgroup bid of the T * splits workgroups of a
// product (T tiles, K split `splits` ways, kps slabs each), on the LDS ring
// at lds (NST stages of the M tile, then NST stages of the Y tile).
template <typename Tr, int BM, int BN, int BK, int NST, int WGM, int WGN, int SCHED>
__device__ __forceinline__ void hx_tile(const ApplyHArgs<typename Tr::R>& a, int splits, int kps,
                                        typename Tr::R* ws, int bid, typename Tr::R* lds) {
  using CF = Cfg<Tr, BM, BN, BK, NST, WGM, WGN>;
  using R = typename Tr::R;
  using C = typename Tr::C;
  constexpr int V = CF::V, FM = CF::FM, FN = CF::FN, BNP = CF::BNP, SA = CF::SA;
  R (*As)[CF::ASTAGE] = reinterpret_cast<R (*)[CF::ASTAGE]>(lds);
  R (*Bs)[CF::BSTAGE] = reinterpret_cast<R (*)[CF::BSTAGE]>(lds + NST * CF::ASTAGE);

  const int64_t m = a.m;
  const int M2 = (int)(2 * m);                       // real rows and K
  const int N = (a.kreal || a.tda) ? a.k : 2 * a.k;  // real columns
  const int Npad = (N + 1) / 2 * 2;                  // packed columns
  const int TM = (M2 + BM - 1) / BM;
  const int TN = (N + BN - 1) / BN;
  const int T = TM * TN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nid = xcd_remap(bid, T * splits);
  const int sp = nid / T;
  const int t = nid - sp * T;
  const int m0 = (t / TN) * BM;
  const int n0 = (t % TN) * BN;
  const int nkt = (M2 + BK - 1) / BK;
  const int kt_beg = sp * kps;
  const int nsl = max(0, min(nkt, kt_beg + kps) - kt_beg);
  const int wm0 = (wave / WGN) * CF::WTM;
  const int wn0 = (wave % WGN) * CF::WTN;

  const R* Md = reinterpret_cast<const R*>(a.D);
  const int64_t ldm = 2 * a.ldd;                      // real leading dimension of M
  const R* Yd = a.yr;
  const unsigned as_base = (unsigned)(uintptr_t)&As[0][0];
  const unsigned bs_base = (unsigned)(uintptr_t)&Bs[0][0];

  // copies of slab kt into ring stage st.  Copy c of this wave is copy
  // g = wave * NCW + c of the slab: M copies first (k column kk, part pa of
  // 64 V rows), then Y copies (row pair kp, block cb of CW columns: V / 2
  // columns per lane).  Rows of M past 2m and k columns past 2m are read
  // from clamped addresses (their products are never stored, or multiply
  // the zero row pairs of Y); columns of Y past N repeat the last ones
  // (never stored).
  auto copy_slab = [&](int kt, int st) {
    const int kk0 = kt * BK;
#pragma unroll
    for (int c = 0; c < CF::NCW; ++c) {
      const int g = wave * CF::NCW + c;
      if (g < CF::ACOP) {
        const int kk = g / CF::PARTS, pa = g % CF::PARTS;
        const int64_t col = min(kk0 + kk, M2 - 1);
        const int64_t row = min((int64_t)(m0 + pa * 64 * V + lane * V), ldm - V);
        const unsigned dst = __builtin_amdgcn_readfirstlane(
            as_base + (unsigned)((st * CF::ASTAGE + kk * SA + pa * 64 * V) * sizeof(R)));
        lds_copy16(Md + col * ldm + row, dst);
      } else {
        const int gb = g - CF::ACOP;
        constexpr int CBS = BNP / CF::CW;
        const int kp = gb / CBS, cb = gb % CBS;
        const int64_t col = min(n0 + cb * CF::CW + lane * (V / 2), Npad - V / 2);
        const int64_t rp = kk0 / 2 + kp;
        const unsigned dst = __builtin_amdgcn_readfirstlane(
            bs_base + (unsigned)((st * CF::BSTAGE + (kp * BNP + cb * CF::CW) * 2) * sizeof(R)));
        lds_copy16(Yd + rp * a.ldyr + 2 * col, dst);
      }
    }
  };

  typename Tr::Acc acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < Tr::NACC; ++r) acc[i][j][r] = R(0);

  const int ak = Tr::a_k(lane), arow = Tr::a_row(lane), bcol = Tr::acc_col(lane);
  const int live = (N - (n0 + wn0) + Tr::NB - 1) / Tr::NB;  // wave-uniform

  constexpr int PRE = NST - 1;
  if (nsl > 0) {
#pragma unroll
    for (int q = 0; q < PRE; ++q) copy_slab(kt_beg + min(q, nsl - 1), q);
    vm_wait<(NST - 2) * CF::NCW>();  // slab 0 landed
  }
  ring_barrier();

  auto kloop = [&](auto NLc) {
    constexpr int NL = decltype(NLc)::value;
    for (int s = 0; s < nsl; ++s) {
      const int st = s % NST;
      copy_slab(kt_beg + min(s + PRE, nsl - 1), (s + PRE) % NST);
      if constexpr (NL > 0) {
        const R* Ast = &As[st][0];
        const R* Bst = &Bs[st][0];
        // fragments of step ks + KB are read before the MFMAs of step ks
        // (two register sets), so the LDS latency hides behind the MFMAs
        R fa[2][FM], fb[2][NL];
        auto load = [&](int ks, int b) {
          const int k = ks + ak;
#pragma unroll
          for (int i = 0; i < FM; ++i) fa[b][i] = Ast[k * SA + wm0 + i * Tr::MB + arow];
#pragma unroll
          for (int j = 0; j < NL; ++j) fb[b][j] = Bst[((k >> 1) * BNP + wn0 + j * Tr::NB + bcol) * 2 + (k & 1)];
        };
        load(0, 0);
#pragma unroll
        for (int ks = 0; ks < BK; ks += Tr::KB) {
          const int b = (ks / Tr::KB) & 1;
          if (ks + Tr::KB < BK) load(ks + Tr::KB, b ^ 1);
          // f32: raised issue priority while this wave feeds the matrix
          // core, so that the other wave on the SIMD takes its copy / wait /
          // barrier part meanwhile (c64 calls 2.5-5% faster on m = 4000,
          // k = 64..260; the f64 tiles, scheduled by sched_group_barrier,
          // were 5-7% slower with it)
          if constexpr (sizeof(R) == 4) __builtin_amdgcn_s_setprio(1);
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < NL; ++j) acc[i][j] = Tr::mfma(fa[b][i], fb[b][j], acc[i][j]);
          if constexpr (sizeof(R) == 4) __builtin_amdgcn_s_setprio(0);
          step_schedule<SCHED>();
        }
      }
      // slab s + 1 landed for this wave: the copies of the NST - 2 slabs
      // after it may still be in flight
      vm_wait<(NST - 2) * CF::NCW>();
      ring_barrier();
    }
  };
  const int nl = min(live, FN);
  static_for_n<0, FN + 1>([&](auto NLc) {
    if (nl == decltype(NLc)::value) kloop(NLc);
  });
  vm_wait<0>();  // the trailing repeat copies

  R* wsp = ws + (int64_t)sp * M2 * N;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < Tr::NACC; r += 2) {
        const int row = m0 + wm0 + i * Tr::MB + Tr::phys_row(r, lane);   // even
        const int col = n0 + wn0 + j * Tr::NB + bcol;
        const R tr = acc[i][j][r], ti = acc[i][j][r + 1];
        if (splits > 1) {
          if (row < M2 && col < N) {
            wsp[(int64_t)col * M2 + row] = tr;
            wsp[(int64_t)col * M2 + row + 1] = ti;
          }
        } else {
          const R pr = shfl1(tr), pi_ = shfl1(ti);
          if (row < M2 && col < N) finish_pair<R, C>(a, row >> 1, col, tr, ti, pr, pi_);
        }
      }
}

template <typename Tr, int BM, int BN, int BK, int NST, int WGM, int WGN, int SCHED = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void hx_kernel(
    const ApplyHArgs<typename Tr::R> a, int splits, int kps, typename Tr::R* ws) {
  using CF = Cfg<Tr, BM, BN, BK, NST, WGM, WGN>;
  using R = typename Tr::R;
  __shared__ __attribute__((aligned(16))) R lds[CF::LDS / sizeof(R)];
  hx_tile<Tr, BM, BN, BK, NST, WGM, WGN, SCHED>(a, splits, kps, ws, blockIdx.x, lds);
}

// A split product in one launch: the last few columns on their own tile
// shape and K split, next to the main columns, without a second stream.
// The f32 remainder workgroups come first (0 .. nrem - 1) and spread over the
// CUs while the main tiles fill the rest; the f64 ones come after the main
// tiles, where they fill the CUs the last main tiles leave idle (2-3% faster
// f64 calls at k = 260, no change in f32).  Each part starts at a multiple of
// 8 (nrem and nmain rounded up, the padding workgroups exit at once) so that
// the XCD of a workgroup stays blockIdx mod 8 in both.
template <typename Tr, int BM, int BN, int BK, int NST, int WGM, int WGN, int SCHED, int BMR, int BNR, int BKR,
          int NSTR, int WGMR, int WGNR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void hx_pair_kernel(
    const ApplyHArgs<typename Tr::R> am, int splits_m, int kps_m, typename Tr::R* ws_m,
    const ApplyHArgs<typename Tr::R> ar, int splits_r, int kps_r, typename Tr::R* ws_r, int nrem, int nrem_live,
    int nmain, int nmain_live) {
  using R = typename Tr::R;
  constexpr size_t LM = Cfg<Tr, BM, BN, BK, NST, WGM, WGN>::LDS;
  constexpr size_t LR = Cfg<Tr, BMR, BNR, BKR, NSTR, WGMR, WGNR>::LDS;
  __shared__ __attribute__((aligned(16))) R lds[(LM > LR ? LM : LR) / sizeof(R)];
  const int bid = blockIdx.x;
  constexpr bool rem_first = sizeof(R) == 4;
  const int rb = rem_first ? bid : bid - nmain;  // remainder workgroup, if >= 0
  const int mb = rem_first ? bid - nrem : bid;   // main workgroup, if >= 0
  if (rem_first ? bid < nrem : bid >= nmain) {
    if (rb < nrem_live) hx_tile<Tr, BMR, BNR, BKR, NSTR, WGMR, WGNR, 0>(ar, splits_r, kps_r, ws_r, rb, lds);
  } else {
    if (mb < nmain_live) hx_tile<Tr, BM, BN, BK, NST, WGM, WGN, SCHED>(am, splits_m, kps_m, ws_m, mb, lds);
  }
}

// Sum the split-K partials in a fixed order and apply the epilogue: one
// thread per complex row i and X column j.
template <typename R, typename C>
__global__ void hx_reduce(const ApplyHArgs<R> a, int splits, const R* ws) {
  const int64_t m = a.m, M2 = 2 * m;
  const int N = (a.kreal || a.tda) ? a.k : 2 * a.k;
  const int64_t total = m * a.k;
  const int64_t split_stride = M2 * N;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / m);
    const int64_t i = t % m;
    if (a.kreal || a.tda) {
      R tr = 0, ti = 0;
      for (int s = 0; s < splits; ++s) {
        const R* w = ws + s * split_stride + (int64_t)j * M2 + 2 * i;
        tr += w[0];
        ti += w[1];
      }
      finish_pair<R, C>(a, i, j, tr, ti, R(0), R(0));
      continue;
    }
    R ur = 0, ui = 0, vr = 0, vi = 0;
    for (int s = 0; s < splits; ++s) {
      const R* w = ws + s * split_stride + (int64_t)(2 * j) * M2 + 2 * i;
      ur += w[0];
      ui += w[1];
      vr += w[M2];
      vi += w[M2 + 1];
    }
    finish_pair<R, C>(a, i, 2 * j, ur, ui, vr, vi);
    finish_pair<R, C>(a, i, 2 * j + 1, vr, vi, ur, ui);
  }
}

struct Plan {
  int cfg, splits, kps;
  int64_t tiles;
};

// Largest K split of one launch: narrow launches need many splits of the
// row tiles to give every CU two workgroups.
constexpr int MAX_SPLITS = 32;

// Pick the tile shape and K split that minimise (rounds of 256 x occ
// workgroups, occ sharing a CU) x occ x (K slabs per workgroup) x (outputs
// per tile) / (relative MFMA efficiency of the shape) x (1 + split_penalty
// per extra split: each split costs a partial-sum write and read).
template <int NCFG>
Plan make_plan(int64_t m2, int64_t n2, const int (&bm)[NCFG], const int (&bn)[NCFG], const int (&bk)[NCFG],
               const double (&eff)[NCFG], const int (&occ)[NCFG], double split_penalty, size_t elem,
               size_t ws_bytes, int ncfg) {
  Plan best{0, 1, 1, ceil_div(m2, bm[0]) * ceil_div(n2, bn[0])};
  double best_cost = 1e300;
  for (int c = 0; c < ncfg; ++c) {
    const int64_t kt = ceil_div(m2, bk[c]);
    const int64_t tiles = ceil_div(m2, bm[c]) * ceil_div(n2, bn[c]);
    for (int s = 1; s <= MAX_SPLITS; ++s) {
      if (s > 1 && (size_t)s * m2 * n2 * elem > ws_bytes) break;
      const int64_t kps = ceil_div(kt, s);
      const int64_t real_s = ceil_div(kt, kps);
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

// CHASE_PH_APPLY_PLAN="cfg,splits" forces a tile shape and K split, so that
// every tile shape and split can be checked for parity on one problem.
template <int NCFG>
void plan_override(Plan& p, int64_t m2, int64_t n2, const int (&bm)[NCFG], const int (&bn)[NCFG],
                   const int (&bk)[NCFG], size_t elem, size_t ws_bytes) {
  const char* e = std::getenv("CHASE_PH_APPLY_PLAN");
  if (!e) return;
  int c = 0, s = 1;
  if (std::sscanf(e, "%d,%d", &c, &s) != 2 || c < 0 || c >= NCFG || s < 1) return;
  const int64_t kt = ceil_div(m2, bk[c]);
  if (s > 1 && (size_t)s * m2 * n2 * elem > ws_bytes) return;
  p.cfg = c;
  p.kps = (int)ceil_div(kt, s);
  p.splits = (int)ceil_div(kt, p.kps);
  p.tiles = ceil_div(m2, bm[c]) * ceil_div(n2, bn[c]);
}

template <typename R, typename C>
Err launch_reduce(const ApplyHArgs<R>& a, int splits, const R* ws, hipStream_t s) {
  if (splits <= 1) return ok();
  const int64_t total = a.m * (int64_t)a.k;
  const int blocks = (int)std::min<int64_t>(ceil_div(total, 256), 8192);
  hipLaunchKernelGGL((hx_reduce<R, C>), dim3(blocks), dim3(256), 0, s, a, splits, ws);
  CHASE_LAUNCH_CHECK();
  return ok();
}

template <typename Tr, int BM, int BN, int BK, int NST, int WGM, int WGN, int SCHED = 0>
Err launch_cfg(const ApplyHArgs<typename Tr::R>& a, const Plan& p, void* ws, hipStream_t s) {
  using R = typename Tr::R;
  using C = typename Tr::C;
  const int64_t grid = p.tiles * p.splits;
  hipLaunchKernelGGL((hx_kernel<Tr, BM, BN, BK, NST, WGM, WGN, SCHED>), dim3((unsigned)grid), dim3(256), 0, s, a, p.splits,
                     p.kps, (R*)ws);
  CHASE_LAUNCH_CHECK();
  return launch_reduce<R, C>(a, p.splits, (const R*)ws, s);
}

// Main part on tile shape (BM, BN, ...), remainder on (BMR, BNR, ...).
template <typename Tr, int BM, int BN, int BK, int NST, int WGM, int WGN, int SCHED, int BMR, int BNR, int BKR,
          int NSTR, int WGMR, int WGNR>
Err launch_pair_cfg(const ApplyHArgs<typename Tr::R>& am, const Plan& pm, void* wsm,
                    const ApplyHArgs<typename Tr::R>& ar, const Plan& pr, void* wsr, hipStream_t s) {
  using R = typename Tr::R;
  using C = typename Tr::C;
  const int live = (int)(pr.tiles * pr.splits);
  const int nrem = (live + 7) / 8 * 8;
  const int main_live = (int)(pm.tiles * pm.splits);
  const int nmain = (main_live + 7) / 8 * 8;
  const int64_t grid = (int64_t)nrem + nmain;
  hipLaunchKernelGGL((hx_pair_kernel<Tr, BM, BN, BK, NST, WGM, WGN, SCHED, BMR, BNR, BKR, NSTR, WGMR, WGNR>),
                     dim3((unsigned)grid), dim3(256), 0, s, am, pm.splits, pm.kps, (R*)wsm, ar, pr.splits, pr.kps,
                     (R*)wsr, nrem, live, nmain, main_live);
  CHASE_LAUNCH_CHECK();
  CHASE_TRY((launch_reduce<R, C>(am, pm.splits, (const R*)wsm, s)));
  return launch_reduce<R, C>(ar, pr.splits, (const R*)wsr, s);
}

// Tile shapes (BM x BN reals, K slab BK, NST ring stages), two workgroups
// per CU (at most 80 KB of LDS):
//  c64:  0  256 x 128, BK 16, 3 stages, 32x32x2 (wave tile 64 x 128), SCHED 1
//        1  256 x 64,  BK 16, 3 stages, 32x32x2 (64 x 64), SCHED 1
//        2  256 x 32,  BK 16, 3 stages, 16x16x4 (64 x 32; narrow launches)
//  c128: 0  128 x 128, BK 8,  4 stages, 16x16x4 f64 (2 x 2 waves of 64 x 64), SCHED 3
//        1  128 x 64,  BK 8,  4 stages (64 x 32)
//        2  128 x 32,  BK 8,  4 stages, 4 x 1 waves (32 x 32; narrow launches)
struct F32Tiles {
  static constexpr int bm[3] = {256, 256, 256}, bn[3] = {128, 64, 32}, bk[3] = {16, 16, 16};
  static constexpr double eff[3] = {1.0, 0.95, 0.8};
  static constexpr int occ[3] = {2, 2, 2};
  static constexpr double split_penalty = 0.01;
};
struct F64Tiles {
  static constexpr int bm[3] = {128, 128, 128}, bn[3] = {128, 64, 32}, bk[3] = {8, 8, 8};
  static constexpr double eff[3] = {1.0, 0.95, 0.8};
  static constexpr int occ[3] = {2, 2, 2};
  static constexpr double split_penalty = 0.02;
};

// Plan over the first ncfg tile shapes (the narrow shape alone: ncfg = 1
// starting at the last one).
template <typename T, typename R>
Plan plan_for(const ApplyHArgs<R>& a, size_t wsb, bool narrow_only) {
  const int64_t m2 = 2 * a.m, n2 = ((a.kreal || a.tda) ? 1 : 2) * (int64_t)a.k;
  if (narrow_only) {
    const int bm[1] = {T::bm[2]}, bn[1] = {T::bn[2]}, bk[1] = {T::bk[2]}, occ[1] = {T::occ[2]};
    const double eff[1] = {T::eff[2]};
    Plan p = make_plan<1>(m2, n2, bm, bn, bk, eff, occ, T::split_penalty, sizeof(R), wsb, 1);
    p.cfg = 2;
    return p;
  }
  Plan p = make_plan<3>(m2, n2, T::bm, T::bn, T::bk, T::eff, T::occ, T::split_penalty, sizeof(R), wsb, 3);
  plan_override<3>(p, m2, n2, T::bm, T::bn, T::bk, sizeof(R), wsb);
  return p;
}

Err launch_plan_f32(const ApplyHArgs<float>& a, const Plan& p, void* ws, hipStream_t s) {
  switch (p.cfg) {
    case 0: return launch_cfg<TF32, 256, 128, 16, 3, 4, 1, 1>(a, p, ws, s);
    case 1: return launch_cfg<TF32, 256, 64, 16, 3, 4, 1, 1>(a, p, ws, s);
    default: return launch_cfg<TF32S, 256, 32, 16, 3, 4, 1>(a, p, ws, s);
  }
}

Err launch_plan_f64(const ApplyHArgs<double>& a, const Plan& p, void* ws, hipStream_t s) {
  switch (p.cfg) {
    case 0: return launch_cfg<TF64, 128, 128, 8, 4, 2, 2, 3>(a, p, ws, s);
    case 1: return launch_cfg<TF64, 128, 64, 8, 4, 2, 2>(a, p, ws, s);
    default: return launch_cfg<TF64, 128, 32, 8, 4, 4, 1>(a, p, ws, s);
  }
}

// the remainder always on the narrow shape (16 x 16 MFMA for c64)
Err launch_pair_f32(const ApplyHArgs<float>& am, const Plan& pm, void* wsm, const ApplyHArgs<float>& ar,
                    const Plan& pr, void* wsr, hipStream_t s) {
  switch (pm.cfg) {
    case 0:
      return launch_pair_cfg<TF32, 256, 128, 16, 3, 4, 1, 1, 256, 32, 16, 3, 4, 1>(am, pm, wsm, ar, pr, wsr, s);
    case 1:
      return launch_pair_cfg<TF32, 256, 64, 16, 3, 4, 1, 1, 256, 32, 16, 3, 4, 1>(am, pm, wsm, ar, pr, wsr, s);
    default: {
      // both parts on the narrow shape: two plain launches in stream order
      CHASE_TRY((launch_cfg<TF32S, 256, 32, 16, 3, 4, 1>(am, pm, wsm, s)));
      return launch_cfg<TF32S, 256, 32, 16, 3, 4, 1>(ar, pr, wsr, s);
    }
  }
}

Err launch_pair_f64(const ApplyHArgs<double>& am, const Plan& pm, void* wsm, const ApplyHArgs<double>& ar,
                    const Plan& pr, void* wsr, hipStream_t s) {
  switch (pm.cfg) {
    case 0:
      return launch_pair_cfg<TF64, 128, 128, 8, 4, 2, 2, 3, 128, 32, 8, 4, 4, 1>(am, pm, wsm, ar, pr, wsr, s);
    case 1:
      return launch_pair_cfg<TF64, 128, 64, 8, 4, 2, 2, 0, 128, 32, 8, 4, 4, 1>(am, pm, wsm, ar, pr, wsr, s);
    default: {
      CHASE_TRY((launch_cfg<TF64, 128, 32, 8, 4, 4, 1>(am, pm, wsm, s)));
      return launch_cfg<TF64, 128, 32, 8, 4, 4, 1>(ar, pr, wsr, s);
    }
  }
}

template <typename R>
Err pack(const ApplyHArgs<R>& a, hipStream_t s) {
  using C = typename ApplyHArgs<R>::C;
  const bool kr = a.kreal || a.tda;
  const int kc = kr ? (a.k + 1) / 2 * 2 : a.k;
  const int tj = kr ? 32 : 16;
  const dim3 grid((unsigned)ceil_div(a.yrows, 64), (unsigned)ceil_div(kc, tj));
  hipLaunchKernelGGL((pack_kernel<R, C>), grid, dim3(256), 0, s, a.X, a.ldx, a.m, a.k, kr ? 1 : 0, a.yr, a.ldyr,
                     a.yrows);
  CHASE_LAUNCH_CHECK();
  return ok();
}

template <typename R>
struct PrecOps;
template <>
struct PrecOps<float> {
  using Tiles = F32Tiles;
  static Err one(const ApplyHArgs<float>& a, const Plan& p, void* ws, hipStream_t s) {
    return launch_plan_f32(a, p, ws, s);
  }
  static Err pair(const ApplyHArgs<float>& am, const Plan& pm, void* wsm, const ApplyHArgs<float>& ar,
                  const Plan& pr, void* wsr, hipStream_t s) {
    return launch_pair_f32(am, pm, wsm, ar, pr, wsr, s);
  }
};
template <>
struct PrecOps<double> {
  using Tiles = F64Tiles;
  static Err one(const ApplyHArgs<double>& a, const Plan& p, void* ws, hipStream_t s) {
    return launch_plan_f64(a, p, ws, s);
  }
  static Err pair(const ApplyHArgs<double>& am, const Plan& pm, void* wsm, const ApplyHArgs<double>& ar,
                  const Plan& pr, void* wsr, hipStream_t s) {
    return launch_pair_f64(am, pm, wsm, ar, pr, wsr, s);
  }
};

// c64 products with 64 < k <= 80 (2k = 130 .. 160 real columns) run on one
// column of wide tiles (256 x 160, 5 MFMA column blocks per wave, K slab 8 so
// that the ring stays within two workgroups per CU), which streams M once,
// instead of a 128-wide main column and a narrow remainder that streams M
// again (k = 73: 226 -> 211 us on m = 4000).  For larger k the same wide
// column after the main tiles was slower than the narrow remainder (k = 260:
// 642 against 595 us, also with a 16-deep slab and two stages), so those keep
// the split below.
constexpr int WIDE_REM = 16;
constexpr int WIDE_BN = 160, WIDE_BK = 8;

Err launch_wide_f32(const ApplyHArgs<float>& a, void* ws, size_t ws_bytes, hipStream_t s) {
  const int bm[1] = {256}, bn[1] = {WIDE_BN}, bk[1] = {WIDE_BK}, occ[1] = {2};
  const double eff[1] = {1.0};
  const Plan p = make_plan<1>(2 * a.m, 2 * (int64_t)a.k, bm, bn, bk, eff, occ, F32Tiles::split_penalty,
                              sizeof(float), ws_bytes, 1);
  return launch_cfg<TF32, 256, WIDE_BN, WIDE_BK, 3, 4, 1, 1>(a, p, ws, s);
}

// When 2k is a few columns past a multiple of 128, the width of the widest
// tiles (e.g. k = 260 or k = 73; k >= 64), the last tile column of a plain
// launch is mostly padding.  The product is then split by columns (H X is
// column-wise, and so is the fused epilogue): the first k - r columns,
// 2(k - r) a multiple of 128, on the widest tiles the plan picks, and the
// last r <= 20 on the narrow tile with their own K split, both in one
// launch (hx_pair_kernel, remainder workgroups first).  Y is packed for all
// k columns before.  (A main part whose 2(k - r) is not a multiple of 128
// would keep a padded tile column and pay the remainder on top.)
template <typename R>
Err launch_split(const ApplyHArgs<R>& a, void* ws, size_t ws_bytes, hipStream_t s) {
  using Ops = PrecOps<R>;
  constexpr int gran = 64;
  const int krem = a.k % gran;
  constexpr int rmax = 20;
  if constexpr (sizeof(R) == 4) {
    if (a.k > gran && a.k <= gran + WIDE_REM && !a.kreal && !a.tda)
      return launch_wide_f32(a, ws, ws ? ws_bytes : 0, s);
  }
  if (!ws || krem == 0 || krem > rmax || a.k < gran || a.kreal || a.tda)
    return Ops::one(a, plan_for<typename Ops::Tiles>(a, ws ? ws_bytes : 0, false), ws, s);
  ApplyHArgs<R> am = a, ar = a;
  am.k = a.k - krem;
  ar.k = krem;
  const int64_t c0 = am.k;
  ar.X = a.X + c0 * a.ldx;
  ar.yr = a.yr + 4 * c0;  // real columns 2 c0 .. of every row pair
  ar.Y = a.Y + c0 * a.ldy;
  if (a.P) ar.P = a.P + c0 * a.ldp;
  if (a.Q) ar.Q = a.Q + c0 * a.ldq;
  if (a.S) ar.S = a.S + c0 * a.lds;
  if (a.dcol) ar.dcol = a.dcol + c0;
  // the remainder's split-K partials (up to MAX_SPLITS) at the top of ws
  size_t rem_bytes = (size_t)MAX_SPLITS * 2 * a.m * 2 * krem * sizeof(R);
  rem_bytes = std::min(ceil_div((int64_t)rem_bytes, (int64_t)256) * 256, (int64_t)(ws_bytes / 4));
  const size_t main_bytes = (ws_bytes - rem_bytes) / 256 * 256;
  const Plan pm = plan_for<typename Ops::Tiles>(am, main_bytes, false);
  const Plan pr = plan_for<typename Ops::Tiles>(ar, rem_bytes, true);
  return Ops::pair(am, pm, ws, ar, pr, static_cast<char*>(ws) + main_bytes, s);
}

// Columns in chunks of at most kcap (the capacity of the packed buffer).
template <typename R>
Err launch_any(const ApplyHArgs<R>& a0, void* ws, size_t ws_bytes, hipStream_t s) {
  if (a0.k <= 0 || a0.m <= 0) return ok();
  if (a0.kcap <= 0 || !a0.yr || !a0.D || a0.ldyr < 4 * (int64_t)a0.kcap + 4 || a0.ldyr % 8 != 0 ||
      a0.yrows < (a0.m + 31) / 32 * 32 || a0.ldd < a0.m || a0.ldd % 8 != 0)
    return fail(CHASE_PH_ERR_ARG, "apply_h: packed buffer or D missing or misaligned");
  for (int c0 = 0; c0 < a0.k; c0 += a0.kcap) {
    ApplyHArgs<R> a = a0;
    a.k = std::min(a0.kcap, a0.k - c0);
    a.X = a0.X + (int64_t)c0 * a0.ldx;
    a.Y = a0.Y + (int64_t)c0 * a0.ldy;
    if (a0.P) a.P = a0.P + (int64_t)c0 * a0.ldp;
    if (a0.Q) a.Q = a0.Q + (int64_t)c0 * a0.ldq;
    if (a0.S) a.S = a0.S + (int64_t)c0 * a0.lds;
    if (a0.dcol) a.dcol = a0.dcol + c0;
    CHASE_TRY(pack<R>(a, s));
    CHASE_TRY(launch_split<R>(a, ws, ws_bytes, s));
  }
  return ok();
}

// D = [A + B, i (A - B)] column-interleaved (m x 2m, ldd); A is conj of the
// buffer when a_conj.  Rows m .. ldd of every column are zero.
template <typename C>
__global__ void make_d_kernel(const c128* A, const c128* B, int64_t ld, int a_conj, C* D, int64_t ldd, int64_t m) {
  const int64_t total = ldd * m;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = t / ldd, i = t % ldd;
    C* d0 = D + (2 * p) * ldd + i;
    C* d1 = d0 + ldd;
    if (i >= m) {
      d0->re = d0->im = d1->re = d1->im = 0;
      continue;
    }
    const c128 x = A[p * ld + i];
    const c128 b = B ? B[p * ld + i] : c128{0.0, 0.0};
    const double ar = x.re, ai = a_conj ? -x.im : x.im;
    d0->re = ar + b.re;        // A + B
    d0->im = ai + b.im;
    d1->re = -(ai - b.im);     // i (A - B)
    d1->im = ar - b.re;
  }
}

}  // namespace

Err launch_apply_h_f32(const ApplyHArgs<float>& a, void* ws, size_t ws_bytes, hipStream_t s) {
  if (a.kreal) return fail(CHASE_PH_ERR_ARG, "apply_h: K-real columns are a c128 mode");
  return launch_any<float>(a, ws, ws_bytes, s);
}

Err launch_apply_h_f64(const ApplyHArgs<double>& a, void* ws, size_t ws_bytes, hipStream_t s) {
  return launch_any<double>(a, ws, ws_bytes, s);
}

template <typename C>
Err make_d(const c128* A, const c128* B, int64_t ld, int a_conj, C* D, int64_t ldd, int64_t m, hipStream_t s) {
  const int64_t total = ldd * m;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(total, 256), 16384));
  hipLaunchKernelGGL((make_d_kernel<C>), dim3(blocks), dim3(256), 0, s, A, B, ld, a_conj, D, ldd, m);
  CHASE_LAUNCH_CHECK();
  return ok();
}

template Err make_d<c64>(const c128*, const c128*, int64_t, int, c64*, int64_t, int64_t, hipStream_t);
template Err make_d<c128>(const c128*, const c128*, int64_t, int, c128*, int64_t, int64_t, hipStream_t);

}  // namespace chase
