// Internal definitions shared by the HIP translation units of libchase_ph.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/chase_ph.h"

namespace chase {

struct c64 {
  float re, im;
};
struct c128 {
  double re, im;
};

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename R>
struct Cplx;
template <>
struct Cplx<float> {
  using T = c64;
};
template <>
struct Cplx<double> {
  using T = c128;
};

// Status with message, returned by internal helpers.
struct Err {
  chase_ph_status st = CHASE_PH_OK;
  std::string msg;
  explicit operator bool() const { return st != CHASE_PH_OK; }
};

inline Err ok() { return Err{}; }
inline Err fail(chase_ph_status st, const std::string& m) { return Err{st, m}; }

#define CHASE_HIP(call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::chase::fail(CHASE_PH_ERR_HIP,                                             \
                           std::string(#call) + ": " + hipGetErrorString(e_));           \
  } while (0)

#define CHASE_TRY(expr)          \
  do {                           \
    ::chase::Err e_ = (expr);    \
    if (e_) return e_;           \
  } while (0)

#define CHASE_LAUNCH_CHECK()                                                             \
  do {                                                                                   \
    hipError_t e_ = hipGetLastError();                                                   \
    if (e_ != hipSuccess)                                                                \
      return ::chase::fail(CHASE_PH_ERR_HIP,                                             \
                           std::string("kernel launch: ") + hipGetErrorString(e_));      \
  } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ----------------------------------------------------------------------------
// Block-structured operator H X from the blocks A, B (apply_h.hip).
//
// Computes, for the active columns of an n x k block X, H X as one real
// GEMM of M = D read as a real 2m x 2m matrix, D = [A + B, i (A - B)]
// column-interleaved (make_d), with the real coordinates of the K-real parts
// of X (packed into yr first), and writes
//   Y = alpha (H X) + beta P + gamma Q + diag(dcol) S
// (P, Q, S optional; alpha, beta, gamma real scalars, dcol a device array of
// per-column real scalars).  Y may alias P or Q (element-wise
// read-before-write in the same thread), not X.
// ----------------------------------------------------------------------------
template <typename R>
struct ApplyHArgs {
  using C = typename Cplx<R>::T;
  const C* D;       // m x 2m, column-major, ldd (multiple of 8, >= m)
  int64_t ldd;
  int64_t m;
  int k;            // active columns
  const C* X;       // n x k, ldx (already offset to the first active column)
  int64_t ldx;
  C* Y;
  int64_t ldy;
  const C* P;       // may be null
  int64_t ldp;
  const C* Q;       // may be null
  int64_t ldq;
  R alpha, beta, gamma;
  const C* S;       // may be null
  int64_t lds;
  const R* dcol;    // k per-column scalars for S (device)
  // 1: every column of X is K-real (x = [a; conj(a)]), so H x = [t; -conj(t)]
  // with t from the real coordinates of a: the product runs on k real columns
  // (c128 path, no P/Q/S)
  int kreal = 0;
  // 1: Hermitian product A X on the resonant block alone (TDA; D built with
  // B = 0, so M is the real form of A): X is m x k, Y = alpha A X + ... is
  // m x k; the product runs on k real columns
  int tda = 0;
  // packed real operand in k-pair layout: yrows (>= m rounded up to 32) row
  // pairs of ldyr (>= 4 kcap + 4, multiple of 8) reals; calls with more than
  // kcap columns run in chunks
  R* yr = nullptr;
  int64_t ldyr = 0;
  int64_t yrows = 0;
  int kcap = 0;
};

// D = [A + B, i (A - B)] column-interleaved (m x 2m, ldd; rows m .. ldd zero)
// from the c128 blocks (ld); A is conj of its buffer when a_conj; B may be
// null (B = 0: D = [A, i A], the real form of A).
template <typename C>
Err make_d(const c128* A, const c128* B, int64_t ld, int a_conj, C* D, int64_t ldd, int64_t m, hipStream_t s);

// ws: device workspace for split-K partial products (ws_bytes may be 0:
// then the K range is never split, nor the columns).
Err launch_apply_h_f32(const ApplyHArgs<float>& a, void* ws, size_t ws_bytes, hipStream_t s);
Err launch_apply_h_f64(const ApplyHArgs<double>& a, void* ws, size_t ws_bytes, hipStream_t s);

// ----------------------------------------------------------------------------
// Generic complex FP64 GEMM (zgemm.hip):
//   C = alpha * op(A) * diag_k(sgn) * op(B) + beta * C
// op(X) = X or X^H.  sgn_k = -1 for k >= kneg (folds S into a product), +1
// otherwise.  Batched with element strides; split-K through a workspace.
// ----------------------------------------------------------------------------
struct ZgemmArgs {
  int transA, transB;  // 0: N, 1: C (conjugate transpose)
  int64_t M, N, K;
  c128 alpha, beta;
  const c128* A;
  int64_t lda, strideA;
  const c128* B;
  int64_t ldb, strideB;
  c128* C;
  int64_t ldc, strideC;
  int64_t kneg;  // K index from which the sign flips (K for none)
  int batch;
  // Exact structure that lets tiles skip work (all default off):
  //  lower_only: only C's tiles on or below the diagonal are needed (a
  //              Hermitian product whose consumer reads its lower triangle;
  //              M == N); tiles strictly above are neither computed nor
  //              written;
  //  a_lower:    op(A) is lower triangular (op(A)[i][k] = 0 for k > i);
  //  b_upper:    op(B) is upper triangular (op(B)[k][j] = 0 for k > j).
  int lower_only = 0, a_lower = 0, b_upper = 0;
  // real_data: A, B and alpha have zero imaginary parts (real matrices held
  // in c128), so only the real-by-real MFMA of each step is issued (a
  // quarter of the work); C gets zero imaginary parts (beta real).
  int real_data = 0;
};
// workspace: device buffer of ws_bytes (may be 0 => no split-K)
Err zgemm(const ZgemmArgs& a, void* ws, size_t ws_bytes, hipStream_t s);

}  // namespace chase
