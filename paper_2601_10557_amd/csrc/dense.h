// Small dense FP64 kernels on padded kp x kp matrices (dense.hip).
#pragma once
#include "common.h"

namespace chase {

struct DenseWs {
  c128* small = nullptr;   // 64 x 64
  c128* panel = nullptr;   // kp_max x 64
  c128* tmp = nullptr;     // kp_max x 64 (batched 64 x 64 blocks)
  c128* U = nullptr;       // kp_max x 64 (one rotation block per Jacobi pair)
  int* flag = nullptr;     // 4 ints
  int* pflag = nullptr;    // kp_max / 8 ints (Jacobi pair rotated?)
  double* dscalar = nullptr;  // 4 doubles
  void* gemm_ws = nullptr;     // split-K partials of the batched GEMMs (may be null)
  size_t gemm_ws_bytes = 0;
  void* hpin = nullptr;        // pinned host staging for small device-to-host reads (may be null)
  size_t hpin_bytes = 0;
};

// Copy bytes from device memory to host memory and wait for it: through the
// pinned staging buffer of ws when it is large enough (a direct transfer,
// no pageable staging on the runtime's side), else straight to host.
Err d2h_small(void* host, const void* dev, size_t bytes, const DenseWs& ws, hipStream_t s);

int pad64(int k);
// M = diag(inner) on the first k, pad on the rest; off-diagonals zeroed
// everywhere when zero_all, else only in the padded rows/columns.
Err fill_padded(c128* M, int kp, int k, double inner, double pad, bool zero_all, hipStream_t s);
// In place lower Cholesky of a Hermitian padded matrix; *failed on breakdown.
Err cholesky_lower(c128* M, int kp, DenseWs& ws, hipStream_t s, bool* failed);
// X = L^{-1} for lower-triangular L (both kp x kp, ld kp); X must not alias L.
Err tri_inverse_lower(const c128* L, c128* X, int kp, DenseWs& ws, hipStream_t s);
// Block Jacobi: G (Hermitian, in place) -> diag(theta), V -> eigenvectors.
Err jacobi_eigh(c128* G, c128* V, int kp, DenseWs& ws, hipStream_t s, int max_sweeps, int* sweeps_out);
// Positive eigenvalues theta of the first k: Ysel (kp x k/2, ld kp) and
// dlam[r] = 1/theta for rank r by descending theta.
Err select_positive(const c128* G, const c128* V, int k, int kp, c128* Ysel, double* dlam, DenseWs& ws,
                    hipStream_t s, int* npos, int* nneg);

// Householder QR (householder.hip): panels of HH_PANEL columns, row-parallel
// launches of HH_PARTS one-wave workgroups.
constexpr int HH_PANEL = 32;
constexpr int HH_PARTS = 512;
struct HouseholderWs {
  c128* Q = nullptr;        // n x kmax (ld n): the accumulated basis
  c128* Vb = nullptr;       // n x HH_PANEL (ld n): explicit reflectors of one panel
  c128* Tb = nullptr;       // HH_PANEL x kmax: compact WY factor of every panel
  c128* W1 = nullptr;       // HH_PANEL x kmax
  c128* W2 = nullptr;       // HH_PANEL x kmax
  c128* taus = nullptr;     // kmax
  double* part = nullptr;   // HH_PARTS
  c128* dpart = nullptr;    // HH_PARTS x HH_PANEL
  double* dsign = nullptr;  // kmax
  int kmax = 0;
  void* gemm_ws = nullptr;  // split-K partials of the GEMMs (may be null)
  size_t gemm_ws_bytes = 0;
};
// In place: X (n x k, ld ldx) -> Q with Q^H Q = I and, if R is non-null,
// R (k x k, ld ldr) upper triangular with a real non-negative diagonal and
// X = Q R (any rank; k <= n, k <= w.kmax).
Err householder_qr(c128* X, int64_t ldx, int64_t n, int k, c128* R, int64_t ldr, const HouseholderWs& w,
                   hipStream_t s);

}  // namespace chase
