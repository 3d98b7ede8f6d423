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
};

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

}  // namespace chase
