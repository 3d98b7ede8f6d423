// General (non-hermitian) dense eigenproblem of the back-up Rayleigh
// quotient of Section 5.3 (geev.hip).
#pragma once
#include "common.h"

namespace chase {

struct GeevWs {
  c128* v = nullptr;      // kmax: Householder vector of the current column
  double* tau = nullptr;  // 1
  int* status = nullptr;  // 1: QR iteration status
};

// G (k x k, ld) -> upper-triangular Schur factor T in place, Z (k x k, ld)
// the unitary Schur vectors (G = Z T Z^H), w (k) the eigenvalues (diagonal
// of T) and Y (k x k, ld) the eigenvectors of T (unit upper triangular up
// to the back-substitution's scaling; eigenvectors of G are Z Y).  Yt is
// k x k scratch (ld k).  *qr_status (host) is 0 on success, 1 if the QR
// iteration did not converge (then Y is not computed).  Synchronises s.
Err nonsym_eig(c128* G, c128* Z, int64_t ld, int k, c128* w, c128* Yt, c128* Y, const GeevWs& ws, hipStream_t s,
               int* qr_status);

// dst (k x k, ldd) = src^H (k x k, lds); dst must not alias src.
Err conj_transpose(const c128* src, int64_t lds, c128* dst, int64_t ldd, int k, hipStream_t s);

// Diagonal threshold of the back-up dual basis (Section 5.3 allows replacing
// zero entries of diag(Q^H S Q)): |d_i| < BACKUP_DIAG_MIN is replaced by 1.
constexpr double BACKUP_DIAG_MIN = 1e-8;
// d_i = Re N_ii (replaced by 1 below BACKUP_DIAG_MIN in modulus) and
// N <- N - diag(d), for the k x k N (ld).
Err backup_diag(c128* N, int64_t ld, int k, double dmin, double* d, hipStream_t s);
// G[i][j] /= d_i for the k x k G (ld).
Err scale_rows_inv(c128* G, int64_t ld, int k, const double* d, hipStream_t s);

// The k/2 eigenvalues with the smallest positive real parts, ascending by
// real part, followed (when fewer than k/2 are positive) by the largest
// non-positive ones, descending: lam (device, k/2) gets the real parts, out
// (k x k/2, ldo) the matching columns of V (k x k, ldv); sel (device, k/2)
// the indices.
Err select_by_real_part(const c128* w, int k, const c128* V, int64_t ldv, int* sel, double* lam, c128* out,
                        int64_t ldo, hipStream_t s);

}  // namespace chase
