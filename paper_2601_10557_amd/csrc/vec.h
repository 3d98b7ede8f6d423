// Elementwise / column-reduction kernels (vec.hip).
#pragma once
#include "common.h"

namespace chase {

// Real coordinates (in the real parts; imaginary parts 0) of the K-real
// pair vectors u, v of S y_j (j < L) and w_j (j < kw): n x (2L + 2kw),
// columns 2q, 2q + 1 for the q-th generator.
Err kreal_build(const c128* Y, int64_t ldy, int L, const c128* W, int64_t ldw, int kw, c128* X, int64_t ldx, int64_t m,
                hipStream_t s);
// Real coordinates sqrt(2) [Re a; Im a] of unit K-real columns [a; conj(a)].
Err kreal_coords(const c128* Q, int64_t ldq, int64_t m, int k, c128* D, int64_t ldd, hipStream_t s);
// x = e_r (n entries).
Err unit_column(c128* x, int64_t n, int64_t r, hipStream_t s);
// In place, columns 2j and 2j + 1: (x, y) -> (x + i y, x - i y) / sqrt(2).
Err pair_mix(c128* X, int64_t ldx, int64_t n, int npair, hipStream_t s);
// In place: orthonormal real coordinates -> orthonormal K-real vectors.
Err kreal_unpack(c128* X, int64_t ldx, int64_t m, int k, hipStream_t s);
Err convert_to_c64(const c128* src, int64_t lds, c64* dst, int64_t ldd, int64_t rows, int cols, hipStream_t s);
Err convert_to_c128(const c64* src, int64_t lds, c128* dst, int64_t ldd, int64_t rows, int cols, hipStream_t s);
Err scale_lower_half(const c128* src, int64_t lds, c128* dst, int64_t ldd, int64_t m, int cols, double g,
                     hipStream_t s);
Err residual_norms(c128* V, int64_t ldv, const c128* TZ, int64_t ldt, const double* dlam, int64_t n, int kk,
                   double* dres, c128* R, int64_t ldr, hipStream_t s);
Err scale_c64(const c64* src, int64_t lds, c64* dst, int64_t ldd, int64_t rows, int cols, float a, hipStream_t s);
// W[:, j] = pw[j] W[:, j] + ce D[:, j]  (pw device, k values)
Err combine_correction(c128* W, int64_t ldw, const c64* D, int64_t ldd, const double* dpw, double ce, int64_t n, int k,
                       hipStream_t s);
// out[j] = Re(x_j^H y_j) over `rows` rows.
Err row_dots(const c128* X, int64_t ldx, const c128* Y, int64_t ldy, int64_t rows, int k, double* out,
             hipStream_t s);
// out[j] = Re(x_j^H y_j) over the 2m rows (Euclidean).
Err plain_dots(const c128* X, int64_t ldx, const c128* Y, int64_t ldy, int64_t m, int k, double* out, hipStream_t s);
Err s_dots(const c128* X, int64_t ldx, const c128* Y, int64_t ldy, int64_t m, int k, double* out, hipStream_t s);
Err lanczos_residual(const c128* w, const c128* v, const c128* vp, c128* r, int64_t ld, int64_t n, int nv,
                     const double* alpha, const double* beta_prev, hipStream_t s);
Err lanczos_advance(c128* vp, c128* v, c128* w, const c128* r, const c128* z, int64_t ld, int64_t n, int nv,
                    const double* bsq, bool shift_prev, hipStream_t s);
// Eigenvalue adjoint (adjoint.hip): dgt[j] = dg[j] / (x_j^H x_j - y_j^H y_j),
// G_A = sum_j dgt_j (x_j x_j^H + conj(y_j) y_j^T),
// G_B = sum_j dgt_j (x_j y_j^H + conj(y_j) x_j^T), both m x m (ldg).
Err adjoint_contract(const c128* V, int64_t ldv, int64_t m, int nev, const double* dg, double* dgt, c128* GA,
                     c128* GB, int64_t ldg, hipStream_t s);
// Message of the last failed chase_ph_eigval_backward_noalloc call on this
// host thread (adjoint.hip).
const char* noalloc_last_error();
Err trace(const c128* G, int64_t ld, int k, double* dout, hipStream_t s);
// *dout = max |G_ij - delta_ij| over the lower triangle of the first k x k
// (colmax: k doubles of device scratch).
Err gram_deviation(const c128* G, int64_t ld, int k, double* colmax, double* dout, hipStream_t s);
// dout[i] = Re G[i, i], i < k.
Err diag_real(const c128* G, int64_t ld, int k, double* dout, hipStream_t s);
Err add_diag(c128* G, int64_t ld, int k, double v, hipStream_t s);
Err gather_columns(const c128* src, int64_t lds, c128* dst, int64_t ldd, int64_t n, int k, const int* dperm,
                   hipStream_t s);

}  // namespace chase
