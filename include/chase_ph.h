/*
 * chase_ph.h -- C ABI of the MI355X (gfx950) pseudo-hermitian ChASE hot path.
 *
 * Method: Di Napoli, Richefort, Wu, "Chebyshev Accelerated Subspace
 * Eigensolver for Pseudo-hermitian Hamiltonians" (arXiv:2601.10557).
 * Problem (Section 1, eqs. 1.1-1.3): the nev smallest positive eigenpairs of
 *     H = [[A, B], [-conj(B), -conj(A)]],  A = A^H,  B = B^T  (m x m each),
 * n = 2m, in the definite case SH = [[A, B], [conj(B), conj(A)]] > 0 with
 * S = diag(I, -I).  K = [[0, I], [I, 0]] (Thm 3.1).
 *
 * Conventions shared by every entry point
 * --------------------------------------
 * - Matrices are column-major with an explicit leading dimension (in
 *   elements).  Complex numbers are interleaved (re, im) pairs: "c128" is
 *   two doubles (torch.complex128), "c64" two floats (torch.complex64).
 * - Pointers named d* are device pointers; h* are host pointers.
 * - Device buffers passed in are borrowed: the caller owns them.  A and B
 *   given to chase_ph_create must stay valid and unmodified until
 *   chase_ph_destroy.  All workspace is owned by the handle (the one
 *   handle-free entry point, chase_ph_eigval_backward_noalloc, uses a fixed
 *   device array of the library instead).
 * - Every call is ordered on the HIP stream given at create time.  Calls
 *   that return host values synchronise that stream before returning.
 * - Errors are reported by status code only; the library never aborts.
 *   Argument errors are detected before any GPU work is queued.  After a
 *   CHASE_PH_ERR_HIP the handle is unusable and must be destroyed.
 *   chase_ph_last_error() returns a handle-owned message for the last error.
 * - One handle per host thread; calls on one handle must not overlap.
 * - No entry point falls back to host computation: every step on vectors
 *   of length n and on k x k matrices runs in the library's own GPU
 *   kernels.  The host keeps O(k) scalars (Ritz values, residuals,
 *   degrees, locking) and diagonalises the Lanczos tridiagonals (at most
 *   lanczos_steps x lanczos_steps) for the spectral estimates of
 *   Section 4.1.
 * - The back-up quotient is the alternative dual basis named at the end of
 *   Section 4.4; Section 5.3 ("Non-hermitian Rayleigh-Quotient as
 *   back-up", carried as removed text in the paper's source) gives its
 *   quotient and the rule of keeping the real parts.
 */
#ifndef CHASE_PH_H
#define CHASE_PH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chase_ph_s* chase_ph_t;

typedef enum {
  CHASE_PH_OK = 0,
  CHASE_PH_ERR_ARG = 1,           /* bad pointer, size, leading dimension or parameter      */
  CHASE_PH_ERR_ALLOC = 2,         /* device or host allocation failed                       */
  CHASE_PH_ERR_HIP = 3,           /* a HIP runtime call or kernel launch failed (sticky)    */
  CHASE_PH_ERR_NOT_DEFINITE = 4,  /* Cholesky of Q^H S H Q failed: SH not HPD on range(Q)   */
  CHASE_PH_ERR_QR = 5,            /* CholeskyQR2 and its shifted fallback both failed       */
  CHASE_PH_ERR_SINGULAR_QSQ = 6,  /* Q^H S Q numerically singular (Section 4.4)             */
  CHASE_PH_ERR_NO_CONVERGENCE = 7, /* max_iter reached; info->locked pairs are valid        */
  CHASE_PH_ERR_EIG = 8            /* the Jacobi eigensolver of the Rayleigh quotient (Alg. 2, */
                                  /* eq. 2.2) left an off-diagonal entry above 1e-16 ||G||_F */
                                  /* after rr_max_sweeps sweeps                               */
} chase_ph_status;

typedef enum {
  CHASE_PH_FP64 = 0,  /* filter in complex FP64 (c128)                                       */
  CHASE_PH_MIXED = 1, /* filter products in complex FP32 (c64): the first filter plainly,     */
                      /* later ones in the residual-correction form of chase_ph_filter_refined*/
                      /* (FP64 residuals and recombination); QR, Rayleigh-Ritz, residuals   */
                      /* and locking always in FP64                                          */
  CHASE_PH_FP32 = 2,  /* stage calls only: run one apply_h / filter in c64                   */
  CHASE_PH_FP64_KREAL = 3 /* chase_ph_apply_h only: c128 with every column of X K-real        */
} chase_ph_precision;

/* Solver parameters (Alg. 3 inputs plus the paper's defaults).  Fill with
 * chase_ph_default_params() and override. */
typedef struct {
  int64_t m;            /* block size; n = 2m                                               */
  int32_t nev;          /* wanted smallest positive eigenpairs                              */
  int32_t nex;          /* extra search vectors; nevex = nev + nex <= m                    */
  int32_t deg;          /* Chebyshev degree in H^2 (applications of H^2 per filter)         */
  int32_t deg_min;      /* per-vector degree range (Section 6.1: 8..20)                     */
  int32_t deg_max;
  int32_t opt_deg;      /* 1: per-vector degrees from the convergence-factor bound          */
  int32_t max_iter;     /* outer iterations (Section 6.1: 25)                               */
  double tol;           /* absolute residual ||H v - lambda v||_2 on unit v                 */
  int32_t precision;    /* chase_ph_precision: FP64 or MIXED                                */
  double switch_tol;    /* MIXED: > 0 keeps pairs with residual above it on the plain c64    */
                        /* filter; <= 0 (default): residual-correction form for every pair  */
  double gamma;         /* lower-half scaling of the initial block (Section 4.6: 1e-3)      */
  int32_t lanczos_steps;/* per run, even (Section 4.1; 26)                                  */
  int32_t lanczos_vecs; /* independent Lanczos runs (4)                                     */
  int32_t a_conj;       /* 1: the buffer dA holds conj(A) column-major (= A row-major)      */
  int32_t rr_backup;    /* 0: the non-hermitian back-up quotient of Section 5.3 only when   */
                        /* Alg. 2 resolves fewer than k/2 positive Ritz values (Q^H S Q     */
                        /* singular); 1: the back-up quotient in every iteration            */
  int32_t definite;     /* 1 (default): S H positive definite, Alg. 2 and S H-inner-product */
                        /* Lanczos.  0: S H may be indefinite (Section 5.3, last paragraph):*/
                        /* Lanczos on S H in the Euclidean inner product, the quotient of   */
                        /* eq. 4.7 by a general eigensolver (chase_ph_oblique_rr_general),  */
                        /* the back-up quotient when Q^H S Q is singular; wanted are the    */
                        /* nev smallest positive real eigenvalues                           */
  int32_t tda;          /* 1: Hermitian ChASE on A alone (Alg. 1; the B = 0 block of         */
                        /* Section 1.1): the nev smallest eigenvalues of A, m-row vectors.  */
                        /* dB is not read (may be NULL); FP64 only, fixed degree deg (in A, */
                        /* not H^2); the stage calls other than chase_ph_apply_h (which     */
                        /* then computes A X) return CHASE_PH_ERR_ARG on such a handle      */
  int32_t nex_auto;     /* tda only.  1: choose the number of extra vectors at solve time   */
                        /* (the automatic nex named as future work in Section 6.1) among    */
                        /* ceil(j nex / 8), j = 1..8, minimising the estimated iterations   */
                        /* x (nev + candidate) from the Lanczos density of A: each          */
                        /* candidate's nev-th and (nev + candidate)-th eigenvalues are       */
                        /* density quantiles, the per-iteration factor of the nev-th pair   */
                        /* is 1 / |T_deg(t)| on the damped interval, and the iterations are */
                        /* those that take a residual of mu_m - mu_1 down to tol (p->nex is */
                        /* the largest candidate and sizes the workspace)                   */
  int32_t rr_max_sweeps; /* sweep limit of the Jacobi eigensolver of the Rayleigh quotient  */
                        /* (default 40); CHASE_PH_ERR_EIG when it is reached unconverged    */
} chase_ph_params;

typedef struct {
  int32_t iterations;      /* outer iterations run                                          */
  int32_t locked;          /* converged pairs returned                                      */
  int32_t shifted_qr_used; /* times the shifted CholeskyQR fallback was taken               */
  int32_t switch_iter;     /* MIXED: first iteration with an FP64 filter (-1: never)        */
  double mu1, mu_nevex0, mu_n; /* Lanczos spectral estimates                                */
  double t_lanczos, t_filter, t_qr, t_rr, t_resid, t_total; /* seconds (stream-timed)       */
  double filter_flops;     /* 8 n^2 real flops per active column per degree: each product  */
                           /* with H is one real GEMM of 4 n^2 per column (a complex GEMM   */
                           /* [A B][X, K conj(X)] would take 8 n^2)                        */
  double rr_flops;         /* 2 n^2 k (H Q on K-real columns) + 12 n k^2 + CholeskyQR2 16 n k^2 */
  double filter_flops_fp32;/* part of filter_flops done in c64                              */
  double* resid_history;   /* optional host array (caller-owned) of max_iter * nevex        */
  int32_t resid_history_len; /* capacity of resid_history in doubles (0 if NULL)           */
  int32_t householder_qr_used; /* times the Householder QR fallback was taken              */
  int32_t backup_rr_used;  /* iterations whose Rayleigh-Ritz used the back-up quotient      */
  int32_t general_rr_used; /* iterations whose Rayleigh-Ritz used the general quotient      */
  int32_t nex_used;        /* extra search vectors of the solve (p->nex unless nex_auto)     */
  int32_t rr_sweeps_max;   /* most Jacobi sweeps one Rayleigh-Ritz step took                 */
  int32_t qr_one_pass;     /* iterations whose Cholesky QR stopped after one pass (Q^H Q     */
                           /* within 1e-13 of I after it: a well-conditioned block)          */
} chase_ph_info;

/* Defaults: deg 20, deg range 8..20, max_iter 25, gamma 1e-3, 26 Lanczos
 * steps x 4 runs, FP64, tol 1e-10, opt_deg 0, definite 1, rr_max_sweeps 40. */
void chase_ph_default_params(chase_ph_params* p);

/* Create a solver handle for H built from the m x m blocks at dA, dB
 * (device, c128, column-major, leading dimension ld >= m).  dA must be
 * Hermitian, dB complex symmetric (dB may be NULL when p->tda = 1).
 * hip_stream may be NULL (default stream).  Allocates all workspace for
 * nevex = nev + nex columns and the real operand D = [A + B, i (A - B)]
 * of the H X products in c128 and, when precision is MIXED, in c64.
 * Section 1, eq. 1.1. */
chase_ph_status chase_ph_create(const chase_ph_params* p, const void* dA, const void* dB,
                                int64_t ld, void* hip_stream, chase_ph_t* out);

/* Free all handle-owned memory.  Accepts NULL. */
chase_ph_status chase_ph_destroy(chase_ph_t h);

/* Message of the last error on handle h; with h = NULL, that of the last
 * failed handle-free call (chase_ph_eigval_backward_noalloc) on this host
 * thread. */
const char* chase_ph_last_error(chase_ph_t h);

/* Y = H X for an n x k block (Section 1, eq. 1.1; the product behind every
 * GEMM of Alg. 2 and eq. 4.1).  H is real-linear on K-real vectors
 * (Thm 3.1): H [a; conj(a)] = [t; -conj(t)] with t = (A + B) Re(a) +
 * i (A - B) Im(a).  Each column is split into its two K-real parts and the
 * product runs as one real GEMM of 4 n^2 k flops against D = [A + B,
 * i (A - B)] (column-interleaved, built by the library from A and B), half
 * the flops of a complex GEMM.  prec: CHASE_PH_FP64 -> dX, dY are c128 (D
 * in c128); CHASE_PH_FP32 -> dX, dY are c64 (D in c64, built on first
 * use); CHASE_PH_FP64_KREAL -> as CHASE_PH_FP64 for a block whose columns
 * are K-real (x = [a; conj(a)], K conj(x) = x): 2 n^2 k flops (the bottom
 * half of dX is not read; the solver's Rayleigh-Ritz basis is of this
 * kind).  dX and dY must not overlap.  0 <= k; ldx, ldy >= n.
 * On a TDA handle (p->tda = 1): Y = A X for an m x k block (ldx, ldy >= m;
 * FP64 or FP32), the same kernel on D = [A, i A]: 8 m^2 k flops. */
chase_ph_status chase_ph_apply_h(chase_ph_t h, int32_t k, const void* dX, int64_t ldx,
                                 void* dY, int64_t ldy, int32_t prec);

/* In place W <- p(H^2) W for an n x k block through the scaled three-term
 * Chebyshev recurrence of eq. 4.1 (Section 4.2, Thm 4.2: only the positive
 * half is filtered).  degs: host array of k degrees, non-decreasing, each
 * >= 1 (NULL: every column gets p->deg).  The filter damps
 * [mu_nevex^2, mu_n^2] and is normalised at mu1^2 (0 < mu1 < mu_nevex < mu_n).
 * prec as in chase_ph_apply_h: FP64 -> dW c128, FP32 -> dW c64. */
chase_ph_status chase_ph_filter(chase_ph_t h, int32_t k, void* dW, int64_t ldw,
                                const int32_t* degs, double mu1, double mu_nevex,
                                double mu_n, int32_t prec);

/* In place W <- p(H^2) W for k unit Ritz vectors (c128, dW) with Ritz
 * values hLam (host, k) and residual vectors dR = H W - W diag(hLam)
 * (c128, n x k), evaluated with c64 matrix products and FP64 refinement:
 *   p(H^2) w = p(lambda^2) w + q(H^2) (H + lambda) r,
 * q the divided difference of the scaled Chebyshev polynomial p of eq. 4.1
 * (Section 4.2), built by the same three-term recurrence with a source
 * term.  The result equals the filter of chase_ph_filter in exact
 * arithmetic; the c64 rounding error is relative to the correction term,
 * which shrinks with the residual.  degs, mu1, mu_nevex, mu_n as in
 * chase_ph_filter; dR is not modified. */
chase_ph_status chase_ph_filter_refined(chase_ph_t h, int32_t k, void* dW, int64_t ldw, const void* dR,
                                        int64_t ldr, const double* hLam, const int32_t* degs, double mu1,
                                        double mu_nevex, double mu_n);

/* In place orthonormalisation of an n x k c128 block dX (Section 2: Cholesky
 * QR, with Householder QR for blocks Cholesky QR cannot handle):
 * CholeskyQR2; the shifted CholeskyQR3 when its first factorisation breaks
 * down; a blocked Householder QR when a factorisation of either breaks
 * down later (a numerically rank-deficient block).  On return dX holds Q
 * with Q^H Q = I whose first j columns span the first j columns of X for
 * every j and, if dR is non-NULL, dR (k x k c128, ldr >= k) holds the
 * upper-triangular R with X = Q R and a real diagonal, positive for the
 * Cholesky variants and non-negative for the Householder one (zero where a
 * column depends on the previous ones).  *used_shift (host, may be NULL) is
 * set to 0 (CholeskyQR2), 1 (shifted CholeskyQR3) or 2 (Householder).
 * k <= 2 * nevex. */
chase_ph_status chase_ph_qr(chase_ph_t h, int32_t k, void* dX, int64_t ldx, void* dR,
                            int64_t ldr, int32_t* used_shift);

/* Oblique Rayleigh-Ritz of Alg. 2 on an orthonormal n x k c128 block dQ
 * (k even, k <= 2 * nevex; Section 4.4, Thm 4.4, Thm 4.5):
 *   T = H Q; M = Q^H S T; L = chol(M); N = I - 2 Q2^H Q2;
 *   G = L^{-1} N L^{-H}; G Y = Y Theta; lambda = 1/theta; Z = L^{-H} Y.
 * Outputs the k/2 positive Ritz values ascending (hRitz, host), the
 * matching k x k/2 coefficient block dZpos (c128, ldz >= k; Ritz vectors
 * are Q Z, not normalised), and dT = H Q (n x k c128, ldt >= n) for reuse
 * by chase_ph_residuals.  CHASE_PH_ERR_NOT_DEFINITE if chol(M) fails,
 * CHASE_PH_ERR_SINGULAR_QSQ if fewer than k/2 positive or k/2 negative
 * eigenvalues of G are resolved away from zero. */
chase_ph_status chase_ph_oblique_rr(chase_ph_t h, int32_t k, const void* dQ, int64_t ldq,
                                    double* hRitz, void* dZpos, int64_t ldz, void* dT,
                                    int64_t ldt);

/* Rayleigh-Ritz with the non-hermitian back-up quotient of Section 5.3, for
 * a block where Alg. 2 fails because Q^H S Q is singular; same arguments
 * and outputs as chase_ph_oblique_rr.  With N = Q^H S Q and D = diag(N)
 * (entries below 1e-8 in modulus replaced by 1, which keeps the dual basis
 * Q_L = [S Q - Q (N - D)] D^{-1} bi-orthogonal to Q):
 *   T = H Q;  G = D^{-1} [Q^H S T - (N - D) Q^H T];  G Y = Y W (general
 *   eigenproblem: Hessenberg reduction, shifted QR, back-substitution).
 * The Ritz values are complex and their real parts are kept: hRitz gets the
 * k/2 smallest positive real parts ascending, followed, if fewer than k/2
 * are positive (the back-up dual basis need not keep the +/- symmetry of
 * Thm 4.5), by the largest non-positive ones descending; dZpos the
 * matching columns of Y.  The solver never locks a non-positive value.  CHASE_PH_ERR_SINGULAR_QSQ if the QR iteration does not
 * converge (30 iterations per eigenvalue, 10 k in total). */
chase_ph_status chase_ph_oblique_rr_backup(chase_ph_t h, int32_t k, const void* dQ, int64_t ldq,
                                           double* hRitz, void* dZpos, int64_t ldz, void* dT,
                                           int64_t ldt);

/* Rayleigh-Ritz for any S H, definite or not (Section 5.3, last paragraph:
 * a non-hermitian quotient does not need S H to be definite), with the dual
 * basis Q_L = S Q (Q^H S Q)^{-1} of eq. 4.6; same arguments and outputs as
 * chase_ph_oblique_rr.  The quotient of eq. 4.7,
 *   T = H Q;  P = Q^H S T;  Q^H S Q = Q_N R (Householder QR);
 *   G = R^{-1} Q_N^H P;  G Y = Y W (general eigenproblem),
 * never factors Q^H S H Q.  Real parts of the Ritz values are kept and the
 * positive half is selected as in chase_ph_oblique_rr_backup.
 * CHASE_PH_ERR_SINGULAR_QSQ if Q^H S Q is numerically singular
 * (min |R_ii| <= 1e3 u max |R_ii|) or the QR iteration does not converge. */
chase_ph_status chase_ph_oblique_rr_general(chase_ph_t h, int32_t k, const void* dQ, int64_t ldq,
                                            double* hRitz, void* dZpos, int64_t ldz, void* dT,
                                            int64_t ldt);

/* Half back-transform and residuals (Section 4.5): for the first kk
 * columns of dZpos, V = Q Z (normalised to unit 2-norm, written to dV,
 * n x kk c128) and resid_j = ||H v_j - lambda_j v_j||_2 computed from the
 * T = H Q of chase_ph_oblique_rr as ||T z_j / nu_j - lambda_j v_j||_2.
 * hRitz: host, kk values; hResid: host out, kk values. */
chase_ph_status chase_ph_residuals(chase_ph_t h, int32_t k, int32_t kk, const void* dQ,
                                   int64_t ldq, const void* dT, int64_t ldt,
                                   const void* dZpos, int64_t ldz, const double* hRitz,
                                   void* dV, int64_t ldv, double* hResid);

/* Run Alg. 3 to completion: Lanczos estimates, then filter / QR /
 * Rayleigh-Ritz / residuals / locking until nev pairs are locked or
 * max_iter.  The random initial block (n x nevex) and Lanczos starts
 * (n x lanczos_vecs) are inputs: dW0 and dLz are device c128 buffers with
 * unscaled complex Gaussian entries (the library applies the gamma
 * scaling of Section 4.6); they are not modified.  Outputs: hEvals (host,
 * nev, ascending), dV (device c128 n x nev, ldv >= n, unit columns),
 * hResid (host, nev, may be NULL), info (may be NULL).  Returns
 * CHASE_PH_ERR_NO_CONVERGENCE with info->locked valid pairs if max_iter is
 * reached first.
 * On a TDA handle (p->tda = 1) the same call runs Alg. 1 on the Hermitian A:
 * Lanczos on A (unscaled starts, dLz m x lanczos_vecs, ldlz >= m), then
 * filter W <- p_deg(A) W (the scaled Chebyshev recurrence of eq. 2.1 on
 * [mu_nevex, mu_m], normalised at mu_1), Cholesky QR of [Y, W] (Y the
 * locked vectors), Rayleigh-Ritz G = Q^H A Q (eq. 2.2; block Jacobi),
 * residuals ||A w - omega w||_2 of unit Ritz vectors and locking of the
 * leading converged pairs.  dW0 (m x (nev + nex), ldw0 >= m; the first
 * nev + info->nex_used columns are used), dV (m x nev, ldv >= m); hEvals
 * are the nev smallest eigenvalues of A, ascending. */
chase_ph_status chase_ph_solve(chase_ph_t h, const void* dW0, int64_t ldw0, const void* dLz,
                               int64_t ldlz, double* hEvals, void* dV, int64_t ldv,
                               double* hResid, chase_ph_info* info);

/* Eigenvalue adjoint for L = sum_i g_i lambda_i over converged pairs (not
 * in the paper; derived from Thm 3.2, u = S v, and eq. 3.5):
 *   G_A = sum_i gt_i (x_i x_i^H + conj(y_i) conj(y_i)^H),
 *   G_B = sum_i gt_i (x_i y_i^H + conj(y_i) x_i^T),
 *   gt_i = g_i / (x_i^H x_i - y_i^H y_i),   v_i = [x_i; y_i] = column i of dV,
 * in the convention grad = dL/dRe + i dL/dIm, projected on Hermitian dA and
 * symmetric dB.  dV: n x nev c128; hG: host nev; dGA, dGB: m x m c128
 * outputs with leading dimension ldg >= m (overwritten). */
chase_ph_status chase_ph_eigval_backward(chase_ph_t h, int32_t nev, const void* dV,
                                         int64_t ldv, const double* hG, void* dGA,
                                         void* dGB, int64_t ldg);

/* Largest nev accepted by chase_ph_eigval_backward_noalloc. */
#define CHASE_PH_NOALLOC_MAX_NEV 16384

/* The eigenvalue adjoint of chase_ph_eigval_backward without a handle and
 * without any device allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same contraction, conventions and outputs, for H of
 * block size m (dV: 2m x nev c128, ldv >= 2m; dGA, dGB: m x m c128,
 * ldg >= m, overwritten; hG: host, nev).  Runs on the current device,
 * ordered on hip_stream (NULL: the null stream; it must belong to the
 * current device), and synchronises that stream before returning.
 * The nev weights and the scaled weights gt live in a fixed array of
 * 2 * CHASE_PH_NOALLOC_MAX_NEV doubles (256 KiB) that the library holds on
 * every device it runs on until the process ends; nothing needs clearing
 * between calls.  Calls that overlap on one device race on that array.
 * Returns CHASE_PH_ERR_ARG for bad arguments or nev > CHASE_PH_NOALLOC_MAX_NEV,
 * CHASE_PH_ERR_HIP if a HIP call or launch fails; chase_ph_last_error(NULL)
 * then gives the message of the last failed call on this host thread. */
chase_ph_status chase_ph_eigval_backward_noalloc(int64_t m, int32_t nev, const void* dV,
                                                 int64_t ldv, const double* hG, void* dGA,
                                                 void* dGB, int64_t ldg, void* hip_stream);

/* Timing of the most recent chase_ph_apply_h / chase_ph_filter launch
 * sequence in milliseconds (HIP events on the handle's stream) and the
 * number of apply_h kernel launches it contained. */
chase_ph_status chase_ph_last_timing(chase_ph_t h, double* ms, int32_t* launches);

/* Matrix-core throughput probe (no handle; runs on the current device and
 * its null stream, allocates and frees a small output buffer): every wave
 * of 8 four-wave workgroups per CU issues 4 x iters MFMAs (iters rounded up
 * to a multiple of 8) on register
 * operands with four independent accumulators.  kind 0:
 * v_mfma_f32_32x32x2f32, kind 1: v_mfma_f64_16x16x4f64.  *tflops (host)
 * gets the best of three timed launches after a warm-up.  Returns 0, or 1
 * for bad arguments, 2 if the buffer cannot be allocated, 3 on a HIP
 * error.  A measured ceiling to set the H X kernels against, beside the
 * published peaks (157.3 and 78.6 TFLOP/s). */
int32_t chase_ph_mfma_probe(int32_t kind, int32_t iters, double* tflops);

/* Per-launch timing of the H X kernels, for roofline reporting.  With
 * enable = 1 every subsequent apply_h kernel launch on this handle (stage
 * calls, the filter, Lanczos and the Rayleigh-Ritz product inside solve) is
 * bracketed by a pair of HIP events on the handle's stream; enable = 0 stops
 * recording.  Either call resets the counters.  At most 65536 launches are
 * recorded per enable. */
chase_ph_status chase_ph_profile(chase_ph_t h, int32_t enable);

/* Sum over the recorded launches of precision prec (CHASE_PH_FP64 or
 * CHASE_PH_FP32) of: kernel time (ms, from the event pairs), algorithmic
 * flops (8 n^2 per column) and algorithmic HBM bytes (A and B read once,
 * X read once, Y written once, P and Q read once if present).
 * Synchronises the stream. */
chase_ph_status chase_ph_profile_read(chase_ph_t h, int32_t prec, double* total_ms, double* flops,
                                      double* bytes, int32_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* CHASE_PH_H */
