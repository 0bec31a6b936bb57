/*
 * frobinv.h -- C ABI of libfrobinv: inversion of a complex matrix M = A + iB
 * with real operations only ("Frobenius inversion"), on AMD MI355X (gfx950).
 *
 * Method: Z. Dai, L.-H. Lim, K. Ye, "Complex matrix inversion via real matrix
 * inversions" (arXiv 2208.01239).  The inverse is given by eq. (Finv):
 *     (A + iB)^{-1} = (A + B A^{-1} B)^{-1} - i A^{-1} B (A + B A^{-1} B)^{-1}.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrices are dense, ROW-MAJOR, FP64, in DEVICE memory of the handle's
 *    device, with a leading dimension (in elements, >= the column count).
 *    A complex matrix is passed "planar": its real part and its imaginary part
 *    are two separate real arrays sharing one leading dimension.
 *  - Ownership: the caller owns every input and output buffer.  Inputs are
 *    read-only; outputs must not alias inputs or each other.  The handle owns a
 *    grow-only device workspace and a pinned host word for status read-back,
 *    released by frob_destroy.  A workspace that a launch captured into a HIP
 *    graph references is never freed before frob_destroy: when a later call
 *    outgrows it, it is set aside and a new one is allocated, so the graph
 *    stays valid until the handle is destroyed.
 *  - Ordering: all device work is enqueued on the handle's stream (see
 *    frob_set_stream).  Each call ends with one synchronization of that stream
 *    to read the factorization status, so outputs are ready on return.
 *  - Errors are reported only through the returned status; nothing is thrown
 *    across the ABI.  On any non-OK status the outputs are unspecified.
 *  - One handle must not be used by two host threads at the same time.
 *  - Supported orders: 1 <= n <= 16384.
 */
#ifndef FROBINV_H
#define FROBINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct frob_handle *frob_handle_t;

typedef enum {
  FROB_OK = 0,
  FROB_SINGULAR = 1,        /* exact zero pivot: M is singular (Lemma 2.3: with A invertible, C = A + B A^{-1} B
                               is invertible iff M is); with the shift disabled, also a singular real part A */
  FROB_NOT_HPD = 2,         /* a Cholesky factorization met a non-positive pivot (Lemma 4.5 says A and C are
                               positive definite whenever M is Hermitian positive definite) */
  FROB_NO_CONVERGENCE = 3,  /* Newton-Schulz refinement cannot converge from the unrefined inverse: the
                               estimate of ||I - M X||_2 is >= 1, or ||I - M X||_F grew (X is returned unrefined) */
  FROB_E_ARG = -1,          /* invalid argument (null pointer, n out of range, leading dimension too small) */
  FROB_E_ALLOC = -2,        /* device or pinned-host allocation failed */
  FROB_E_HIP = -3,          /* a HIP runtime call failed */
  FROB_E_INTERNAL = -4,
  FROB_E_CAPTURE = -5       /* the call needs a larger workspace while the handle's stream is being captured
                               into a HIP graph: run it once outside the capture first */
} frob_status_t;

/* What to do about the real part A (Section 4.2, Algorithm 6, "almost sure
 * Frobenius inversion").  The shift works on (1 + i mu) M, whose real part
 * A - mu B is singular for at most n values of mu (Lemma 4.3). */
typedef enum {
  FROB_SHIFT_OFF = 0,   /* Algorithm 5 only; a singular A is reported as FROB_SINGULAR (stage 1)          */
  FROB_SHIFT_AUTO = 1,  /* Algorithm 5; if the LU of A meets an exact zero pivot, redo with Algorithm 6    */
  FROB_SHIFT_ON = 2,    /* always Algorithm 6                                                               */
  FROB_SHIFT_PHASE = 3, /* Algorithm 5 on e^{i theta} M (opts->theta), the inverse rotated back:
                           M^{-1} = e^{i theta} (e^{i theta} M)^{-1}.  Real part cos(t) A - sin(t) B, imaginary
                           part sin(t) A + cos(t) B; theta = atan(mu) is Algorithm 6, theta = -pi/2 gives the
                           formula for invertible B of Section 2.3, M^{-1} = B^{-1}A (A B^{-1} A + B)^{-1}
                           - i (A B^{-1} A + B)^{-1} (Algorithm 5 on B - iA)                              */
  FROB_SHIFT_COND = 4   /* conditioning-aware: theta = 0, -pi/2, pi/4, -pi/4 in turn until
                           u kappa_1(C_theta) <= opts->cond_tol (kappa_1(C) = ||C||_1 ||C^{-1}||_1, formed
                           exactly from C and from Re of the rotated inverse, which is C^{-1}); keeps the
                           inverse with the smallest kappa_1(C_theta); singular real parts are skipped     */
} frob_shift_t;

/* Operand precision of the matrix-core products inside the factorizations,
 * triangular solves and GEMMs (the mixed-precision variant).  Storage stays
 * FP64; FP32/BF16 operands are rounded when a tile is staged and accumulated
 * in FP32.  Pivot search, scaling, the Cholesky diagonal blocks and the small
 * triangular base cases stay FP64.  FP64 accuracy is recovered with
 * Newton-Schulz refinement (opts.refine), whose residual I - M X is formed in
 * FP64. */
typedef enum {
  FROB_PREC_F64 = 0,
  FROB_PREC_F32 = 1,
  FROB_PREC_BF16 = 2
} frob_prec_t;

typedef struct {
  int shift;            /* frob_shift_t, default FROB_SHIFT_AUTO                                            */
  double mu;            /* shift to use when shifting; mu <= 0 draws mu ~ U(0,1) from the handle's generator  */
  uint64_t seed;        /* 0: keep the handle's generator state; otherwise reseed it first                   */
  int refine;           /* maximum number of Newton-Schulz steps X <- X + X (I - M X) (0 = none)           */
  int prec;             /* frob_prec_t, default FROB_PREC_F64                                               */
  double refine_tol;    /* stop refining once ||I - M X||_F / sqrt(n) <= refine_tol (<= 0: 1e-14)            */
  int refine_flags;     /* FROB_REFINE_* bits, default 0                                                    */
  double theta;         /* rotation angle for FROB_SHIFT_PHASE (radians)                                    */
  double cond_tol;      /* target of FROB_SHIFT_COND for u kappa_1(C) (<= 0: 1e-10)                          */
  int panel;            /* panel width of the look-ahead LUs of A and C (orders >= 1024): 0 = 64 (measured
                           fastest at n = 4096); 16, 32, 48 or 64; other values FROB_E_ARG.  Ignored below
                           order 1024 and by the HPD, complex and batched paths                            */
  int reserved;
} frob_opts_t;

/* refine_flags: when refinement ends at the step limit (opts.refine steps
 * applied), do not form the residual of the returned inverse (result.resid is
 * then NaN).  Saves the three n x n x n products that only measure it. */
#define FROB_REFINE_SKIP_FINAL_RESID 1
/* refine_flags: with FP64 factorizations (opts.prec = FROB_PREC_F64), form the
 * correction X R of each step with FP32 matrix-core operands and FP32
 * accumulation; the residual R = I - M X stays FP64.  The correction is as
 * small as the error of X, so its FP32 rounding adds about
 * 6e-8 kappa(M) times that error: a step still contracts while
 * kappa(M) << 1e7.  Ignored when opts.prec is not FROB_PREC_F64. */
#define FROB_REFINE_F32_CORRECTION 2
/* refine_flags: report kappa_1(C) = ||C||_1 ||C^{-1}||_1 in result.cond1_C
 * (two column-sum passes over n x n; C^{-1} is the real part of the inverse
 * of the matrix inverted). */
#define FROB_REPORT_COND 4

typedef struct {
  int info;             /* 1-based column of the failing pivot, 0 if none                                   */
  int stage;            /* 0 none, 1 factorization of the real part, 2 factorization of C = A + B A^{-1} B   */
  double mu_used;       /* shift actually applied (0 if none)                                               */
  int shifts_tried;     /* number of shifts drawn (Algorithm 6 re-draws when A - mu B is singular)           */
  int refine_steps;     /* Newton-Schulz steps applied                                                     */
  double resid0;        /* ||I - M X||_F / sqrt(n) of the unrefined inverse (refine > 0 only)              */
  double resid;         /* the same for the returned inverse (refine > 0 only; NaN if skipped, see above)   */
  double norm2_est;     /* power-iteration estimate (a lower bound) of ||I - M X||_2 for the unrefined inverse,
                           formed only when ||I - M X||_F >= 1; 0 otherwise                                */
  double cond1_C;       /* kappa_1(C) = ||C||_1 ||C^{-1}||_1 of the inversion used (FROB_SHIFT_COND, or with
                           FROB_REPORT_COND); 0 otherwise                                                   */
  double theta;         /* rotation used by FROB_SHIFT_PHASE / FROB_SHIFT_COND (0 otherwise)                 */
} frob_result_t;

/* Fill *opts with the defaults (FROB_SHIFT_AUTO, mu drawn, no refinement). */
void frob_default_opts(frob_opts_t *opts);

/* Create a handle on HIP device `device`; its work goes to the device's null
 * stream until frob_set_stream selects another.  Returns FROB_E_ARG for a bad
 * device, FROB_E_HIP on runtime failure. */
frob_status_t frob_create(frob_handle_t *handle, int device);
frob_status_t frob_destroy(frob_handle_t handle);
/* Use `stream` (a hipStream_t; NULL is the null stream) for all later work.
 * The caller keeps ownership of the stream. */
frob_status_t frob_set_stream(frob_handle_t handle, void *stream);
/* Bytes of device workspace currently held by the handle. */
size_t frob_workspace_bytes(frob_handle_t handle);

/* General complex matrix: Algorithm 5 (Frobenius inversion with LU
 * decomposition), with Algorithm 6 per opts->shift.  Computes
 *   LU of A (partial pivoting), Y = A^{-1} B, C = A + B Y, C^{-1},
 *   Re X = C^{-1}, Im X = -Y C^{-1}
 * so that Xr + i Xi = (A + iB)^{-1}.
 *   A, B   : n x n, leading dimensions lda, ldb (inputs)
 *   Xr, Xi : n x n, leading dimension ldx (outputs)
 *   opts   : may be NULL (defaults); res: may be NULL. */
frob_status_t frob_inv_general(frob_handle_t handle, int n, const double *A, int lda, const double *B, int ldb,
                               double *Xr, double *Xi, int ldx, const frob_opts_t *opts, frob_result_t *res);

/* Hermitian positive definite M = A + iB: Algorithm 7 (Frobenius inversion
 * with Cholesky decomposition).  A must be symmetric positive definite and B
 * skew-symmetric (Lemma 4.5); only the lower triangle of A and the full B are
 * read.  Computes A = R1^T R1, R1^T X1 = B, R1 Y = X1, C = A - X1^T X1,
 * C = R2^T R2, Re X = C^{-1} (symmetric), Im X = -Y C^{-1} (skew).
 * No shift is needed (A is always invertible); opts->shift is ignored.
 * Returns FROB_NOT_HPD (stage 1 or 2) if either Cholesky factorization fails. */
frob_status_t frob_inv_hpd(frob_handle_t handle, int n, const double *A, int lda, const double *B, int ldb,
                           double *Xr, double *Xi, int ldx, const frob_opts_t *opts, frob_result_t *res);

/* A and B both symmetric positive definite (M = A + iB complex symmetric;
 * the class named at the end of Section 4.3): Algorithm 7 with step 5 read
 * as C = A + X1^T X1, since B A^{-1} B = (R1^{-T} B)^T (R1^{-T} B) for
 * symmetric B; every other step as in frob_inv_hpd (lower triangle of A read,
 * full B).  The inverse is complex symmetric.  Returns FROB_NOT_HPD (stage 1)
 * if A is not positive definite, (stage 2) if C is not. */
frob_status_t frob_inv_spd_pair(frob_handle_t handle, int n, const double *A, int lda, const double *B, int ldb,
                                double *Xr, double *Xi, int ldx, const frob_opts_t *opts, frob_result_t *res);

/* Linear system (A + iB)(x + iy) = c + id for nrhs right-hand sides
 * (Algorithm 3 with the sign of step 7 taken as y = y1 - y2, which is what
 * eq. (Finv) gives).  No inverse is formed: LU of A, Y = A^{-1} B,
 * C = A + B Y, LU of C, [x1 y1] = C^{-1} [c d], [x2 y2] = Y [y1 x1],
 * x = x1 + x2, y = y1 - y2.
 *   c, d : n x nrhs inputs (leading dimension ldc)
 *   x, y : n x nrhs outputs (leading dimension ldxy)
 * opts->shift as for frob_inv_general (the shifted system is solved for
 * (1 + i mu) M, and the solution is unchanged). */
frob_status_t frob_solve(frob_handle_t handle, int n, int nrhs, const double *A, int lda, const double *B, int ldb,
                         const double *c, const double *d, int ldc, double *x, double *y, int ldxy,
                         const frob_opts_t *opts, frob_result_t *res);

/* FP32-storage twins of frob_inv_general (Algorithm 5 with Algorithm 6),
 * frob_inv_hpd (Algorithm 7) and frob_solve (Algorithm 3): the same
 * arguments with float matrices (row-major, leading dimensions in elements,
 * device memory, caller-owned).  The operands are widened into FP64 copies in
 * the handle's workspace (4 n^2 doubles, or 2 n^2 + 4 n nrhs for the solve,
 * ahead of the FP64 call's own), the FP64 entry point runs on them with the
 * given options (opts->prec selects FP64, FP32 or BF16 matrix-core operands;
 * opts->refine refines before rounding), and the results are rounded to FP32.
 * Status and result as for the FP64 calls; on FROB_NO_CONVERGENCE the
 * unrefined inverse is returned. */
frob_status_t frob_inv_general_f32(frob_handle_t handle, int n, const float *A, int lda, const float *B, int ldb,
                                   float *Xr, float *Xi, int ldx, const frob_opts_t *opts, frob_result_t *res);
frob_status_t frob_inv_hpd_f32(frob_handle_t handle, int n, const float *A, int lda, const float *B, int ldb,
                               float *Xr, float *Xi, int ldx, const frob_opts_t *opts, frob_result_t *res);
frob_status_t frob_solve_f32(frob_handle_t handle, int n, int nrhs, const float *A, int lda, const float *B, int ldb,
                             const float *c, const float *d, int ldc, float *x, float *y, int ldxy,
                             const frob_opts_t *opts, frob_result_t *res);

/* Newton-Schulz refinement of a caller-supplied approximate inverse X of
 * M = A + iB, in place (the refinement the precision line applies after a
 * low-precision inversion; not in the paper):
 *   R = I - M X (FP64, Gauss's three-multiplication products, Proposition 2.2),
 *   X <- X + X R   (so that I - M X_new = R^2),
 * for at most opts->refine steps (>= 1), the correction's operands in
 * opts->prec (FROB_PREC_F64, F32 or BF16, or FP32 with
 * FROB_REFINE_F32_CORRECTION), until ||R||_F / sqrt(n) <= opts->refine_tol
 * or the FP64 rounding floor.  The iteration converges iff the spectral
 * radius of R_0 is below one.  A start with ||R_0||_F >= 1 is accepted when a
 * power-iteration estimate of ||R_0||_2 is below one, tentatively: if
 * ||R||_F grows before dropping below one, X is restored.  Returns
 * FROB_NO_CONVERGENCE (X unchanged) when the estimate is >= 1 or the norm grew.
 *   A, B   : n x n (leading dimensions lda, ldb), the matrix M
 *   Xr, Xi : n x n (leading dimension ldx), input and output
 *   res    : resid0, resid, norm2_est, refine_steps (may be NULL) */
frob_status_t frob_refine(frob_handle_t handle, int n, const double *A, int lda, const double *B, int ldb,
                          double *Xr, double *Xi, int ldx, const frob_opts_t *opts, frob_result_t *res);

/* Frobenius inversion over an iterated quadratic extension (Section 2.4,
 * Theorem 2.10 (ii)): F_m = R[xi_1, ..., xi_m] / <xi_k^2 + tau_k>, tau_k > 0
 * (m = 1: the complex numbers; m = 2, tau = (1, 1): bicomplex numbers).  A
 * matrix X = sum_alpha C_alpha xi^alpha is given by its 2^m real coefficient
 * planes, plane p holding C_alpha with alpha_k = bit k-1 of p.  The inverse
 * is computed recursively on the top generator with eq. (lem:inverse)
 * (Algorithm 1 over x^2 + tau_m: two inversions and three products over
 * F_{m-1}), products by Gauss's three-multiplication scheme (Theorem 2.10
 * (i)), and the F_1 inversions by frob_inv_general (xi_1 = i sqrt(tau_1)):
 * 2^m real LU inversions and 3 (3^m - 2^m) real products in total, plus the
 * products inside each complex inversion.
 *   m         : 1 .. 4;  tau : host array of m values > 0
 *   C, X      : host arrays of 2^m device pointers to n x n planes (ldc, ldx)
 *   opts      : options of every complex inversion (shift, precision, refinement)
 * Workspace: (2^(m+1) n^2 + temporaries) doubles ahead of the inversion's own.
 * A generic X is invertible through this route; FROB_SINGULAR is returned when
 * one of the F_1 inversions meets a singular matrix (stage and info from it). */
frob_status_t frob_inv_tower(frob_handle_t handle, int m, int n, const double *tau, const double *const *C, int ldc,
                             double *const *X, int ldx, const frob_opts_t *opts, frob_result_t *res);

/* Newton iterations whose every step is one Frobenius inversion (the
 * applications of Section 5 of the paper).  Stopping rule of Section 5.3:
 * stop when ||X_k - X_{k-1}||_max / ||X_k||_max <= tol, with the max norm of
 * eq. (maxnorm) (the largest |entry| over both parts), or after max_iter
 * steps. */
/* Which inversion every Newton step uses: Frobenius inversion (Algorithm 5,
 * frob_inv_general) or the complex-LU baseline (Algorithm 4, frob_cinv_lu in
 * its getri form), the two the paper compares in Section 5. */
#define FROB_NEWTON_FROBENIUS 0
#define FROB_NEWTON_COMPLEX_LU 1

typedef struct {
  double tol;           /* <= 0: 1e-3 (the paper's choice for sign and polar)                                */
  int max_iter;         /* <= 0: 100                                                                      */
  frob_opts_t inv;      /* options of every Frobenius inversion (shift, precision, refinement); zeroed =   */
                        /* defaults; unused by the complex-LU baseline                                     */
  int inverse;          /* FROB_NEWTON_FROBENIUS (0) or FROB_NEWTON_COMPLEX_LU; other values: FROB_E_ARG   */
} frob_newton_opts_t;

typedef struct {
  int iterations;       /* Newton steps taken                                                              */
  double last_change;   /* ||X_k - X_{k-1}||_max / ||X_k||_max of the last step                            */
  frob_result_t inv;    /* result of the last inversion                                                    */
} frob_newton_result_t;

/* Fill *opts with the defaults (tol 1e-3, 100 steps, frob_default_opts). */
void frob_default_newton_opts(frob_newton_opts_t *opts);

/* Matrix sign function (Section 5.3, eq. (sign)) by the Newton iteration
 * X_{k+1} = (X_k + X_k^{-1}) / 2, X_0 = X (eq. (iter)), every inverse by
 * frob_inv_general.  X must have no eigenvalue on the imaginary axis.
 *   Xr, Xi : n x n input (leading dimension ldx); Sr, Si : n x n output (lds)
 * Workspace: 4 n^2 doubles ahead of the inversion's own.  A step whose
 * inversion fails returns that status (FROB_SINGULAR: X_k singular). */
frob_status_t frob_sign(frob_handle_t handle, int n, const double *Xr, const double *Xi, int ldx, double *Sr,
                        double *Si, int lds, const frob_newton_opts_t *opts, frob_newton_result_t *res);

/* Polar decomposition X = Q P (Section 5.5): the unitary factor by
 * X_{k+1} = (X_k + X_k^{-H}) / 2, X_0 = X (eq. (iter2)), then P = Q^H X
 * (a complex matrix-core product).  X must be invertible.
 *   Qr, Qi : unitary factor (ldq);  Pr, Pi : Hermitian factor (ldp) */
frob_status_t frob_polar(frob_handle_t handle, int n, const double *Xr, const double *Xi, int ldx, double *Qr,
                         double *Qi, int ldq, double *Pr, double *Pi, int ldp, const frob_newton_opts_t *opts,
                         frob_newton_result_t *res);

/* Sylvester equation A Y + Y B = C (Section 5.4) for A (p x p) and B (q x q)
 * with sign(A) = I and sign(B) = I: the Newton iteration on
 * [[A, -C], [0, -B]] (order p + q), whose sign is [[I, -2Y], [0, -I]];
 * Y = -(1/2) times its upper right block.
 *   A : p x p (lda), B : q x q (ldb), C : p x q (ldc), Y : p x q output (ldy) */
frob_status_t frob_sylvester(frob_handle_t handle, int p, int q, const double *Ar, const double *Ai, int lda,
                             const double *Br, const double *Bi, int ldb, const double *Cr, const double *Ci, int ldc,
                             double *Yr, double *Yi, int ldy, const frob_newton_opts_t *opts,
                             frob_newton_result_t *res);

/* Lyapunov equation A Y + Y A^H = C (Section 5.4, B = A^H), sign(A) = I:
 * frob_sylvester with B = A^H formed in the block matrix.  A, C, Y : p x p. */
frob_status_t frob_lyapunov(frob_handle_t handle, int p, const double *Ar, const double *Ai, int lda,
                            const double *Cr, const double *Ci, int ldc, double *Yr, double *Yi, int ldy,
                            const frob_newton_opts_t *opts, frob_newton_result_t *res);

/* Baseline: inversion with LU decomposition in complex arithmetic
 * (Algorithm 4), planar storage, four real matrix-core products per complex
 * tile product.  form 0: as printed (U X1 = I, X2 L = X1, X^{-1} = X2 P);
 * form 1: LAPACK getri style (U^{-1} by a triangular inverse, then
 * X L = U^{-1}, then the column permutation). */
frob_status_t frob_cinv_lu(frob_handle_t handle, int n, const double *Mr, const double *Mi, int ldm, double *Xr,
                           double *Xi, int ldx, int form, frob_result_t *res);

/* Baseline: inversion with Cholesky decomposition in complex arithmetic
 * (Algorithm 8) for Hermitian positive definite M (lower triangle read).
 * form 0: as printed (R^H X1 = I, R X2 = X1); form 1: LAPACK potri style
 * (W = R^{-H} by a triangular inverse, X = W^H W). */
frob_status_t frob_cinv_chol(frob_handle_t handle, int n, const double *Mr, const double *Mi, int ldm, double *Xr,
                             double *Xi, int ldx, int form, frob_result_t *res);

/* Reverse-mode derivative of the inversion for a batch of matrices (the
 * adjoint line of growth): with X = M^{-1} and G = dL/dRe X + i dL/dIm X,
 *   dM = dL/dRe M + i dL/dIm M = -X^H G X^H
 * (from dX = -X dM X; for L = Re tr(W X), G = W^H).  Both complex products
 * use Gauss's three-real-multiplication scheme (Proposition 2.2, tau = 1):
 * three batched real matrix-core GEMMs each instead of four.
 *   storage : FROB_PREC_F64 (double arrays, FP64 GEMMs) or FROB_PREC_F32
 *             (float arrays, FP32 GEMMs with FP32 accumulation)
 *   Xr, Xi, Gr, Gi : batch x n x n inputs, contiguous (matrix b at offset b n^2)
 *   dMr, dMi       : batch x n x n outputs; must not alias the inputs
 * Returns FROB_E_ARG for bad sizes, a bad storage code, null or aliased pointers. */
frob_status_t frob_inv_adjoint(frob_handle_t handle, int batch, int n, int storage, const void *Xr, const void *Xi,
                               const void *Gr, const void *Gi, void *dMr, void *dMi);

/* Batched inversion of matrices of uneven order in one persistent launch
 * (the batching line of growth).  Each workgroup inverts whole matrices,
 * largest order first, with Algorithm 5 (kind 0, general) or Algorithm 7
 * (kind 1, Hermitian positive definite: A symmetric positive definite, B
 * skew-symmetric, lower triangle of A read).
 *   count           : number of matrices
 *   nmax            : upper bound of the orders, 1 <= nmax <= 512 (sizes the workspace)
 *   n_dev, kind_dev : device arrays of count orders (1..nmax) and kinds
 *   A_dev, B_dev    : device arrays of count device pointers to n x n inputs (contiguous, row-major)
 *   Xr_dev, Xi_dev  : device arrays of count device pointers to n x n outputs
 *   info_dev        : device array of count status words: 0, or 1000000 * stage + column (1-based first
 *                     zero pivot (kind 0) or non-positive pivot (kind 1); stage 1 = A, stage 2 = C)
 *   storage         : FROB_PREC_F64 (double matrices) or FROB_PREC_F32 (float matrices, FP32 arithmetic)
 * Asynchronous on the handle's stream: no host synchronization, no allocation
 * once the workspace has grown to fit (a first call of the same shape), and
 * no memset (queue reset by a kernel), so a call can be captured in a HIP
 * graph and replayed.  Captured before a first eager call of its shape, it
 * returns FROB_E_CAPTURE; the workspace it captured outlives later growth of
 * the handle's workspace (see Ownership).  The panel width per (kind, order class) comes from
 * frob_batched_tune (default 16). */
frob_status_t frob_inv_batched(frob_handle_t handle, int count, int nmax, const int *n_dev, const int *kind_dev,
                               const void *const *A_dev, const void *const *B_dev, void *const *Xr_dev,
                               void *const *Xi_dev, int *info_dev, int storage);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * batched inversion as frob_inv_batched, same arguments and results, with its
 * scratch (queue head, processing order, per-workgroup slots of three
 * nmax x nmax matrices) in a fixed device array of 128 MiB that the library
 * holds on every GPU it runs on until the process ends.  Nothing is
 * allocated or freed and the handle's workspace is not used.  Limits:
 * count <= 1048576, nmax <= 512; the persistent grid is two workgroups per
 * compute unit, the number of slots that fit, or count, whichever is smallest
 * (at least 20 slots fit; all 512 for nmax <= 102 in FP64 and nmax <= 145 in
 * FP32).  Returns FROB_E_ARG
 * beyond the limits.  Calls that overlap on one GPU (concurrent streams,
 * handles or threads) share the array and race: order them.  Each call
 * rewrites the queue head and order before its kernel reads them. */
frob_status_t frob_inv_batched_noalloc(frob_handle_t handle, int count, int nmax, const int *n_dev,
                                       const int *kind_dev, const void *const *A_dev, const void *const *B_dev,
                                       void *const *Xr_dev, void *const *Xi_dev, int *info_dev, int storage);

/* Autotuner for frob_inv_batched: for each kind and order class (<= 64, 128,
 * 256, 512) times the persistent kernel on synthetic diagonally dominant
 * batches with panel widths 8, 16 and 32 and keeps the fastest in the handle.
 * table_out (may be NULL) receives [kind][class] as 8 ints.  Synchronous;
 * allocates its own test matrices. */
frob_status_t frob_batched_tune(frob_handle_t handle, int storage, int table_out[8]);

/* Kernel timing with HIP events (for measurement).  When enabled, the library
 * records an event pair on the handle's stream around every launch of a
 * kernel class and accumulates, per class, the number of launches, their
 * summed duration in milliseconds, their algorithmic FP64 flop count and
 * their algorithmic HBM bytes (operands read once, outputs written once;
 * 0 where a class does not state them).
 * Class 0: the n x n x n matrix-core GEMMs of the inversion paths (B Y and
 * -Y C^{-1}).  Class 4: batched launches.  Class 5: adjoint products.
 * Class 6: the trailing-update GEMMs of the look-ahead LU factorizations on
 * the handle's second stream (real LU, orders >= 1024; flops 2 m w k per
 * launch for an m x w update of rank k).  Enabling resets the counters.  Reading is valid after a call
 * returned (its final synchronization resolves the events). */
frob_status_t frob_profile_enable(frob_handle_t handle, int on);
frob_status_t frob_profile_read(frob_handle_t handle, int kernel_class, long long *launches, double *total_ms,
                                double *flops, double *bytes);

/* Human-readable name of a status code (static string). */
const char *frob_status_string(frob_status_t status);

#ifdef __cplusplus
}
#endif
#endif /* FROBINV_H */
