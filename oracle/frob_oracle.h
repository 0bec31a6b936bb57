/*
 * frob_oracle.h -- plain, slow FP64 CPU oracle for Frobenius inversion of a
 * complex matrix M = A + iB (Dai, Lim, Ye, "Complex matrix inversion via real
 * matrix inversions", arXiv 2208.01239).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  The product path
 * (libfrobinv) shares no code, header, helper or table with it.
 *
 * Conventions (all functions):
 *   - matrices are dense, row-major, n x n (or n x p for right-hand sides),
 *     leading dimension equal to the column count, FP64;
 *   - a complex matrix is passed as two real arrays (real part, imaginary part);
 *   - every input is read-only; outputs are caller-allocated;
 *   - `flops` (may be NULL) receives the real-flop count of the run: a complex
 *     multiply counts 6, a complex add/subtract 2, a complex divide 11, a real
 *     operation 1 (the paper's accounting in the proof of Theorem 4.1);
 *   - return value: 0 on success; otherwise a positive code described per
 *     function.  A zero pivot is detected exactly (pivot == 0.0), following the
 *     LAPACK convention.
 */
#ifndef FROB_ORACLE_H
#define FROB_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

/* Return codes: info = k+1 of the first zero pivot, offset by the stage. */
#define ORC_STAGE_A 1000000   /* factorization of the real part (or of A - mu B) failed */
#define ORC_STAGE_C 2000000   /* factorization of C = A + B A^{-1} B failed (M singular, Lemma 2.3) */

/* Algorithm 4 (inversion with LU decomposition) carried out in complex
 * arithmetic: GEPP with |z| = hypot(re, im) and the lowest row index on ties,
 * then U X1 = I by backward substitution, X2 L = X1 by forward substitution,
 * X = X2 P.  Returns k+1 if the k-th pivot (0-based) is exactly zero.
 * piv (may be NULL) receives the n row interchanges. */
int orc_cinv_lu(int n, const double *Mr, const double *Mi, double *Xr, double *Xi,
                int *piv, double *flops);

/* Gauss-Jordan elimination of [M | I] with partial pivoting (complex).  An
 * independent route to the same inverse, used only to cross-check orc_cinv_lu. */
int orc_cinv_gj(int n, const double *Mr, const double *Mi, double *Xr, double *Xi);

/* Algorithm 5 (Frobenius inversion with LU decomposition), real arithmetic.
 * Output X = Xr + i Xi = (A + iB)^{-1}.  Returns ORC_STAGE_A + k + 1 if A has a
 * zero pivot, ORC_STAGE_C + k + 1 if C = A + B A^{-1} B has one. */
int orc_frob_lu(int n, const double *A, const double *B, double *Xr, double *Xi, double *flops);

/* Algorithm 6 (almost sure Frobenius inversion) with the shift mu supplied by
 * the caller: X1 = A - mu B, X2 = mu A + B, Algorithm 5 on X1 + i X2, then
 * X5 = X3 - mu X4, X6 = mu X3 + X4 where X3 + i X4 = (X1 + i X2)^{-1}. */
int orc_frob_shift(int n, const double *A, const double *B, double mu,
                   double *Xr, double *Xi, double *flops);

/* Algorithm 7 (Frobenius inversion with Cholesky decomposition) for Hermitian
 * positive definite A + iB (A symmetric positive definite, B skew-symmetric;
 * Lemma 4.5).  Reads the full A and B.  Returns ORC_STAGE_A + k + 1 if the
 * Cholesky factorization of A meets a non-positive pivot, ORC_STAGE_C + k + 1
 * if that of C = A - X1^T X1 does. */
int orc_frob_chol(int n, const double *A, const double *B, double *Xr, double *Xi, double *flops);

/* Algorithm 8 (inversion with Cholesky decomposition) in complex arithmetic:
 * M = R^H R, R^H X1 = I, R X2 = X1.  Returns k+1 on a non-positive pivot. */
int orc_cinv_chol(int n, const double *Mr, const double *Mi, double *Xr, double *Xi, double *flops);

/* Algorithm 3 (linear system with Frobenius inversion and LU), for p
 * right-hand sides: solves (A + iB)(x + iy) = c + id with c, d, x, y of shape
 * n x p.  Step 7 is taken as x = x1 + x2, y = y1 - y2 (the printed sign of y is
 * reversed; the corrected sign follows from eq. (Finv)).  Return codes as for
 * orc_frob_lu. */
int orc_frob_solve(int n, int p, const double *A, const double *B, const double *c, const double *d,
                   double *x, double *y, double *flops);

/* Adjoint of inversion: dM = -X^H G X^H (complex triple loops), i.e. the
 * gradient of L(M) = Re tr(W M^{-1}) when G = W^H, in the convention
 * dL = Re sum(conj(dM) .* dM_direction). */
void orc_adjoint(int n, const double *Xr, const double *Xi, const double *Gr, const double *Gi,
                 double *dMr, double *dMi);

/* Plain complex matrix product Z = X Y (n x k times k x m), for residuals. */
void orc_cmatmul(int n, int k, int m, const double *Xr, const double *Xi, const double *Yr,
                 const double *Yi, double *Zr, double *Zi);

/* Number of OpenMP threads the oracle uses (1 when built without OpenMP). */
/* Section 5.3, eq. (iter): the matrix sign function by the Newton iteration
 * X_{k+1} = (X_k + X_k^{-1}) / 2, X_0 = X, each inverse by Algorithm 4; stop
 * when ||X_k - X_{k-1}||_max / ||X_k||_max <= eps (eq. (maxnorm)) or at kmax
 * steps.  *iters receives the number of steps.  Returns 0 or the failing
 * inversion's info. */
int orc_sign_newton(int n, const double *Xr, const double *Xi, double eps, int kmax, double *Sr, double *Si,
                    int *iters);
/* Section 5.5, eq. (iter2): the unitary polar factor Q by X_{k+1} =
 * (X_k + X_k^{-H}) / 2 with the same stopping rule, and P = Q^H X. */
int orc_polar_newton(int n, const double *Xr, const double *Xi, double eps, int kmax, double *Qr, double *Qi,
                     double *Pr, double *Pi, int *iters);
/* Section 5.4: A Y + Y B = C (A p x p, B q x q, C p x q, sign(A) = I, sign(B) =
 * I) by the Newton iteration on [[A, -C], [0, -B]], whose sign is
 * [[I, -2Y], [0, -I]]. */
int orc_sylvester_newton(int p, int q, const double *Ar, const double *Ai, const double *Br, const double *Bi,
                         const double *Cr, const double *Ci, double eps, int kmax, double *Yr, double *Yi,
                         int *iters);
/* Algorithm 7 for the class closing Section 4.3: A and B symmetric positive
 * definite (M = A + iB complex symmetric, not Hermitian).  With B symmetric,
 * B A^{-1} B = X1^T X1, so step 5 reads X4 = A + X3; every other step as
 * printed.  Same return codes as orc_frob_chol. */
int orc_frob_chol_spd_pair(int n, const double *A, const double *B, double *Xr, double *Xi, double *flops);
/* Section 2.4: matrices over the iterated quadratic extension F_m with
 * xi_k^2 = -tau_k (every f_k = x^2 + tau_k), stored as 2^m real n x n planes
 * (plane p = coefficient of xi^alpha, alpha_k = bit k-1 of p), contiguous.
 * orc_tower_mul: the product from the definition of F_m.
 * orc_tower_inv: the inverse from X Z = 1 through the real regular
 * representation (order 2^m n) and Gaussian elimination with partial
 * pivoting; returns 0 or the 1-based zero-pivot index. */
void orc_tower_mul(int m, int n, const double *tau, const double *X, const double *Y, double *Z);
int orc_tower_inv(int m, int n, const double *tau, const double *C, double *Xinv);
/* M x = b for p right-hand sides (b, x: n x p planar) by complex GEPP and
 * `steps` steps of iterative refinement with the residual b - M x
 * accumulated in double-double (error-free transformations, no fused
 * multiply-add), each correction solved with the same factors.  A reference
 * accurate to about the unit roundoff while u kappa(M) < 1.  *last (may be
 * NULL) receives the largest relative size (max norm) of the final correction
 * over the columns.  Returns 0 or the 1-based index of an exactly zero pivot. */
int orc_csolve_refined(int n, int p, const double *Mr, const double *Mi, const double *Br, const double *Bi,
                       int steps, double *Xr, double *Xi, double *last);
int orc_num_threads(void);
int orc_set_num_threads(int t);

#ifdef __cplusplus
}
#endif
#endif
