/*
 * frob_oracle.c -- plain, slow FP64 CPU oracle for Frobenius inversion.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the package smoke check and
 * the benchmark's CPU-baseline leg, never by the product library.  It shares no
 * code with the GPU path.
 *
 * Reference: Z. Dai, L.-H. Lim, K. Ye, "Complex matrix inversion via real
 * matrix inversions" (arXiv 2208.01239).  Each routine below names the
 * algorithm or equation of the paper it writes out.  The routines follow the
 * paper's steps in the paper's order, with unblocked textbook loops: Gaussian
 * elimination with partial pivoting (Section 3, used by Algorithms 3-5), the
 * row-oriented Cholesky factorization, and column-by-column substitution.
 * OpenMP is used only across independent rows or right-hand sides, so every
 * output element is computed by one thread in a fixed order and results do not
 * depend on the thread count.
 *
 * Build with -O2 -ffp-contract=off (no fused multiply-add, no fast-math) so the
 * arithmetic is IEEE double with round-to-nearest-even on every operation.
 */
#include "frob_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Complex scalars written out on their real and imaginary parts.            */
/* ------------------------------------------------------------------------- */
typedef struct { double re, im; } cx;

static inline cx cx_make(double r, double i) { cx z; z.re = r; z.im = i; return z; }
static inline cx cx_add(cx a, cx b) { return cx_make(a.re + b.re, a.im + b.im); }
static inline cx cx_sub(cx a, cx b) { return cx_make(a.re - b.re, a.im - b.im); }
static inline cx cx_mul(cx a, cx b) { return cx_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static inline cx cx_conj(cx a) { return cx_make(a.re, -a.im); }
/* (a + ib) / (c + id) = ((ac + bd) + i(bc - ad)) / (c^2 + d^2) */
static inline cx cx_div(cx a, cx b) {
  double den = b.re * b.re + b.im * b.im;
  return cx_make((a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den);
}
static inline double cx_abs(cx a) { return hypot(a.re, a.im); }

#define FL_CMUL 6.0
#define FL_CADD 2.0
#define FL_CDIV 11.0

static cx *cx_alloc(int n, int m) { return (cx *)calloc((size_t)n * (size_t)m, sizeof(cx)); }
static double *re_alloc(int n, int m) { return (double *)calloc((size_t)n * (size_t)m, sizeof(double)); }

static void cx_from_planar(int n, int m, const double *re, const double *im, cx *z) {
  for (size_t t = 0; t < (size_t)n * (size_t)m; ++t) z[t] = cx_make(re[t], im ? im[t] : 0.0);
}
static void cx_to_planar(int n, int m, const cx *z, double *re, double *im) {
  for (size_t t = 0; t < (size_t)n * (size_t)m; ++t) { re[t] = z[t].re; im[t] = z[t].im; }
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of later calls (t >= 1); returns the previous count.  Timing only. */
int orc_set_num_threads(int t) {
#ifdef _OPENMP
  const int prev = omp_get_max_threads();
  if (t >= 1) omp_set_num_threads(t);
  return prev;
#else
  (void)t;
  return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Complex Gaussian elimination with partial pivoting: P M = L U, in place.   */
/* Pivot: largest |z| in the column, lowest row index on ties.  Whole rows    */
/* are interchanged, so the stored multipliers end up in the rows of P M.     */
/* Returns k+1 if the k-th pivot is exactly zero.                             */
/* ------------------------------------------------------------------------- */
static int cx_getrf(int n, cx *W, int *piv, double *fl) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = cx_abs(W[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double a = cx_abs(W[(size_t)i * n + k]);
      if (a > best) { best = a; p = i; }
    }
    piv[k] = p;
    if (best == 0.0) return k + 1;
    if (p != k)
      for (int j = 0; j < n; ++j) {
        cx t = W[(size_t)k * n + j]; W[(size_t)k * n + j] = W[(size_t)p * n + j]; W[(size_t)p * n + j] = t;
      }
    const cx d = W[(size_t)k * n + k];
#pragma omp parallel for schedule(static)
    for (int i = k + 1; i < n; ++i) {
      cx l = cx_div(W[(size_t)i * n + k], d);
      W[(size_t)i * n + k] = l;
      for (int j = k + 1; j < n; ++j)
        W[(size_t)i * n + j] = cx_sub(W[(size_t)i * n + j], cx_mul(l, W[(size_t)k * n + j]));
    }
    double r = (double)(n - k - 1);
    *fl += r * FL_CDIV + r * r * (FL_CMUL + FL_CADD);
  }
  return 0;
}

/* Real Gaussian elimination with partial pivoting (|a| = fabs), same rules. */
static int re_getrf(int n, double *W, int *piv, double *fl) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = fabs(W[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double a = fabs(W[(size_t)i * n + k]);
      if (a > best) { best = a; p = i; }
    }
    piv[k] = p;
    if (best == 0.0) return k + 1;
    if (p != k)
      for (int j = 0; j < n; ++j) {
        double t = W[(size_t)k * n + j]; W[(size_t)k * n + j] = W[(size_t)p * n + j]; W[(size_t)p * n + j] = t;
      }
    const double d = W[(size_t)k * n + k];
#pragma omp parallel for schedule(static)
    for (int i = k + 1; i < n; ++i) {
      double l = W[(size_t)i * n + k] / d;
      W[(size_t)i * n + k] = l;
      for (int j = k + 1; j < n; ++j) W[(size_t)i * n + j] -= l * W[(size_t)k * n + j];
    }
    double r = (double)(n - k - 1);
    *fl += r + 2.0 * r * r;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 4: inversion with LU decomposition (complex arithmetic).          */
/*   1. X = P^T L U;  2. U X1 = I (backward substitution against the full      */
/*   identity);  3. X2 L = X1 (substitution along each row);  4. X^{-1} = X2 P */
/* ------------------------------------------------------------------------- */
int orc_cinv_lu(int n, const double *Mr, const double *Mi, double *Xr, double *Xi, int *piv_out,
                double *flops) {
  double fl = 0.0;
  cx *W = cx_alloc(n, n), *X1 = cx_alloc(n, n), *X2 = cx_alloc(n, n);
  int *piv = (int *)calloc((size_t)n, sizeof(int));
  cx_from_planar(n, n, Mr, Mi, W);
  int info = cx_getrf(n, W, piv, &fl);
  if (piv_out) memcpy(piv_out, piv, sizeof(int) * (size_t)n);
  if (info) goto done;

  /* step 2: U X1 = I, one column of the identity at a time */
#pragma omp parallel for schedule(dynamic, 8)
  for (int c = 0; c < n; ++c) {
    for (int i = n - 1; i >= 0; --i) {
      cx s = cx_make(i == c ? 1.0 : 0.0, 0.0);
      for (int j = i + 1; j < n; ++j) s = cx_sub(s, cx_mul(W[(size_t)i * n + j], X1[(size_t)j * n + c]));
      X1[(size_t)i * n + c] = cx_div(s, W[(size_t)i * n + i]);
    }
  }
  fl += (double)n * ((double)n * (n - 1) / 2.0 * (FL_CMUL + FL_CADD) + n * FL_CDIV);

  /* step 3: X2 L = X1 with L unit lower triangular; row r of X2 solves
   * sum_{k>=j} X2[r][k] L[k][j] = X1[r][j], from the last column down. */
#pragma omp parallel for schedule(static)
  for (int r = 0; r < n; ++r) {
    for (int j = n - 1; j >= 0; --j) {
      cx s = X1[(size_t)r * n + j];
      for (int k = j + 1; k < n; ++k) s = cx_sub(s, cx_mul(X2[(size_t)r * n + k], W[(size_t)k * n + j]));
      X2[(size_t)r * n + j] = s;
    }
  }
  fl += (double)n * ((double)n * (n - 1) / 2.0 * (FL_CMUL + FL_CADD));

  /* step 4: X^{-1} = X2 P with P = S_{n-1} ... S_0 (S_k swaps k and piv[k]):
   * right-multiplying by S_{n-1} first means swapping columns from the last
   * interchange back to the first. */
  for (int k = n - 1; k >= 0; --k) {
    int p = piv[k];
    if (p == k) continue;
    for (int r = 0; r < n; ++r) {
      cx t = X2[(size_t)r * n + k]; X2[(size_t)r * n + k] = X2[(size_t)r * n + p]; X2[(size_t)r * n + p] = t;
    }
  }
  cx_to_planar(n, n, X2, Xr, Xi);
done:
  if (flops) *flops = fl;
  free(W); free(X1); free(X2); free(piv);
  return info;
}

/* ------------------------------------------------------------------------- */
/* Gauss-Jordan elimination on [M | I] with partial pivoting (cross-check).    */
/* ------------------------------------------------------------------------- */
int orc_cinv_gj(int n, const double *Mr, const double *Mi, double *Xr, double *Xi) {
  int m = 2 * n;
  cx *W = cx_alloc(n, m);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) W[(size_t)i * m + j] = cx_make(Mr[(size_t)i * n + j], Mi[(size_t)i * n + j]);
    W[(size_t)i * m + n + i] = cx_make(1.0, 0.0);
  }
  int info = 0;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = cx_abs(W[(size_t)k * m + k]);
    for (int i = k + 1; i < n; ++i) {
      double a = cx_abs(W[(size_t)i * m + k]);
      if (a > best) { best = a; p = i; }
    }
    if (best == 0.0) { info = k + 1; break; }
    if (p != k)
      for (int j = 0; j < m; ++j) {
        cx t = W[(size_t)k * m + j]; W[(size_t)k * m + j] = W[(size_t)p * m + j]; W[(size_t)p * m + j] = t;
      }
    cx d = W[(size_t)k * m + k];
    for (int j = 0; j < m; ++j) W[(size_t)k * m + j] = cx_div(W[(size_t)k * m + j], d);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      cx f = W[(size_t)i * m + k];
      for (int j = 0; j < m; ++j) W[(size_t)i * m + j] = cx_sub(W[(size_t)i * m + j], cx_mul(f, W[(size_t)k * m + j]));
    }
  }
  if (!info)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        Xr[(size_t)i * n + j] = W[(size_t)i * m + n + j].re;
        Xi[(size_t)i * n + j] = W[(size_t)i * m + n + j].im;
      }
  free(W);
  return info;
}

/* ------------------------------------------------------------------------- */
/* Real substitution helpers for the LU factors of a real matrix F = P^T L U.  */
/* ------------------------------------------------------------------------- */

/* L U Z = P R for the p columns of Z (n x p, in place: Z holds R on entry).
 * Row interchanges applied in the order they were made, then forward
 * substitution with the unit lower L and backward substitution with U. */
static void re_getrs_cols(int n, int p, const double *F, const int *piv, double *Z, double *fl) {
  for (int k = 0; k < n; ++k) {
    int q = piv[k];
    if (q == k) continue;
    for (int c = 0; c < p; ++c) {
      double t = Z[(size_t)k * p + c]; Z[(size_t)k * p + c] = Z[(size_t)q * p + c]; Z[(size_t)q * p + c] = t;
    }
  }
#pragma omp parallel for schedule(static)
  for (int c = 0; c < p; ++c) {
    for (int i = 0; i < n; ++i) {
      double s = Z[(size_t)i * p + c];
      for (int j = 0; j < i; ++j) s -= F[(size_t)i * n + j] * Z[(size_t)j * p + c];
      Z[(size_t)i * p + c] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = Z[(size_t)i * p + c];
      for (int j = i + 1; j < n; ++j) s -= F[(size_t)i * n + j] * Z[(size_t)j * p + c];
      Z[(size_t)i * p + c] = s / F[(size_t)i * n + i];
    }
  }
  *fl += (double)p * (2.0 * (double)n * n);
}

/* Row-wise right solve Z F = R with F = P^T L U: for each row r, solve
 * V U = R[r] (substitution from the first column), W L = V (from the last
 * column), then Z[r] = W P (column interchanges undone last to first). */
static void re_right_solve(int n, int rows, const double *F, const int *piv, const double *R, double *Z,
                           double *fl) {
#pragma omp parallel for schedule(static)
  for (int r = 0; r < rows; ++r) {
    double *z = Z + (size_t)r * n;
    const double *rr = R + (size_t)r * n;
    for (int j = 0; j < n; ++j) {
      double s = rr[j];
      for (int k = 0; k < j; ++k) s -= z[k] * F[(size_t)k * n + j];
      z[j] = s / F[(size_t)j * n + j];
    }
    for (int j = n - 1; j >= 0; --j) {
      double s = z[j];
      for (int k = j + 1; k < n; ++k) s -= z[k] * F[(size_t)k * n + j];
      z[j] = s;
    }
    for (int k = n - 1; k >= 0; --k) {
      int q = piv[k];
      if (q == k) continue;
      double t = z[k]; z[k] = z[q]; z[q] = t;
    }
  }
  *fl += (double)rows * (2.0 * (double)n * n);
}

/* Z = A + B Y (n x n times n x p), plain triple loop. */
static void re_add_mul(int n, int p, const double *Aadd, const double *B, const double *Y, double *Z,
                       double *fl) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < p; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += B[(size_t)i * n + k] * Y[(size_t)k * p + j];
      Z[(size_t)i * p + j] = (Aadd ? Aadd[(size_t)i * p + j] : 0.0) + s;
    }
  *fl += 2.0 * (double)n * n * p;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 5: Frobenius inversion with LU decomposition.                     */
/*   1. A = P1^T L1 U1;  2. L1 U1 X1 = P1 B;  3. X2 = A + B X1;                */
/*   4. X2 = P2^T L2 U2;  5. [X3; X4] X2 = [I; X1];  output X3 - i X4.         */
/* Step 5 is printed with the blocks side by side; the shapes only conform    */
/* when the two right-hand sides are stacked row-wise, which is the reading   */
/* used here (X3 = X2^{-1}, X4 = X1 X2^{-1}, as eq. (Finv) requires).         */
/* ------------------------------------------------------------------------- */
int orc_frob_lu(int n, const double *A, const double *B, double *Xr, double *Xi, double *flops) {
  double fl = 0.0;
  int info = 0;
  double *F1 = re_alloc(n, n), *X1 = re_alloc(n, n), *X2 = re_alloc(n, n), *I = re_alloc(n, n),
         *X3 = re_alloc(n, n), *X4 = re_alloc(n, n);
  int *piv1 = (int *)calloc((size_t)n, sizeof(int)), *piv2 = (int *)calloc((size_t)n, sizeof(int));
  memcpy(F1, A, sizeof(double) * (size_t)n * n);
  int k = re_getrf(n, F1, piv1, &fl);                         /* step 1 */
  if (k) { info = ORC_STAGE_A + k; goto done; }
  memcpy(X1, B, sizeof(double) * (size_t)n * n);
  re_getrs_cols(n, n, F1, piv1, X1, &fl);                     /* step 2: X1 = A^{-1} B */
  re_add_mul(n, n, A, B, X1, X2, &fl);                        /* step 3: X2 = A + B X1 */
  k = re_getrf(n, X2, piv2, &fl);                             /* step 4 */
  if (k) { info = ORC_STAGE_C + k; goto done; }
  for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
  re_right_solve(n, n, X2, piv2, I, X3, &fl);                 /* step 5: X3 X2 = I  */
  re_right_solve(n, n, X2, piv2, X1, X4, &fl);                /*         X4 X2 = X1 */
  for (size_t t = 0; t < (size_t)n * n; ++t) { Xr[t] = X3[t]; Xi[t] = -X4[t]; }
done:
  if (flops) *flops = fl;
  free(F1); free(X1); free(X2); free(I); free(X3); free(X4); free(piv1); free(piv2);
  return info;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 6: almost sure Frobenius inversion, mu given by the caller.       */
/* ------------------------------------------------------------------------- */
int orc_frob_shift(int n, const double *A, const double *B, double mu, double *Xr, double *Xi,
                   double *flops) {
  double fl = 0.0;
  size_t nn = (size_t)n * n;
  double *X1 = re_alloc(n, n), *X2 = re_alloc(n, n), *X3 = re_alloc(n, n), *X4 = re_alloc(n, n);
  for (size_t t = 0; t < nn; ++t) {                           /* step 2 */
    X1[t] = A[t] - mu * B[t];
    X2[t] = mu * A[t] + B[t];
  }
  fl += 4.0 * (double)nn;
  double f5 = 0.0;
  int info = orc_frob_lu(n, X1, X2, X3, X4, &f5);             /* step 3: X3 + i X4 = (X1 + i X2)^{-1} */
  fl += f5;
  if (!info) {
    for (size_t t = 0; t < nn; ++t) {                         /* step 4 */
      Xr[t] = X3[t] - mu * X4[t];
      Xi[t] = mu * X3[t] + X4[t];
    }
    fl += 4.0 * (double)nn;
  }
  if (flops) *flops = fl;
  free(X1); free(X2); free(X3); free(X4);
  return info;
}

/* ------------------------------------------------------------------------- */
/* Real Cholesky A = R^T R, R upper triangular (row-oriented):               */
/*   r_jj = sqrt(a_jj - sum_{k<j} r_kj^2),                                     */
/*   r_ji = (a_ji - sum_{k<j} r_kj r_ki) / r_jj  for i > j.                    */
/* Reads the upper triangle of A.  Returns j+1 on a pivot that is not > 0.    */
/* ------------------------------------------------------------------------- */
static int re_potrf_upper(int n, const double *A, double *R, double *fl) {
  memset(R, 0, sizeof(double) * (size_t)n * n);
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= R[(size_t)k * n + j] * R[(size_t)k * n + j];
    if (!(s > 0.0)) return j + 1;
    double rjj = sqrt(s);
    R[(size_t)j * n + j] = rjj;
#pragma omp parallel for schedule(static)
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)j * n + i];
      for (int k = 0; k < j; ++k) t -= R[(size_t)k * n + j] * R[(size_t)k * n + i];
      R[(size_t)j * n + i] = t / rjj;
    }
    *fl += 2.0 * j + 1.0 + (double)(n - j - 1) * (2.0 * j + 1.0);
  }
  return 0;
}

/* R^T Z = Rhs (R^T lower triangular), all p columns; Rhs may be NULL for I. */
static void re_trsm_upperT(int n, int p, const double *R, const double *Rhs, double *Z, double *fl) {
#pragma omp parallel for schedule(dynamic, 8)
  for (int c = 0; c < p; ++c)
    for (int i = 0; i < n; ++i) {
      double s = Rhs ? Rhs[(size_t)i * p + c] : (i == c ? 1.0 : 0.0);
      for (int k = 0; k < i; ++k) s -= R[(size_t)k * n + i] * Z[(size_t)k * p + c];
      Z[(size_t)i * p + c] = s / R[(size_t)i * n + i];
    }
  *fl += (double)p * ((double)n * n);
}

/* R Z = Rhs (R upper triangular), all p columns, backward substitution. */
static void re_trsm_upper(int n, int p, const double *R, const double *Rhs, double *Z, double *fl) {
#pragma omp parallel for schedule(dynamic, 8)
  for (int c = 0; c < p; ++c)
    for (int i = n - 1; i >= 0; --i) {
      double s = Rhs[(size_t)i * p + c];
      for (int k = i + 1; k < n; ++k) s -= R[(size_t)i * n + k] * Z[(size_t)k * p + c];
      Z[(size_t)i * p + c] = s / R[(size_t)i * n + i];
    }
  *fl += (double)p * ((double)n * n);
}

/* ------------------------------------------------------------------------- */
/* Algorithm 7: Frobenius inversion with Cholesky decomposition.              */
/*   1. A = R1^T R1;  2. R1^T X1 = B;  3. R1 X2 = X1;  4. X3 = X1^T X1         */
/*   (symmetric: upper triangle computed, then mirrored, as in the count of   */
/*   Proposition 4.6);  5. X4 = A - X3;  6. X4 = R2^T R2;  7. R2^T X5 = I;     */
/*   8. R2 X6 = X5;  9. X7 = X2 X6;  output X6 - i X7.                         */
/* Steps 2 and 7 are printed as "backward" substitutions; R^T is lower        */
/* triangular, so they are forward substitutions here.                        */
/* ------------------------------------------------------------------------- */
/* step5_sign = -1: Algorithm 7 as printed (B skew: B A^{-1} B = -X1^T X1);
 * step5_sign = +1: the class closing Section 4.3, A and B symmetric positive
 * definite (B symmetric: B A^{-1} B = +X1^T X1), so step 5 reads X4 = A + X3. */
static int frob_chol_steps(int n, const double *A, const double *B, double step5_sign, double *Xr, double *Xi,
                           double *flops) {
  double fl = 0.0;
  int info = 0;
  size_t nn = (size_t)n * n;
  double *R1 = re_alloc(n, n), *X1 = re_alloc(n, n), *X2 = re_alloc(n, n), *X3 = re_alloc(n, n),
         *X4 = re_alloc(n, n), *R2 = re_alloc(n, n), *X5 = re_alloc(n, n), *X6 = re_alloc(n, n),
         *X7 = re_alloc(n, n);
  int k = re_potrf_upper(n, A, R1, &fl);                      /* step 1 */
  if (k) { info = ORC_STAGE_A + k; goto done; }
  re_trsm_upperT(n, n, R1, B, X1, &fl);                       /* step 2 */
  re_trsm_upper(n, n, R1, X1, X2, &fl);                       /* step 3 */
#pragma omp parallel for schedule(dynamic, 8)
  for (int i = 0; i < n; ++i)                                 /* step 4 */
    for (int j = i; j < n; ++j) {
      double s = 0.0;
      for (int t = 0; t < n; ++t) s += X1[(size_t)t * n + i] * X1[(size_t)t * n + j];
      X3[(size_t)i * n + j] = s;
      X3[(size_t)j * n + i] = s;
    }
  fl += 2.0 * (double)n * ((double)n * (n + 1) / 2.0);
  for (size_t t = 0; t < nn; ++t) X4[t] = A[t] + step5_sign * X3[t];   /* step 5 */
  fl += (double)nn;
  k = re_potrf_upper(n, X4, R2, &fl);                         /* step 6 */
  if (k) { info = ORC_STAGE_C + k; goto done; }
  re_trsm_upperT(n, n, R2, NULL, X5, &fl);                    /* step 7 */
  re_trsm_upper(n, n, R2, X5, X6, &fl);                       /* step 8 */
  re_add_mul(n, n, NULL, X2, X6, X7, &fl);                    /* step 9 */
  for (size_t t = 0; t < nn; ++t) { Xr[t] = X6[t]; Xi[t] = -X7[t]; }
done:
  if (flops) *flops = fl;
  free(R1); free(X1); free(X2); free(X3); free(X4); free(R2); free(X5); free(X6); free(X7);
  return info;
}

int orc_frob_chol(int n, const double *A, const double *B, double *Xr, double *Xi, double *flops) {
  return frob_chol_steps(n, A, B, -1.0, Xr, Xi, flops);
}

int orc_frob_chol_spd_pair(int n, const double *A, const double *B, double *Xr, double *Xi, double *flops) {
  return frob_chol_steps(n, A, B, 1.0, Xr, Xi, flops);
}

/* ------------------------------------------------------------------------- */
/* Algorithm 8: inversion with Cholesky decomposition (complex arithmetic).    */
/*   M = R^H R with r_jj = sqrt(m_jj - sum_{k<j} |r_kj|^2) real and            */
/*   r_ji = (m_ji - sum_{k<j} conj(r_kj) r_ki) / r_jj;  R^H X1 = I;  R X2 = X1 */
/* Reads the upper triangle of M (M is taken to be exactly Hermitian).        */
/* ------------------------------------------------------------------------- */
int orc_cinv_chol(int n, const double *Mr, const double *Mi, double *Xr, double *Xi, double *flops) {
  double fl = 0.0;
  int info = 0;
  cx *M = cx_alloc(n, n), *R = cx_alloc(n, n), *X1 = cx_alloc(n, n), *X2 = cx_alloc(n, n);
  cx_from_planar(n, n, Mr, Mi, M);
  for (int j = 0; j < n && !info; ++j) {
    double s = M[(size_t)j * n + j].re;
    for (int k = 0; k < j; ++k) {
      cx r = R[(size_t)k * n + j];
      s -= r.re * r.re + r.im * r.im;
    }
    if (!(s > 0.0)) { info = j + 1; break; }
    double rjj = sqrt(s);
    R[(size_t)j * n + j] = cx_make(rjj, 0.0);
#pragma omp parallel for schedule(static)
    for (int i = j + 1; i < n; ++i) {
      cx t = M[(size_t)j * n + i];
      for (int k = 0; k < j; ++k) t = cx_sub(t, cx_mul(cx_conj(R[(size_t)k * n + j]), R[(size_t)k * n + i]));
      R[(size_t)j * n + i] = cx_make(t.re / rjj, t.im / rjj);
    }
    fl += 4.0 * j + 1.0 + (double)(n - j - 1) * ((FL_CMUL + FL_CADD) * j + 2.0);
  }
  if (info) goto done;
  /* R^H X1 = I: (R^H)[i][k] = conj(R[k][i]), lower triangular */
#pragma omp parallel for schedule(dynamic, 8)
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      cx s = cx_make(i == c ? 1.0 : 0.0, 0.0);
      for (int k = 0; k < i; ++k) s = cx_sub(s, cx_mul(cx_conj(R[(size_t)k * n + i]), X1[(size_t)k * n + c]));
      double d = R[(size_t)i * n + i].re;
      X1[(size_t)i * n + c] = cx_make(s.re / d, s.im / d);
    }
  fl += (double)n * ((double)n * (n - 1) / 2.0 * (FL_CMUL + FL_CADD) + 2.0 * n);
  /* R X2 = X1, backward substitution */
#pragma omp parallel for schedule(dynamic, 8)
  for (int c = 0; c < n; ++c)
    for (int i = n - 1; i >= 0; --i) {
      cx s = X1[(size_t)i * n + c];
      for (int k = i + 1; k < n; ++k) s = cx_sub(s, cx_mul(R[(size_t)i * n + k], X2[(size_t)k * n + c]));
      double d = R[(size_t)i * n + i].re;
      X2[(size_t)i * n + c] = cx_make(s.re / d, s.im / d);
    }
  fl += (double)n * ((double)n * (n - 1) / 2.0 * (FL_CMUL + FL_CADD) + 2.0 * n);
  cx_to_planar(n, n, X2, Xr, Xi);
done:
  if (flops) *flops = fl;
  free(M); free(R); free(X1); free(X2);
  return info;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 3: linear system with Frobenius inversion and LU factorization.   */
/*   1. A = P1^T L1 U1;  2. L1 U1 X1 = P1 B;  3. X2 = A + B X1;                */
/*   4. X2 = P2^T L2 U2;  5. L2 U2 [x1, y1] = P2 [c, d];                       */
/*   6. L1 U1 [x2, y2] = P1 B [y1, x1];  7. x = x1 + x2, y = y1 - y2.          */
/* ------------------------------------------------------------------------- */
int orc_frob_solve(int n, int p, const double *A, const double *B, const double *c, const double *d,
                   double *x, double *y, double *flops) {
  double fl = 0.0;
  int info = 0;
  int q = 2 * p;
  double *F1 = re_alloc(n, n), *X1 = re_alloc(n, n), *X2 = re_alloc(n, n), *CD = re_alloc(n, q),
         *YX = re_alloc(n, q), *T = re_alloc(n, q);
  int *piv1 = (int *)calloc((size_t)n, sizeof(int)), *piv2 = (int *)calloc((size_t)n, sizeof(int));
  memcpy(F1, A, sizeof(double) * (size_t)n * n);
  int k = re_getrf(n, F1, piv1, &fl);                         /* step 1 */
  if (k) { info = ORC_STAGE_A + k; goto done; }
  memcpy(X1, B, sizeof(double) * (size_t)n * n);
  re_getrs_cols(n, n, F1, piv1, X1, &fl);                     /* step 2 */
  re_add_mul(n, n, A, B, X1, X2, &fl);                        /* step 3 */
  k = re_getrf(n, X2, piv2, &fl);                             /* step 4 */
  if (k) { info = ORC_STAGE_C + k; goto done; }
  for (int i = 0; i < n; ++i)                                 /* step 5: [c, d] -> [x1, y1] */
    for (int j = 0; j < p; ++j) {
      CD[(size_t)i * q + j] = c[(size_t)i * p + j];
      CD[(size_t)i * q + p + j] = d[(size_t)i * p + j];
    }
  re_getrs_cols(n, q, X2, piv2, CD, &fl);
  for (int i = 0; i < n; ++i)                                 /* step 6: [y1, x1] */
    for (int j = 0; j < p; ++j) {
      YX[(size_t)i * q + j] = CD[(size_t)i * q + p + j];
      YX[(size_t)i * q + p + j] = CD[(size_t)i * q + j];
    }
  re_add_mul(n, q, NULL, B, YX, T, &fl);                      /*   T = B [y1, x1] */
  re_getrs_cols(n, q, F1, piv1, T, &fl);                      /*   [x2, y2] = A^{-1} T */
  for (int i = 0; i < n; ++i)                                 /* step 7 */
    for (int j = 0; j < p; ++j) {
      x[(size_t)i * p + j] = CD[(size_t)i * q + j] + T[(size_t)i * q + j];
      y[(size_t)i * p + j] = CD[(size_t)i * q + p + j] - T[(size_t)i * q + p + j];
    }
  fl += 2.0 * (double)n * p;
done:
  if (flops) *flops = fl;
  free(F1); free(X1); free(X2); free(CD); free(YX); free(T); free(piv1); free(piv2);
  return info;
}

/* ------------------------------------------------------------------------- */
/* Adjoint: dM = -X^H G X^H.  From d(M^{-1}) = -M^{-1} dM M^{-1}:             */
/* for L = Re tr(W X), dL = Re tr(-X W X dM) = Re sum(conj(-X^H W^H X^H) .* dM)*/
/* so with G = W^H the gradient in that convention is -X^H G X^H.             */
/* ------------------------------------------------------------------------- */
void orc_adjoint(int n, const double *Xr, const double *Xi, const double *Gr, const double *Gi, double *dMr,
                 double *dMi) {
  cx *X = cx_alloc(n, n), *G = cx_alloc(n, n), *T = cx_alloc(n, n);
  cx_from_planar(n, n, Xr, Xi, X);
  cx_from_planar(n, n, Gr, Gi, G);
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i)          /* T = X^H G: T[i][j] = sum_k conj(X[k][i]) G[k][j] */
    for (int j = 0; j < n; ++j) {
      cx s = cx_make(0.0, 0.0);
      for (int k = 0; k < n; ++k) s = cx_add(s, cx_mul(cx_conj(X[(size_t)k * n + i]), G[(size_t)k * n + j]));
      T[(size_t)i * n + j] = s;
    }
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i)          /* dM = -T X^H: dM[i][j] = -sum_k T[i][k] conj(X[j][k]) */
    for (int j = 0; j < n; ++j) {
      cx s = cx_make(0.0, 0.0);
      for (int k = 0; k < n; ++k) s = cx_add(s, cx_mul(T[(size_t)i * n + k], cx_conj(X[(size_t)j * n + k])));
      dMr[(size_t)i * n + j] = -s.re;
      dMi[(size_t)i * n + j] = -s.im;
    }
  free(X); free(G); free(T);
}

void orc_cmatmul(int n, int k, int m, const double *Xr, const double *Xi, const double *Yr, const double *Yi,
                 double *Zr, double *Zi) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) {
      cx s = cx_make(0.0, 0.0);
      for (int t = 0; t < k; ++t)
        s = cx_add(s, cx_mul(cx_make(Xr[(size_t)i * k + t], Xi[(size_t)i * k + t]),
                             cx_make(Yr[(size_t)t * m + j], Yi[(size_t)t * m + j])));
      Zr[(size_t)i * m + j] = s.re;
      Zi[(size_t)i * m + j] = s.im;
    }
}

/* ------------------------------------------------------------------------- */
/* Section 5 (experiments): Newton iterations built on inversion.             */
/* The max norm of eq. (maxnorm) is the largest |entry| over both parts.      */
/* ------------------------------------------------------------------------- */
static double planar_maxabs(size_t cnt, const double *re, const double *im) {
  double m = 0.0;
  for (size_t t = 0; t < cnt; ++t) {
    const double a = fabs(re[t]), b = fabs(im[t]);
    if (a > m) m = a;
    if (b > m) m = b;
  }
  return m;
}

/* Section 5.3, eq. (iter): X_{k+1} = (X_k + X_k^{-1}) / 2 from X_0 = X, each
 * inverse by Algorithm 4; stop when ||X_k - X_{k-1}||_max / ||X_k||_max <= eps
 * or k >= kmax.  Returns 0, or the info of the inversion that failed. */
int orc_sign_newton(int n, const double *Xr, const double *Xi, double eps, int kmax, double *Sr, double *Si,
                    int *iters) {
  const size_t nn = (size_t)n * n;
  double *Ir = re_alloc(n, n), *Ii = re_alloc(n, n);
  memcpy(Sr, Xr, nn * sizeof(double));
  memcpy(Si, Xi, nn * sizeof(double));
  int k = 0, info = 0;
  while (k < kmax) {
    info = orc_cinv_lu(n, Sr, Si, Ir, Ii, NULL, NULL);
    if (info) break;
    double dmax = 0.0;
    for (size_t t = 0; t < nn; ++t) {
      const double nr = 0.5 * (Sr[t] + Ir[t]), ni = 0.5 * (Si[t] + Ii[t]);
      const double dr = fabs(nr - Sr[t]), di = fabs(ni - Si[t]);
      if (dr > dmax) dmax = dr;
      if (di > dmax) dmax = di;
      Sr[t] = nr;
      Si[t] = ni;
    }
    ++k;
    if (dmax <= eps * planar_maxabs(nn, Sr, Si)) break;
  }
  if (iters) *iters = k;
  free(Ir); free(Ii);
  return info;
}

/* Section 5.5, eq. (iter2): X_{k+1} = (X_k + X_k^{-H}) / 2 from X_0 = X (the
 * unitary polar factor Q in the limit), the same stopping rule, then
 * P = Q^H X.  Returns 0, or the info of the inversion that failed. */
int orc_polar_newton(int n, const double *Xr, const double *Xi, double eps, int kmax, double *Qr, double *Qi,
                     double *Pr, double *Pi, int *iters) {
  const size_t nn = (size_t)n * n;
  double *Ir = re_alloc(n, n), *Ii = re_alloc(n, n), *Nr = re_alloc(n, n), *Ni = re_alloc(n, n);
  memcpy(Qr, Xr, nn * sizeof(double));
  memcpy(Qi, Xi, nn * sizeof(double));
  int k = 0, info = 0;
  while (k < kmax) {
    info = orc_cinv_lu(n, Qr, Qi, Ir, Ii, NULL, NULL);
    if (info) break;
    double dmax = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const size_t t = (size_t)i * n + j, tt = (size_t)j * n + i;   /* (X^{-H})_{ij} = conj((X^{-1})_{ji}) */
        Nr[t] = 0.5 * (Qr[t] + Ir[tt]);
        Ni[t] = 0.5 * (Qi[t] - Ii[tt]);
        const double dr = fabs(Nr[t] - Qr[t]), di = fabs(Ni[t] - Qi[t]);
        if (dr > dmax) dmax = dr;
        if (di > dmax) dmax = di;
      }
    memcpy(Qr, Nr, nn * sizeof(double));
    memcpy(Qi, Ni, nn * sizeof(double));
    ++k;
    if (dmax <= eps * planar_maxabs(nn, Qr, Qi)) break;
  }
  if (iters) *iters = k;
  if (!info) {
    /* P = Q^H X: P[i][j] = sum_t conj(Q[t][i]) X[t][j] */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        cx s = cx_make(0.0, 0.0);
        for (int t = 0; t < n; ++t)
          s = cx_add(s, cx_mul(cx_make(Qr[(size_t)t * n + i], -Qi[(size_t)t * n + i]),
                               cx_make(Xr[(size_t)t * n + j], Xi[(size_t)t * n + j])));
        Pr[(size_t)i * n + j] = s.re;
        Pi[(size_t)i * n + j] = s.im;
      }
  }
  free(Ir); free(Ii); free(Nr); free(Ni);
  return info;
}

/* Section 5.4: the Sylvester equation A Y + Y B = C (A p x p, B q x q, C p x q)
 * with sign(A) = I and sign(B) = I, through
 *   sign([[A, -C], [0, -B]]) = [[I, -2Y], [0, -I]]:
 * the Newton iteration of Section 5.3 on the (p + q) x (p + q) block matrix,
 * then Y = -(1/2) times its upper right block.  Returns 0 or the failing info. */
int orc_sylvester_newton(int p, int q, const double *Ar, const double *Ai, const double *Br, const double *Bi,
                         const double *Cr, const double *Ci, double eps, int kmax, double *Yr, double *Yi,
                         int *iters) {
  const int N = p + q;
  double *Xr = re_alloc(N, N), *Xi = re_alloc(N, N), *Sr = re_alloc(N, N), *Si = re_alloc(N, N);
  for (int i = 0; i < p; ++i) {
    for (int j = 0; j < p; ++j) {
      Xr[(size_t)i * N + j] = Ar[(size_t)i * p + j];
      Xi[(size_t)i * N + j] = Ai[(size_t)i * p + j];
    }
    for (int j = 0; j < q; ++j) {
      Xr[(size_t)i * N + p + j] = -Cr[(size_t)i * q + j];
      Xi[(size_t)i * N + p + j] = -Ci[(size_t)i * q + j];
    }
  }
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) {
      Xr[(size_t)(p + i) * N + p + j] = -Br[(size_t)i * q + j];
      Xi[(size_t)(p + i) * N + p + j] = -Bi[(size_t)i * q + j];
    }
  const int info = orc_sign_newton(N, Xr, Xi, eps, kmax, Sr, Si, iters);
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < q; ++j) {
      Yr[(size_t)i * q + j] = -0.5 * Sr[(size_t)i * N + p + j];
      Yi[(size_t)i * q + j] = -0.5 * Si[(size_t)i * N + p + j];
    }
  free(Xr); free(Xi); free(Sr); free(Si);
  return info;
}

/* ------------------------------------------------------------------------- */
/* Section 2.4: matrices over an iterated quadratic extension                 */
/*   F_m = R[xi_1, ..., xi_m] / <xi_1^2 + tau_1, ..., xi_m^2 + tau_m>          */
/* (eq. (K_m quotient) with every f_k = x^2 + tau_k), written as              */
/* X = sum_alpha C_alpha xi^alpha (eq. (iterquadmat)), alpha in {0,1}^m.       */
/* Plane p holds C_alpha with alpha_k = bit k-1 of p.                         */
/* Basis products: xi^a xi^b = s(a, b) xi^(a xor b) with s(a, b) the product  */
/* of -tau_k over the k where both a_k and b_k are 1.                         */
/* ------------------------------------------------------------------------- */
static double tower_sign(int m, const double *tau, int a, int b) {
  double s = 1.0;
  for (int k = 0; k < m; ++k)
    if ((a >> k) & (b >> k) & 1) s *= -tau[k];
  return s;
}

/* Z = X Y in F_m^{n x n} from the definition: Z_g = sum_a s(a, a^g) X_a Y_(a^g). */
void orc_tower_mul(int m, int n, const double *tau, const double *X, const double *Y, double *Z) {
  const int P = 1 << m;
  const size_t nn = (size_t)n * n;
  memset(Z, 0, nn * (size_t)P * sizeof(double));
  for (int g = 0; g < P; ++g)
    for (int a = 0; a < P; ++a) {
      const int b = a ^ g;
      const double s = tower_sign(m, tau, a, b);
      const double *Xa = X + (size_t)a * nn, *Yb = Y + (size_t)b * nn;
      double *Zg = Z + (size_t)g * nn;
#pragma omp parallel for schedule(static)
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          double acc = 0.0;
          for (int t = 0; t < n; ++t) acc += Xa[(size_t)i * n + t] * Yb[(size_t)t * n + j];
          Zg[(size_t)i * n + j] += s * acc;
        }
    }
}

/* X^{-1} in F_m^{n x n} from its definition X Z = 1: multiplication by X is a
 * real linear map on the 2^m coefficient matrices of Z (the regular
 * representation: block (g, b) = s(g^b, b) C_(g^b)); the coefficients of the
 * inverse solve it with right-hand side "1" (the identity in plane 0, zeros
 * elsewhere), by real Gaussian elimination with partial pivoting.  Returns the
 * 1-based zero-pivot index of the 2^m n system, or 0. */
int orc_tower_inv(int m, int n, const double *tau, const double *C, double *Xinv) {
  const int P = 1 << m;
  const int N = P * n;
  const size_t nn = (size_t)n * n;
  double *L = re_alloc(N, N), *Z = re_alloc(N, n);
  int *piv = (int *)calloc((size_t)N, sizeof(int));
  for (int g = 0; g < P; ++g)
    for (int b = 0; b < P; ++b) {
      const int a = g ^ b;
      const double s = tower_sign(m, tau, a, b);
      const double *Ca = C + (size_t)a * nn;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) L[(size_t)(g * n + i) * N + b * n + j] = s * Ca[(size_t)i * n + j];
    }
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  double fl = 0.0;
  int info = re_getrf(N, L, piv, &fl);
  if (!info) {
    re_getrs_cols(N, n, L, piv, Z, &fl);
    for (int b = 0; b < P; ++b)
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Xinv[(size_t)b * nn + (size_t)i * n + j] = Z[(size_t)(b * n + i) * n + j];
  }
  free(L); free(Z); free(piv);
  return info;
}

/* ------------------------------------------------------------------------- */
/* Reference solutions of M x = b accurate beyond u kappa(M), for checking   */
/* results that are themselves refined: complex GEPP (as in Algorithm 4),     */
/* then iterative refinement whose residual r = b - M x is accumulated in     */
/* double-double arithmetic (error-free products by Dekker's splitting,       */
/* error-free sums by Knuth's TwoSum; no fused multiply-add anywhere), the    */
/* correction solved with the same LU factors.  With u kappa(M) < 1 each step */
/* gains a factor of about u kappa(M) until the result is accurate to about   */
/* the unit roundoff.                                                         */
/* ------------------------------------------------------------------------- */
typedef struct { double hi, lo; } dd;

static inline void two_sum(double a, double b, double *s, double *e) {
  const double x = a + b, bb = x - a;
  *s = x;
  *e = (a - (x - bb)) + (b - bb);
}
static inline void split(double a, double *h, double *l) {
  const double c = 134217729.0 * a;   /* 2^27 + 1 */
  *h = c - (c - a);
  *l = a - *h;
}
static inline void two_prod(double a, double b, double *p, double *e) {
  double ah, al, bh, bl;
  split(a, &ah, &al);
  split(b, &bh, &bl);
  const double x = a * b;
  *p = x;
  *e = ((ah * bh - x) + ah * bl + al * bh) + al * bl;
}
static inline dd dd_add_d(dd a, double b) {
  double s, e;
  two_sum(a.hi, b, &s, &e);
  e += a.lo;
  double s2, e2;
  two_sum(s, e, &s2, &e2);
  dd r = {s2, e2};
  return r;
}
static inline dd dd_add_prod(dd a, double x, double y) {   /* a + x * y */
  double p, e;
  two_prod(x, y, &p, &e);
  a = dd_add_d(a, p);
  return dd_add_d(a, e);
}

/* Solve with the factors of cx_getrf (W, piv): z <- U^{-1} L^{-1} P z. */
static void cx_getrs1(int n, const cx *W, const int *piv, cx *z) {
  for (int k = 0; k < n; ++k) {
    const int q = piv[k];
    if (q != k) { cx t = z[k]; z[k] = z[q]; z[q] = t; }
  }
  for (int i = 0; i < n; ++i) {
    cx s = z[i];
    for (int j = 0; j < i; ++j) s = cx_sub(s, cx_mul(W[(size_t)i * n + j], z[j]));
    z[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    cx s = z[i];
    for (int j = i + 1; j < n; ++j) s = cx_sub(s, cx_mul(W[(size_t)i * n + j], z[j]));
    z[i] = cx_div(s, W[(size_t)i * n + i]);
  }
}

/* x (n x p, planar) solves M x = b; `steps` refinement steps (0: plain GEPP).
 * *last (if not NULL) receives the largest ||dx||_inf / ||x||_inf of the final
 * correction over the columns.  Returns 0 or k + 1 for an exactly zero pivot. */
int orc_csolve_refined(int n, int p, const double *Mr, const double *Mi, const double *Br, const double *Bi,
                       int steps, double *Xr, double *Xi, double *last) {
  double fl = 0.0;
  cx *W = cx_alloc(n, n);
  int *piv = (int *)calloc((size_t)n, sizeof(int));
  cx_from_planar(n, n, Mr, Mi, W);
  const int info = cx_getrf(n, W, piv, &fl);
  double worst = 0.0;
  if (!info) {
#pragma omp parallel for schedule(dynamic, 1) reduction(max : worst)
    for (int c = 0; c < p; ++c) {
      cx *x = cx_alloc(n, 1), *r = cx_alloc(n, 1);
      for (int i = 0; i < n; ++i) x[i] = cx_make(Br[(size_t)i * p + c], Bi[(size_t)i * p + c]);
      cx_getrs1(n, W, piv, x);
      for (int it = 0; it < steps; ++it) {
        /* r = b - M x in double-double, rounded once */
        for (int i = 0; i < n; ++i) {
          dd re = {Br[(size_t)i * p + c], 0.0}, im = {Bi[(size_t)i * p + c], 0.0};
          const double *mr = Mr + (size_t)i * n, *mi = Mi + (size_t)i * n;
          for (int j = 0; j < n; ++j) {
            /* (mr + i mi)(xr + i xi) = (mr xr - mi xi) + i (mr xi + mi xr) */
            re = dd_add_prod(re, -mr[j], x[j].re);
            re = dd_add_prod(re, mi[j], x[j].im);
            im = dd_add_prod(im, -mr[j], x[j].im);
            im = dd_add_prod(im, -mi[j], x[j].re);
          }
          r[i] = cx_make(re.hi + re.lo, im.hi + im.lo);
        }
        cx_getrs1(n, W, piv, r);
        double dmax = 0.0, xmax = 0.0;
        for (int i = 0; i < n; ++i) {
          x[i] = cx_add(x[i], r[i]);
          dmax = fmax(dmax, fmax(fabs(r[i].re), fabs(r[i].im)));
          xmax = fmax(xmax, fmax(fabs(x[i].re), fabs(x[i].im)));
        }
        if (it == steps - 1 && xmax > 0.0) worst = fmax(worst, dmax / xmax);
      }
      for (int i = 0; i < n; ++i) { Xr[(size_t)i * p + c] = x[i].re; Xi[(size_t)i * p + c] = x[i].im; }
      free(x); free(r);
    }
  }
  if (last) *last = worst;
  free(W); free(piv);
  return info;
}
