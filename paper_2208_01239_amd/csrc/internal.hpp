// internal.hpp -- launchers and drivers shared between the translation units of
// libfrobinv.  Nothing here is part of the public C ABI (include/frobinv.h).
#pragma once

#include "common.hpp"

struct frob_handle;

namespace frob {

// ----------------------------------------------------------------- GEMM (FP64)
enum { GEMM_CFG_128x128 = 0, GEMM_CFG_64x64 = 1, GEMM_CFG_128x32 = 2, GEMM_CFG_32x128 = 3 };
// GEMM_NEED_FULL_M: one block row must cover all of M (in-place left products);
// GEMM_NEED_FULL_N: one block column must cover all of N (in-place right products).
enum { GEMM_NEED_ANY = 0, GEMM_NEED_FULL_M = 1, GEMM_NEED_FULL_N = 2 };
int gemm_pick_cfg(int M, int N, int need);

// C = alpha op(A) op(B) + beta C, see gemm_f64.hip.
void gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, DOp A, int triA, DOp B,
              int triB, double beta, DOut C, bool lowerOnly = false, int batch = 1, long long sA = 0,
              long long sB = 0, long long sC = 0, int need = GEMM_NEED_ANY);

// Batched variant with separate strides for the row-index arrays.
void gemm_f64_batched(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, DOp A, int triA, DOp B,
                      int triB, double beta, DOut C, bool lowerOnly, int batch, long long sA, long long sB,
                      long long sC, int rsA, int rsB, int rsC, int need = GEMM_NEED_ANY);

// ------------------------------------------------------ low-precision GEMM
// Same product with the operands rounded to FP32 or BF16 when staged and FP32
// accumulation (gemm_lp.hip); storage FP64 or FP32.
enum { LP_NONE = 0, LP_F32 = 1, LP_BF16 = 2 };
void gemm_lp(hipStream_t s, int mode, bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
             const int* rA, const double* B, int ldb, const int* rB, double beta, double* C, int ldc, const int* rC,
             bool lowerOnly, int batch, long long sA, long long sB, long long sC);
void gemm_lp(hipStream_t s, int mode, bool ta, bool tb, int M, int N, int K, double alpha, const float* A, int lda,
             const int* rA, const float* B, int ldb, const int* rB, double beta, float* C, int ldc, const int* rC,
             bool lowerOnly, int batch, long long sA, long long sB, long long sC);
// While a LowPrecScope is alive on the calling host thread, gemm_f64 sends its
// plain products (no triangular operand, no in-place requirement, no column
// scatter, K >= 32) to gemm_lp in that mode: the mixed-precision
// factorizations reuse the FP64 drivers unchanged.
int lp_mode();
struct LowPrecScope {
  int prev;
  explicit LowPrecScope(int mode);
  ~LowPrecScope();
};
// While a GridCapScope is alive on the calling host thread, gemm_f64 launches
// at most that many workgroups (rounded down to a multiple of 8), each taking
// several tiles: the look-ahead's trailing updates then leave compute units
// free for the panel chain on the other stream.  0 = no cap.
int grid_cap();
struct GridCapScope {
  int prev;
  explicit GridCapScope(int blocks);
  ~GridCapScope();
};

// Planar complex GEMM, C = alpha op(A) op(B) + beta C with real alpha/beta and
// op in {N, T, C (conjugate transpose)}; four real MFMA products per tile.
enum { OP_N = 0, OP_T = 1, OP_C = 2 };
void gemm_z64(hipStream_t s, int opA, int opB, int M, int N, int K, double alpha, ZOp A, int triA, ZOp B,
              int triB, double beta, ZOut C, bool lowerOnly = false, int need = GEMM_NEED_ANY);
void gemm_z64_batched(hipStream_t s, int opA, int opB, int M, int N, int K, double alpha, ZOp A, int triA, ZOp B,
                      int triB, double beta, ZOut C, bool lowerOnly, int batch, long long sA, long long sB,
                      long long sC, int rsA, int rsB, int rsC, int need = GEMM_NEED_ANY);

// ------------------------------------------------------- small triangular solves
// In-place solve with a triangle of order nt <= 64 (one LDS-resident block):
//   left:  op(T) X = B   (B is nt x nr),   right: X op(T) = B  (B is nr x nt).
// `tri` describes op(T) (lower/upper, unit/non-unit) in logical coordinates;
// `trans` selects op(T) = T^T.
void trsm_small_f64(hipStream_t s, bool right, int tri, bool trans, int nt, int nr, DOp T, DOut B);
// Complex analogue; with `identity` set the right-hand side is the identity
// (B is then output only, nr = nt).
void trsm_small_z64(hipStream_t s, bool right, int tri, int opT, int nt, int nr, ZOp T, ZOut B, bool identity);
size_t trsm_z_work_elems(int nt);   // doubles, both planes

// --------------------------------------------------- blocked triangular drivers
// Recursive triangular solve (left or right) built from the small solves and
// GEMM updates.  Arguments as for trsm_small_*, any order nt.
// `work` must hold trsm_work_elems(nt) doubles (diagonal-block inverses).
size_t trsm_work_elems(int nt);
void trsm_f64(hipStream_t s, bool right, int tri, bool trans, int nt, int nr, DOp T, DOut B, double* work);
// Inverses of the diagonal blocks of op(T) of order nb (a power of two >= 64),
// written on the diagonal of D (n x n, ld D.ld); `tmp` holds n*nb/4 + 64 doubles.
void dinv_f64(hipStream_t s, int tri, bool trans, int n, DOp T, int nb, double* D, int ldd, double* tmp);
void trsm_z64(hipStream_t s, bool right, int tri, int opT, int nt, int nr, ZOp T, ZOut B, double* work);
// W = op(T)^{-1} for a triangle of order n into a separate plain buffer W
// (n x n, ld ldw; the other triangle is set to zero).  tmp holds trtri_tmp_elems(n).
size_t trtri_tmp_elems(int n);
void trtri_f64(hipStream_t s, int tri, bool trans, int n, DOp T, double* W, int ldw, double* tmp);
size_t trtri_z_tmp_elems(int n);
void trtri_z64(hipStream_t s, int tri, int opT, int n, ZOp T, double* Wre, double* Wim, int ldw, double* tmp);

// ------------------------------------------------------------- factorizations
// LU with partial pivoting of the n x n matrix a (row-major, lda), in place,
// pivoting through the index array perm (initialised to the identity here):
// logical row i of P A = L U lives in physical row perm[i].  *info (device)
// receives the 1-based column of the first exactly-zero pivot or stays 0.
// `work` holds getrf_work_elems(n) doubles.
//
// With q > 0 the q columns right of the matrix (a + n, same rows and lda) take
// the row interchanges and the elimination without a pivot search: they end
// holding L^{-1} P times their input, rows addressed through perm.  With the
// look-ahead they are updated with the trailing columns on the second stream.
//
// With a LookAhead (a second stream and events owned by the handle) orders
// n >= LA_MIN are factored in panels of LA_NB columns with a look-ahead of
// one panel: the update of the next panel's columns stays on `s`, the update
// of the remaining columns runs on the second stream, concurrently with the
// next panel's factorization.  The call returns with all work ordered on `s`.
struct LookAhead {
  hipStream_t s1 = nullptr;
  hipEvent_t ev[8] = {};
  frob_handle* prof = nullptr;   // times the second stream's trailing-update GEMMs when profiling is on
  int nb = 64;                   // panel width of the real LU (16, 32, 48 or 64; set per call)
};
// Panel widths (real, complex): the next panel's update is then one
// recursion-node launch (real nodes up to 64 columns, complex up to 32).
// Measured at n = 4096: real 64 / 48 / 32 -> 42.1 / 44.3 / 42.5 ms per
// Frobenius inversion, complex 32 / 64 -> 39.8 / 44.0 ms per complex LU
// inversion; 128 to 512 were slower still.
constexpr int LA_NB = 64;
// Panels per super-panel of the real LU: columns right of a super-panel take
// its panels as one rank-(LA_SUPER * LA_NB) update.
constexpr int LA_SUPER = 1;
constexpr int ZLA_NB = 32;
constexpr int LA_MIN = 1024;
// Workgroups of a trailing update on the second stream: fewer than the chip
// holds, so the panel chain's single-workgroup leaves find a free compute unit.
constexpr int LA_GRID_CAP = 224;
// Largest order whose Frobenius LUs carry B / the identity as extra columns:
// the second stream's extra updates (n^3 flops each) fit beside the panel
// chain at n = 2048 and 4096 (faster) but not at 8192 (slower).
constexpr int LA_CARRY_MAX = 4096;
size_t getrf_work_elems(int n);
void getrf_f64(hipStream_t s, int n, double* a, int lda, int* perm, int* info, double* work,
               const LookAhead* la = nullptr, int q = 0);
// whether getrf_f64 factors order n with the look-ahead
bool getrf_lookahead_on(int n, const LookAhead* la);
size_t getrf_z_work_elems(int n);
void getrf_z64(hipStream_t s, int n, double* re, double* im, int lda, int* perm, int* info, double* work,
               const LookAhead* la = nullptr);
// Cholesky A = L L^T (lower, in place in the lower triangle of a; the strict
// upper triangle is not referenced).  *info receives the 1-based index of the
// first non-positive pivot.
size_t potrf_work_elems(int n);
void potrf_f64(hipStream_t s, int n, double* a, int lda, int* info, double* work);
size_t potrf_z_work_elems(int n);
void potrf_z64(hipStream_t s, int n, double* re, double* im, int lda, int* info, double* work);

// ------------------------------------------------------------ elementwise ops
void iota_i32(hipStream_t s, int n, int* p);
void fill_i32(hipStream_t s, int n, int v, int* p);
// R <- I - R for a planar complex n x n R; *sumsq (device) <- ||I - R||_F^2
void resid_form_f64(hipStream_t s, int n, double* Rr, double* Ri, int ld, double* sumsq);
void copy_f64(hipStream_t s, int m, int n, const double* src, int lds, const int* src_rows, double* dst, int ldd);
void fill_f64(hipStream_t s, int m, int n, double v, double* dst, int ldd);
void identity_f64(hipStream_t s, int n, double* dst, int ldd);
// Y = a X + b Y  (m x n)
void axpby_f64(hipStream_t s, int m, int n, double a, const double* X, int ldx, double b, double* Y, int ldy);
// Z = a X + b Y
void lincomb_f64(hipStream_t s, int m, int n, double a, const double* X, int ldx, double b, const double* Y, int ldy,
                 double* Z, int ldz);
// Xr += P - Q, Xi += P + Q
void acc_rot_f64(hipStream_t s, int m, int n, const double* P, int ldp, const double* Q, int ldq, double* Xr,
                 double* Xi, int ldx);
// (X1, X2) = (A - mu B, mu A + B): shift in; used in-place-safe on distinct buffers
void rotate_f64(hipStream_t s, int m, int n, double mu, const double* A, int lda, const double* B, int ldb,
                double* X1, int ld1, double* X2, int ld2);
// (X1, X2) = (c A - s B, s A + c B): the parts of e^{i theta} (A + iB) for c = cos, s = sin
void rot_f64(hipStream_t s, int m, int n, double c, double sn, const double* A, int lda, const double* B, int ldb,
             double* X1, int ld1, double* X2, int ld2);
// *out = ||a||_1 (largest column sum of |a|) for an n x n matrix; colsum holds n doubles
void norm1_f64(hipStream_t s, int n, const double* a, int lda, double* colsum, double* out);
// dst[:, perm[k]] = src[:, k]
void permute_cols_f64(hipStream_t s, int m, int n, const double* src, int lds, const int* perm, double* dst,
                      int ldd);
// Mirror the strict lower triangle into the upper one: a[j][i] = sign * a[i][j]
void mirror_lower_f64(hipStream_t s, int n, double* a, int lda, double sign);
// Zero the strict upper triangle
void zero_upper_f64(hipStream_t s, int n, double* a, int lda);
// Newton iterations on the inversion: X <- (X + op(I)) / 2 with op(I) = I or
// I^H (herm), and maxes[0] / maxes[1] <- the max norms of the change and of
// the new iterate (as the bit patterns of non-negative doubles).
void newton_step(hipStream_t s, int n, double* Xr, double* Xi, int ldx, const double* Ir, const double* Ii, int ldi,
                 bool herm, unsigned long long* maxes);
// X = [[A, -C], [0, -B]] (B = A^H when lyap) of order p + q, leading dimension p + q
void sylvester_assemble(hipStream_t s, int p, int q, const double* Ar, const double* Ai, int lda, const double* Br,
                        const double* Bi, int ldb, bool lyap, const double* Cr, const double* Ci, int ldc,
                        double* Xr, double* Xi);
// Y = -(1/2) times the upper right p x q block of S (order p + q)
void sylvester_extract(hipStream_t s, int p, int q, const double* Sr, const double* Si, double* Yr, double* Yi,
                       int ldy);
// Gauss's scheme over x^2 + tau (Proposition 2.2): with P1 in Z0, P2 in Z1 and
// P3 = (X0 + X1)(Y0 + Y1): Z0 <- P1 - tau P2, Z1 <- P3 - P1 - P2 (cnt elements)
void gauss3_combine_f64(hipStream_t s, long long cnt, double* Z0, double* Z1, const double* P3, double tau);
// Widen / round between FP32 and FP64 storage (m x n, leading dimensions)
void convert_f32_f64(hipStream_t s, int m, int n, const float* src, int lds, double* dst, int ldd);
void convert_f64_f32(hipStream_t s, int m, int n, const double* src, int lds, float* dst, int ldd);

}  // namespace frob
