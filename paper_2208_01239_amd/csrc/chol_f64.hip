// chol_f64.hip -- Cholesky factorization A = L L^T (lower, row-major) in FP64.
//
// Recursive: factor A11, L21 = A21 L11^{-T} (right triangular solve), lower
// half of A22 -= L21 L21^T (one GEMM writing only the lower triangle), factor
// A22.  The base case factors a diagonal block of order <= 64 held in the
// registers of one workgroup (square root and pivot test on the diagonal in
// FP64).  The first non-positive (or NaN) pivot stops the factorization and
// is recorded in *info (1-based).
#include "common.hpp"
#include "internal.hpp"
#include "tri_dev.hpp"

namespace frob {

namespace {

constexpr int CB = 64;

// Base case, order n <= 64, right-looking with the matrix in registers:
// thread (ti, tj) of a 16 x 16 grid owns the 4 x 4 block at rows 4 ti,
// columns 4 tj (blocks above the diagonal stay idle).  Per column j every
// thread reads column j (as updated so far) from a parity-double-buffered
// LDS copy, forms L(:, j) with the reciprocal of the pivot's square root
// (scaling as LAPACK's potf2 does), updates its block, and the owners of
// column j + 1 publish it: one barrier per column.
__global__ __launch_bounds__(256) void k_potrf_small_f64(double* a, int lda, int n, int k0, int* info) {
  __shared__ double colbuf[2][CB];
  const int tid = threadIdx.x;
  if (*info != 0) return;  // an earlier block already failed (uniform)
  const int ti = tid >> 4, tj = tid & 15;
  const bool low = ti >= tj;
  double blk[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = 4 * ti + r, k = 4 * tj + c;
      const bool in = i < n && k <= i;
      blk[r][c] = in ? a[(long long)min(i, n - 1) * lda + min(k, n - 1)] : 0.0;
    }
  if (tj == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) colbuf[0][4 * ti + r] = blk[r][0];
  }
  __syncthreads();
  int bad = 0;
  for (int jb = 0; jb < CB / 4 && !bad; ++jb) {
    StaticFor<0, 4>::run([&](auto jcc) {
      constexpr int jc = decltype(jcc)::value;
      const int j = 4 * jb + jc;
      if (bad || j >= n) return;  // uniform
      const int par = j & 1;
      const double djj = colbuf[par][j];
      if (!(djj > 0.0)) {   // uniform: every thread read the same value
        bad = j + 1;
        return;
      }
      // the column's entries are read unconditionally (one LDS round trip),
      // then selected
      double ci[4], ck[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) ci[r] = colbuf[par][4 * ti + r];
#pragma unroll
      for (int c = 0; c < 4; ++c) ck[c] = colbuf[par][4 * tj + c];
      const double d = sqrt(djj), rd = 1.0 / d;
      double li[4], lk[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * ti + r;
        li[r] = i > j ? ci[r] * rd : (i == j ? d : 0.0);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k = 4 * tj + c;
        lk[c] = k > j ? ck[c] * rd : 0.0;
      }
      if (low) {
        if (tj == jb) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (4 * ti + r >= j) blk[r][jc] = li[r];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) blk[r][c] = fma(-li[r], lk[c], blk[r][c]);
      }
      // publish column j + 1 (its updates from columns <= j are complete)
      constexpr int nc = (jc + 1) & 3;
      const int jn = j + 1;
      if (tj == jn / 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) colbuf[par ^ 1][4 * ti + r] = blk[r][nc];
      }
      __syncthreads();
    });
  }
  if (bad) {
    if (tid == 0) *info = k0 + bad;
    return;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = 4 * ti + r, k = 4 * tj + c;
      if (i < n && k <= i) a[(long long)i * lda + k] = blk[r][c];
    }
}

void potrf_rec(hipStream_t s, double* a, int lda, int n, int k0, int* info, double* work) {
  if (n <= CB) {
    hipLaunchKernelGGL(k_potrf_small_f64, dim3(1), dim3(256), 0, s, a, lda, n, k0, info);
    FROB_LAUNCH_CHECK();
    return;
  }
  int n1 = (n / 2 + CB - 1) / CB * CB;
  if (n1 >= n) n1 = n - CB;
  const int n2 = n - n1;
  potrf_rec(s, a, lda, n1, k0, info, work);
  // L21 = A21 L11^{-T}:  X op(T) = B with T = L11 (stored lower), op = transpose (upper)
  DOp L11{a, lda, nullptr};
  DOut A21{a + (long long)n1 * lda, lda, nullptr, nullptr};
  trsm_f64(s, true, TRI_UPPER, true, n1, n2, L11, A21, work);
  // A22 -= L21 L21^T, lower triangle only
  DOp L21{a + (long long)n1 * lda, lda, nullptr};
  DOut A22{a + (long long)n1 * lda + n1, lda, nullptr, nullptr};
  gemm_f64(s, false, true, n2, n2, n1, -1.0, L21, TRI_NONE, L21, TRI_NONE, 1.0, A22, true);
  potrf_rec(s, a + (long long)n1 * lda + n1, lda, n2, k0 + n1, info, work);
}

}  // namespace

size_t potrf_work_elems(int n) { return trsm_work_elems(n / 2 + CB); }

void potrf_f64(hipStream_t s, int n, double* a, int lda, int* info, double* work) {
  if (n <= 0) return;
  potrf_rec(s, a, lda, n, 0, info, work);
}

}  // namespace frob
