// chol_f64.hip -- Cholesky factorization A = L L^T (lower, row-major) in FP64.
//
// Recursive: factor A11, L21 = A21 L11^{-T} (right triangular solve), lower
// half of A22 -= L21 L21^T (one GEMM writing only the lower triangle), factor
// A22.  The base case keeps a diagonal block of order <= 64 in LDS and runs
// the right-looking algorithm there in FP64 (square root and pivot test on
// the diagonal).  The first non-positive (or NaN) pivot stops the
// factorization and is recorded in *info (1-based).
#include "common.hpp"
#include "internal.hpp"

namespace frob {

namespace {

constexpr int CB = 64;

__global__ __launch_bounds__(256) void k_potrf_small_f64(double* a, int lda, int n, int k0, int* info) {
  __shared__ double S[CB][CB + 1];
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  if (*info != 0) return;  // an earlier block already failed
  for (int e = tid; e < CB * CB; e += 256) {
    const int i = e / CB, k = e % CB;
    S[i][k] = (i < n && k <= i) ? a[(long long)i * lda + k] : 0.0;
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      const double d = S[j][j];
      if (!(d > 0.0)) s_bad = j + 1;
      else S[j][j] = sqrt(d);
    }
    __syncthreads();
    if (s_bad) break;
    const double ljj = S[j][j];
    for (int i = j + 1 + tid; i < n; i += 256) S[i][j] = S[i][j] / ljj;
    __syncthreads();
    const int rem = n - j - 1;
    for (int e = tid; e < rem * rem; e += 256) {
      const int i = j + 1 + e / rem, k = j + 1 + e % rem;
      if (k <= i) S[i][k] -= S[i][j] * S[k][j];
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) *info = k0 + s_bad;
    return;
  }
  for (int e = tid; e < CB * CB; e += 256) {
    const int i = e / CB, k = e % CB;
    if (i < n && k <= i) a[(long long)i * lda + k] = S[i][k];
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
