// chol_z64.hip -- complex (planar FP64) Cholesky M = L L^H (lower, row-major)
// for the complex-arithmetic baseline (Algorithm 8).  Same recursion as
// chol_f64.hip: factor M11, L21 = M21 L11^{-H}, lower half of
// M22 -= L21 L21^H, factor M22; base case of order <= 32 in LDS with a real
// positive diagonal test.
#include "common.hpp"
#include "internal.hpp"

namespace frob {

namespace {

constexpr int CZ = 32;

__global__ __launch_bounds__(256) void k_zpotrf_small(double* ar, double* ai, int lda, int n, int k0, int* info) {
  __shared__ double Sr[CZ][CZ + 1];
  __shared__ double Si[CZ][CZ + 1];
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  if (*info != 0) return;
  for (int e = tid; e < CZ * CZ; e += 256) {
    const int i = e / CZ, k = e % CZ;
    const bool ok = i < n && k <= i;
    Sr[i][k] = ok ? ar[(long long)i * lda + k] : 0.0;
    Si[i][k] = ok ? ai[(long long)i * lda + k] : 0.0;
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      const double d = Sr[j][j];  // the diagonal of a Hermitian matrix is real
      if (!(d > 0.0)) s_bad = j + 1;
      else { Sr[j][j] = sqrt(d); Si[j][j] = 0.0; }
    }
    __syncthreads();
    if (s_bad) break;
    const double ljj = Sr[j][j];
    for (int i = j + 1 + tid; i < n; i += 256) { Sr[i][j] /= ljj; Si[i][j] /= ljj; }
    __syncthreads();
    const int rem = n - j - 1;
    for (int e = tid; e < rem * rem; e += 256) {
      const int i = j + 1 + e / rem, k = j + 1 + e % rem;
      if (k <= i) {
        // M[i][k] -= L[i][j] conj(L[k][j])
        const double xr = Sr[i][j], xi = Si[i][j], yr = Sr[k][j], yi = -Si[k][j];
        Sr[i][k] -= xr * yr - xi * yi;
        Si[i][k] -= xr * yi + xi * yr;
      }
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) *info = k0 + s_bad;
    return;
  }
  for (int e = tid; e < CZ * CZ; e += 256) {
    const int i = e / CZ, k = e % CZ;
    if (i < n && k <= i) {
      ar[(long long)i * lda + k] = Sr[i][k];
      ai[(long long)i * lda + k] = Si[i][k];
    }
  }
}

void zpotrf_rec(hipStream_t s, double* ar, double* ai, int lda, int n, int k0, int* info, double* work) {
  if (n <= CZ) {
    hipLaunchKernelGGL(k_zpotrf_small, dim3(1), dim3(256), 0, s, ar, ai, lda, n, k0, info);
    FROB_LAUNCH_CHECK();
    return;
  }
  int n1 = (n / 2 + CZ - 1) / CZ * CZ;
  if (n1 >= n) n1 = n - CZ;
  const int n2 = n - n1;
  zpotrf_rec(s, ar, ai, lda, n1, k0, info, work);
  const long long o21 = (long long)n1 * lda, o22 = (long long)n1 * lda + n1;
  // L21 = M21 L11^{-H}: X op(T) = B with T = L11 (stored lower), op = conjugate transpose (upper)
  ZOp L11{ar, ai, lda, nullptr};
  ZOut M21{ar + o21, ai + o21, lda, nullptr, nullptr};
  trsm_z64(s, true, TRI_UPPER, OP_C, n1, n2, L11, M21, work);
  ZOp L21{ar + o21, ai + o21, lda, nullptr};
  ZOut M22{ar + o22, ai + o22, lda, nullptr, nullptr};
  gemm_z64(s, OP_N, OP_C, n2, n2, n1, -1.0, L21, TRI_NONE, L21, TRI_NONE, 1.0, M22, true);
  zpotrf_rec(s, ar + o22, ai + o22, lda, n2, k0 + n1, info, work);
}

}  // namespace

size_t potrf_z_work_elems(int n) { return trsm_z_work_elems(n / 2 + CZ); }

void potrf_z64(hipStream_t s, int n, double* re, double* im, int lda, int* info, double* work) {
  if (n <= 0) return;
  zpotrf_rec(s, re, im, lda, n, 0, info, work);
}

}  // namespace frob
