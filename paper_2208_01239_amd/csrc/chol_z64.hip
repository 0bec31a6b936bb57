// chol_z64.hip -- complex (planar FP64) Cholesky M = L L^H (lower, row-major)
// for the complex-arithmetic baseline (Algorithm 8).  Same recursion as
// chol_f64.hip: factor M11, L21 = M21 L11^{-H}, lower half of
// M22 -= L21 L21^H, factor M22; base case of order <= 32 in registers with a
// real positive diagonal test.
#include "common.hpp"
#include "internal.hpp"
#include "tri_dev.hpp"

namespace frob {

namespace {

constexpr int CZ = 32;

// Base case, order n <= 32, right-looking with the matrix in registers (the
// design of the real base case in chol_f64.hip): one wave, thread (ti, tj)
// of an 8 x 8 grid owns the 4 x 4 complex block at rows 4 ti, columns 4 tj;
// per column the column is read from a parity-double-buffered LDS copy
// (unconditionally, one LDS round trip), scaled by the reciprocal of the
// (real) pivot's square root, the block is updated with
// M(i, k) -= L(i, j) conj(L(k, j)), and column j + 1 is published.
__global__ __launch_bounds__(64) void k_zpotrf_small(double* ar, double* ai, int lda, int n, int k0, int* info) {
  __shared__ double cbr[2][CZ], cbi[2][CZ];
  const int tid = threadIdx.x;
  if (*info != 0) return;  // an earlier block already failed (uniform)
  const int ti = tid >> 3, tj = tid & 7;
  const bool low = ti >= tj;
  double br[4][4], bi[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = 4 * ti + r, k = 4 * tj + c;
      const bool in = i < n && k <= i;
      const long long o = (long long)min(i, n - 1) * lda + min(k, n - 1);
      br[r][c] = in ? ar[o] : 0.0;
      bi[r][c] = in ? ai[o] : 0.0;
    }
  if (tj == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      cbr[0][4 * ti + r] = br[r][0];
      cbi[0][4 * ti + r] = bi[r][0];
    }
  }
  __syncthreads();
  int bad = 0;
  for (int jb = 0; jb < CZ / 4 && !bad; ++jb) {
    StaticFor<0, 4>::run([&](auto jcc) {
      constexpr int jc = decltype(jcc)::value;
      const int j = 4 * jb + jc;
      if (bad || j >= n) return;  // uniform
      const int par = j & 1;
      const double djj = cbr[par][j];   // the diagonal of a Hermitian matrix is real
      double cir[4], cii[4], ckr[4], cki[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        cir[r] = cbr[par][4 * ti + r];
        cii[r] = cbi[par][4 * ti + r];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        ckr[c] = cbr[par][4 * tj + c];
        cki[c] = cbi[par][4 * tj + c];
      }
      if (!(djj > 0.0)) {
        bad = j + 1;
        return;
      }
      const double d = sqrt(djj), rd = 1.0 / d;
      double lir[4], lii[4], lkr[4], lki[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * ti + r;
        lir[r] = i > j ? cir[r] * rd : (i == j ? d : 0.0);
        lii[r] = i > j ? cii[r] * rd : 0.0;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k = 4 * tj + c;
        lkr[c] = k > j ? ckr[c] * rd : 0.0;
        lki[c] = k > j ? cki[c] * rd : 0.0;
      }
      if (low) {
        if (tj == jb) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (4 * ti + r >= j) {
              br[r][jc] = lir[r];
              bi[r][jc] = lii[r];
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            // -= (lir + i lii)(lkr - i lki)
            br[r][c] = fma(-lii[r], lki[c], fma(-lir[r], lkr[c], br[r][c]));
            bi[r][c] = fma(lir[r], lki[c], fma(-lii[r], lkr[c], bi[r][c]));
          }
      }
      constexpr int nc = (jc + 1) & 3;
      if (tj == (j + 1) / 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          cbr[par ^ 1][4 * ti + r] = br[r][nc];
          cbi[par ^ 1][4 * ti + r] = bi[r][nc];
        }
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
      if (i < n && k <= i) {
        ar[(long long)i * lda + k] = br[r][c];
        ai[(long long)i * lda + k] = bi[r][c];
      }
    }
}

void zpotrf_rec(hipStream_t s, double* ar, double* ai, int lda, int n, int k0, int* info, double* work) {
  if (n <= CZ) {
    hipLaunchKernelGGL(k_zpotrf_small, dim3(1), dim3(64), 0, s, ar, ai, lda, n, k0, info);
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
