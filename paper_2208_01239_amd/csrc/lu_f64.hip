// lu_f64.hip -- LU factorization with partial pivoting (GEPP) in FP64.
//
// Recursive column splitting: factor the left half, solve U12 = L11^{-1} A12,
// update A22 -= L21 U12 with one matrix-core GEMM, factor the right half.  The
// recursion stops at a "leaf" panel narrow enough to live in the registers of
// one 1024-thread workgroup (rows-per-thread x columns = 32 doubles per
// thread), where the pivot search is a wave64 shuffle reduction followed by a
// 16-entry LDS reduction, with the lowest row index winning ties.
//
// Pivoting never moves data: rows are addressed through the index array perm
// (logical row i of P A lives in physical row perm[i]), so a row interchange
// is a swap of two integers and the stored multipliers of earlier columns
// follow automatically.  An exactly-zero pivot column is recorded in *info
// (1-based, first occurrence) and factoring continues, as LAPACK does.
#include <climits>

#include "common.hpp"
#include "internal.hpp"

namespace frob {

namespace {

constexpr int LEAF_THREADS = 1024;

template <int R, int W>
__global__ __launch_bounds__(LEAF_THREADS) void k_lu_leaf_f64(double* __restrict__ a, int lda, int* __restrict__ perm,
                                                              int k0, int mm, int nc, int* info) {
  __shared__ double s_rv[LEAF_THREADS / 64];
  __shared__ int s_ri[LEAF_THREADS / 64];
  __shared__ double s_prow[W];
  __shared__ double s_jrow[W];
  __shared__ int s_pph, s_jph;

  const int t = threadIdx.x;
  double v[R][W];
  int ph[R];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int q = t + s * LEAF_THREADS;
    ph[s] = -1;
#pragma unroll
    for (int c = 0; c < W; ++c) v[s][c] = 0.0;
    if (q < mm) {
      ph[s] = perm[k0 + q];
      const double* row = a + (long long)ph[s] * lda + k0;
#pragma unroll
      for (int c = 0; c < W; ++c)
        if (c < nc) v[s][c] = row[c];
    }
  }

  int first_zero = 0;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    if (j >= nc) continue;  // uniform: every thread skips the same columns
    // local candidate: largest |v| in column j among own rows q >= j
    double best = -1.0;
    int bq = INT_MAX;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int q = t + s * LEAF_THREADS;
      if (q >= j && q < mm) {
        const double x = fabs(v[s][j]);
        if (x > best) { best = x; bq = q; }
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int oq = __shfl_xor(bq, off);
      if (ob > best || (ob == best && oq < bq)) { best = ob; bq = oq; }
    }
    if ((t & 63) == 0) { s_rv[t >> 6] = best; s_ri[t >> 6] = bq; }
    __syncthreads();
    best = s_rv[0];
    bq = s_ri[0];
#pragma unroll
    for (int w = 1; w < LEAF_THREADS / 64; ++w) {
      const double ob = s_rv[w];
      const int oq = s_ri[w];
      if (ob > best || (ob == best && oq < bq)) { best = ob; bq = oq; }
    }
    // A column of NaNs yields no candidate (NaN compares false): keep row j so
    // the pivot row is always one of the panel's rows and NaN propagates.
    const int p = (best >= 0.0 && bq >= j && bq < mm) ? bq : j;
    // publish the pivot row and row j
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int q = t + s * LEAF_THREADS;
      if (q == p) {
#pragma unroll
        for (int c = 0; c < W; ++c) s_prow[c] = v[s][c];
        s_pph = ph[s];
      }
      if (q == j) {
#pragma unroll
        for (int c = 0; c < W; ++c) s_jrow[c] = v[s][c];
        s_jph = ph[s];
      }
    }
    __syncthreads();
    if (p != j) {
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const int q = t + s * LEAF_THREADS;
        if (q == j) {
#pragma unroll
          for (int c = 0; c < W; ++c) v[s][c] = s_prow[c];
          ph[s] = s_pph;
        } else if (q == p) {
#pragma unroll
          for (int c = 0; c < W; ++c) v[s][c] = s_jrow[c];
          ph[s] = s_jph;
        }
      }
    }
    const double piv = s_prow[j];
    if (piv == 0.0) {
      if (!first_zero) first_zero = k0 + j + 1;
    } else {
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const int q = t + s * LEAF_THREADS;
        if (q > j && q < mm) {
          const double l = v[s][j] / piv;
          v[s][j] = l;
#pragma unroll
          for (int c = 0; c < W; ++c)
            if (c > j) v[s][c] -= l * s_prow[c];
        }
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int q = t + s * LEAF_THREADS;
    if (q < mm) {
      double* row = a + (long long)ph[s] * lda + k0;
#pragma unroll
      for (int c = 0; c < W; ++c)
        if (c < nc) row[c] = v[s][c];
      perm[k0 + q] = ph[s];
    }
  }
  if (t == 0 && first_zero && *info == 0) *info = first_zero;
}

// widest leaf for a panel with mm rows
inline int leaf_width(int mm) {
  const int R = ceil_div(mm, LEAF_THREADS);
  if (R <= 2) return 16;
  if (R <= 4) return 8;
  if (R <= 8) return 4;
  if (R <= 16) return 2;
  return 0;
}

void launch_leaf(hipStream_t s, double* a, int lda, int* perm, int k0, int mm, int nc, int* info) {
  const int R = ceil_div(mm, LEAF_THREADS);
  dim3 g(1), b(LEAF_THREADS);
  if (R <= 1) hipLaunchKernelGGL((k_lu_leaf_f64<1, 16>), g, b, 0, s, a, lda, perm, k0, mm, nc, info);
  else if (R <= 2) hipLaunchKernelGGL((k_lu_leaf_f64<2, 16>), g, b, 0, s, a, lda, perm, k0, mm, nc, info);
  else if (R <= 4) hipLaunchKernelGGL((k_lu_leaf_f64<4, 8>), g, b, 0, s, a, lda, perm, k0, mm, nc, info);
  else if (R <= 8) hipLaunchKernelGGL((k_lu_leaf_f64<8, 4>), g, b, 0, s, a, lda, perm, k0, mm, nc, info);
  else if (R <= 16) hipLaunchKernelGGL((k_lu_leaf_f64<16, 2>), g, b, 0, s, a, lda, perm, k0, mm, nc, info);
  else throw std::runtime_error("getrf_f64: matrix order above 16384 is not supported");
  FROB_LAUNCH_CHECK();
}

// factor columns [k0, k0 + n) over logical rows [k0, m)
void getrf_rec(hipStream_t s, double* a, int lda, int* perm, int k0, int m, int n, int* info) {
  const int mm = m - k0;
  const int wmax = leaf_width(mm);
  if (n <= wmax) {
    launch_leaf(s, a, lda, perm, k0, mm, n, info);
    return;
  }
  int n1 = (n / 2 + 7) / 8 * 8;
  if (n1 >= n) n1 = n / 2;
  const int n2 = n - n1;
  getrf_rec(s, a, lda, perm, k0, m, n1, info);
  // U12 = L11^{-1} A12 (unit lower), rows through perm
  DOp L11{a + k0, lda, perm + k0};
  DOut A12{a + k0 + n1, lda, perm + k0, nullptr};
  trsm_f64(s, false, TRI_LOWER_UNIT, false, n1, n2, L11, A12);
  // A22 -= L21 U12
  DOp L21{a + k0, lda, perm + k0 + n1};
  DOp U12{a + k0 + n1, lda, perm + k0};
  DOut A22{a + k0 + n1, lda, perm + k0 + n1, nullptr};
  gemm_f64(s, false, false, m - k0 - n1, n2, n1, -1.0, L21, TRI_NONE, U12, TRI_NONE, 1.0, A22);
  getrf_rec(s, a, lda, perm, k0 + n1, m, n2, info);
}

}  // namespace

void getrf_f64(hipStream_t s, int n, double* a, int lda, int* perm, int* info) {
  if (n <= 0) return;
  iota_i32(s, n, perm);
  getrf_rec(s, a, lda, perm, 0, n, n, info);
}

}  // namespace frob
