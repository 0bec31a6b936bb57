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
#include "devutil.hpp"

namespace frob {

namespace {

constexpr int LEAF_THREADS = 1024;

// One workgroup factors an mm x nc panel (nc <= W) held in registers: thread t
// owns logical rows t, t + 1024, ... .  The panel moves between HBM and the
// registers through an LDS stage in rounds of SROWS rows, with all global
// loads of a round issued before any is consumed (the rows are scattered by
// the pivot indirection, so these loads are latency-bound).  Per column: every
// wave reduces its candidates and publishes the winning row (value, index,
// physical row, W entries) to a parity-double-buffered LDS slot, the owner of
// row j publishes row j, one barrier, then every thread picks the global
// winner from the slots, swaps, and updates its rows.
//
// With n2 > 0 the kernel also applies its factorization to the n2 columns to
// the right of the panel (the sibling panel of a bottom recursion node):
// U12 = L11^{-1} A12 by substitution in wave 0, then A22 -= L21 U12 with L21
// still in registers.  That replaces a triangular-solve launch and a GEMM
// launch per bottom node.
constexpr int STAGE = 8192;  // doubles in the LDS stage (64 KiB)

template <int R, int W>
__global__ __launch_bounds__(LEAF_THREADS) void k_lu_leaf_f64(double* __restrict__ a, int lda, int* __restrict__ perm,
                                                              int k0, int mm, int nc, int n2, int* info) {
  constexpr int NW = LEAF_THREADS / 64;
  constexpr int SROWS = STAGE / W;                       // rows per staging round
  constexpr int PER = STAGE / LEAF_THREADS;              // staged elements per thread per round
  static_assert(STAGE % LEAF_THREADS == 0 && STAGE % W == 0, "stage shape");
  __shared__ double stage[STAGE];
  __shared__ int s_ph[SROWS];
  __shared__ double s_cv[2][NW];
  __shared__ int s_ci[2][NW];
  __shared__ int s_cph[2][NW];
  __shared__ double s_crow[2][NW][W];
  __shared__ double s_jrow[2][W];
  __shared__ int s_jph[2];
  __shared__ double s_u[W][W];

  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  double v[R][W];
  int ph[R];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    ph[s] = -1;
#pragma unroll
    for (int c = 0; c < W; ++c) v[s][c] = 0.0;
  }

  // ---- load the panel (columns k0 .. k0 + nc) through the stage ----
  for (int r0 = 0; r0 < mm; r0 += SROWS) {
    const int nrow = min(SROWS, mm - r0);
    int pr[PER];
    double x[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + i * LEAF_THREADS, r = e / W;
      pr[i] = r < nrow ? perm[k0 + r0 + r] : 0;
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + i * LEAF_THREADS, r = e / W, c = e % W;
      x[i] = (r < nrow && c < nc) ? a[(long long)pr[i] * lda + k0 + c] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + i * LEAF_THREADS;
      stage[e] = x[i];
      if (e % W == 0 && e / W < nrow) s_ph[e / W] = pr[i];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int q = t + s * LEAF_THREADS;
      if (q >= r0 && q < r0 + nrow) {
        ph[s] = s_ph[q - r0];
#pragma unroll
        for (int c = 0; c < W; ++c) v[s][c] = stage[(q - r0) * W + c];
      }
    }
    __syncthreads();
  }

  // ---- factor ----
  int first_zero = 0;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    if (j >= nc) continue;  // uniform
    const int par = j & 1;
    double best = -1.0;
    int bq = INT_MAX;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int q = t + s * LEAF_THREADS;
      const double xv = fabs(v[s][j]);
      const bool ok = q >= j && q < mm && xv > best;
      best = ok ? xv : best;
      bq = ok ? q : bq;
    }
    double wbest;
    int wq;
    const int wl = wave_argmax(best, bq, wbest, wq);
    if (lane == wl) {
      const int s = (wq - t) / LEAF_THREADS;
#pragma unroll
      for (int ss = 0; ss < R; ++ss)
        if (ss == s) {
#pragma unroll
          for (int c = 0; c < W; ++c) s_crow[par][wv][c] = v[ss][c];
          s_cph[par][wv] = ph[ss];
        }
    }
    if (lane == 0) { s_cv[par][wv] = wbest; s_ci[par][wv] = wq; }
    if ((j & (LEAF_THREADS - 1)) == t) {
#pragma unroll
      for (int c = 0; c < W; ++c) s_jrow[par][c] = v[j / LEAF_THREADS][c];
      s_jph[par] = ph[j / LEAF_THREADS];
    }
    __syncthreads();
    double gb = -1.0;
    int gq = INT_MAX, gw = -1;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const double cv = s_cv[par][w];
      const int ci = s_ci[par][w];
      const bool ok = ci != INT_MAX && (cv > gb || (cv == gb && ci < gq));
      gb = ok ? cv : gb;
      gq = ok ? ci : gq;
      gw = ok ? w : gw;
    }
    const bool have = gw >= 0;               // false only for an all-NaN column
    const int p = have ? gq : j;
    double prow[W];
#pragma unroll
    for (int c = 0; c < W; ++c) prow[c] = have ? s_crow[par][gw][c] : s_jrow[par][c];
    const int pph = have ? s_cph[par][gw] : s_jph[par];
    if (p != j) {
      // row j takes the pivot row, row p takes the old row j
      if ((j & (LEAF_THREADS - 1)) == t) {
#pragma unroll
        for (int c = 0; c < W; ++c) v[j / LEAF_THREADS][c] = prow[c];
        ph[j / LEAF_THREADS] = pph;
      }
      if ((p & (LEAF_THREADS - 1)) == t) {
#pragma unroll
        for (int ss = 0; ss < R; ++ss)
          if (ss == p / LEAF_THREADS) {
#pragma unroll
            for (int c = 0; c < W; ++c) v[ss][c] = s_jrow[par][c];
            ph[ss] = s_jph[par];
          }
      }
    }
    const double piv = prow[j];
    if (piv == 0.0) {
      if (!first_zero) first_zero = k0 + j + 1;
    } else {
      // scale by the reciprocal unless it would overflow (as LAPACK's getf2 does)
      const bool recip = fabs(piv) >= 2.2250738585072014e-308;
      const double rp = 1.0 / piv;
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const int q = t + s * LEAF_THREADS;
        const bool below = q > j && q < mm;
        const double l = below ? (recip ? v[s][j] * rp : v[s][j] / piv) : 0.0;
        if (below) v[s][j] = l;
#pragma unroll
        for (int c = 0; c < W; ++c)
          if (c > j) v[s][c] -= l * prow[c];
      }
    }
  }
  if (t == 0 && first_zero && *info == 0) *info = first_zero;

  // ---- store the panel (and the new row order) through the stage ----
  for (int r0 = 0; r0 < mm; r0 += SROWS) {
    const int nrow = min(SROWS, mm - r0);
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int q = t + s * LEAF_THREADS;
      if (q >= r0 && q < r0 + nrow) {
        s_ph[q - r0] = ph[s];
        perm[k0 + q] = ph[s];
#pragma unroll
        for (int c = 0; c < W; ++c) stage[(q - r0) * W + c] = v[s][c];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + i * LEAF_THREADS, r = e / W, c = e % W;
      if (r < nrow && c < nc) a[(long long)s_ph[r] * lda + k0 + c] = stage[e];
    }
    __syncthreads();
  }

  if (n2 <= 0) return;
  // ---- sibling update: columns k0 + nc .. k0 + nc + n2 ----
  const int cs = k0 + nc;
  for (int r0 = 0; r0 < mm; r0 += SROWS) {
    const int nrow = min(SROWS, mm - r0);
    // physical rows of this round (final order) and the sibling block
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int q = t + s * LEAF_THREADS;
      if (q >= r0 && q < r0 + nrow) s_ph[q - r0] = ph[s];
    }
    __syncthreads();
    double x[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + i * LEAF_THREADS, r = e / W, c = e % W;
      x[i] = (r < nrow && c < n2) ? a[(long long)s_ph[r] * lda + cs + c] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) stage[t + i * LEAF_THREADS] = x[i];
    __syncthreads();
    if (r0 == 0 && t < 64) {
      // U12 = L11^{-1} A12: top rows q < nc are lanes q of wave 0 (s = 0)
#pragma unroll
      for (int k = 0; k < W; ++k) {
        if (k < nc) {
          if (t > k && t < nc) {
            const double l = v[0][k];
#pragma unroll
            for (int c = 0; c < W; ++c) stage[t * W + c] -= l * stage[k * W + c];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      }
      for (int e = t; e < W * W; e += 64) s_u[e / W][e % W] = (e / W < nc) ? stage[e] : 0.0;
    }
    __syncthreads();
    // A22 -= L21 U12 on the staged rows below the top nc rows
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int q = t + s * LEAF_THREADS;
      if (q >= r0 && q < r0 + nrow && q >= nc) {
#pragma unroll
        for (int c = 0; c < W; ++c) {
          double acc = stage[(q - r0) * W + c];
#pragma unroll
          for (int k = 0; k < W; ++k)
            if (k < nc) acc -= v[s][k] * s_u[k][c];
          stage[(q - r0) * W + c] = acc;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + i * LEAF_THREADS, r = e / W, c = e % W;
      if (r < nrow && c < n2) a[(long long)s_ph[r] * lda + cs + c] = stage[e];
    }
    __syncthreads();
  }
}

// widest leaf for a panel with mm rows
inline int leaf_width(int mm) {
  const int R = ceil_div(mm, LEAF_THREADS);
  if (R <= 1) return 16;
  if (R <= 2) return 8;
  if (R <= 4) return 8;
  if (R <= 8) return 4;
  if (R <= 16) return 2;
  return 0;
}

void launch_leaf(hipStream_t s, double* a, int lda, int* perm, int k0, int mm, int nc, int n2, int* info) {
  const int R = ceil_div(mm, LEAF_THREADS);
  if (nc > leaf_width(mm) || n2 > leaf_width(mm)) throw std::runtime_error("getrf_f64: leaf wider than its template");
  dim3 g(1), b(LEAF_THREADS);
  if (R <= 1) hipLaunchKernelGGL((k_lu_leaf_f64<1, 16>), g, b, 0, s, a, lda, perm, k0, mm, nc, n2, info);
  else if (R <= 2) hipLaunchKernelGGL((k_lu_leaf_f64<2, 8>), g, b, 0, s, a, lda, perm, k0, mm, nc, n2, info);
  else if (R <= 4) hipLaunchKernelGGL((k_lu_leaf_f64<4, 8>), g, b, 0, s, a, lda, perm, k0, mm, nc, n2, info);
  else if (R <= 8) hipLaunchKernelGGL((k_lu_leaf_f64<8, 4>), g, b, 0, s, a, lda, perm, k0, mm, nc, n2, info);
  else if (R <= 16) hipLaunchKernelGGL((k_lu_leaf_f64<16, 2>), g, b, 0, s, a, lda, perm, k0, mm, nc, n2, info);
  else throw std::runtime_error("getrf_f64: matrix order above 16384 is not supported");
  FROB_LAUNCH_CHECK();
}

// factor columns [k0, k0 + n) over logical rows [k0, m)
void getrf_rec(hipStream_t s, double* a, int lda, int* perm, int k0, int m, int n, int* info, double* work) {
  const int mm = m - k0;
  const int wmax = leaf_width(mm);
  if (n <= wmax) {
    launch_leaf(s, a, lda, perm, k0, mm, n, 0, info);
    return;
  }
  int n1 = (n / 2 + 7) / 8 * 8;
  if (n1 >= n) n1 = n / 2;
  const int n2 = n - n1;
  if (n1 <= wmax && n2 <= wmax) {
    // bottom node: the left leaf also updates its sibling's columns
    launch_leaf(s, a, lda, perm, k0, mm, n1, n2, info);
    getrf_rec(s, a, lda, perm, k0 + n1, m, n2, info, work);
    return;
  }
  getrf_rec(s, a, lda, perm, k0, m, n1, info, work);
  // U12 = L11^{-1} A12 (unit lower), rows through perm
  DOp L11{a + k0, lda, perm + k0};
  DOut A12{a + k0 + n1, lda, perm + k0, nullptr};
  trsm_f64(s, false, TRI_LOWER_UNIT, false, n1, n2, L11, A12, work);
  // A22 -= L21 U12
  DOp L21{a + k0, lda, perm + k0 + n1};
  DOp U12{a + k0 + n1, lda, perm + k0};
  DOut A22{a + k0 + n1, lda, perm + k0 + n1, nullptr};
  gemm_f64(s, false, false, m - k0 - n1, n2, n1, -1.0, L21, TRI_NONE, U12, TRI_NONE, 1.0, A22);
  getrf_rec(s, a, lda, perm, k0 + n1, m, n2, info, work);
}

}  // namespace

size_t getrf_work_elems(int n) { return trsm_work_elems(n / 2 + 8); }

void getrf_f64(hipStream_t s, int n, double* a, int lda, int* perm, int* info, double* work) {
  if (n <= 0) return;
  iota_i32(s, n, perm);
  getrf_rec(s, a, lda, perm, 0, n, n, info, work);
}

}  // namespace frob
