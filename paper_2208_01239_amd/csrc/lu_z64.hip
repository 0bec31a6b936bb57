// lu_z64.hip -- complex (planar FP64) LU with partial pivoting for the
// complex-arithmetic baseline (Algorithm 4).  Same design as lu_f64.hip:
// recursive column splitting, register-resident leaf panels in one
// 1024-thread workgroup, pivoting through the row-index array perm, staged
// panel I/O, fused sibling update at bottom nodes.  The pivot measure is
// |Re| + |Im| (LAPACK's izamax convention); ties go to the lowest row.
#include "common.hpp"
#include "devutil.hpp"
#include "internal.hpp"

namespace frob {

namespace {

constexpr int ZLT = 1024;
constexpr int ZSTAGE = 4096;  // doubles per plane in the LDS stage

struct zc {
  double r, i;
};
__device__ __forceinline__ zc zmul(zc a, zc b) { return zc{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
// 1 / z by Smith's scaling
__device__ __forceinline__ zc zrecip(zc z) {
  if (fabs(z.r) >= fabs(z.i)) {
    const double t = z.i / z.r, d = z.r + z.i * t;
    return zc{1.0 / d, -t / d};
  }
  const double t = z.r / z.i, d = z.r * t + z.i;
  return zc{t / d, -1.0 / d};
}

template <int R, int W>
__global__ __launch_bounds__(ZLT) void k_lu_leaf_z64(double* __restrict__ ar, double* __restrict__ ai, int lda,
                                                     int* __restrict__ perm, int k0, int mm, int nc, int n2,
                                                     int* info) {
  constexpr int NW = ZLT / 64;
  constexpr int SROWS = ZSTAGE / W;
  constexpr int PER = ZSTAGE / ZLT;
  static_assert(ZSTAGE % ZLT == 0 && ZSTAGE % W == 0, "stage shape");
  __shared__ double sr_[ZSTAGE];
  __shared__ double si_[ZSTAGE];
  __shared__ int s_ph[SROWS];
  __shared__ double s_cv[2][NW];
  __shared__ int s_ci[2][NW];
  __shared__ int s_cph[2][NW];
  __shared__ double s_crr[2][NW][W];
  __shared__ double s_cri[2][NW][W];
  __shared__ double s_jr[2][W];
  __shared__ double s_ji[2][W];
  __shared__ int s_jph[2];
  __shared__ double s_ur[W][W];
  __shared__ double s_ui[W][W];

  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  double vr[R][W], vi[R][W];
  int ph[R];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    ph[s] = -1;
#pragma unroll
    for (int c = 0; c < W; ++c) { vr[s][c] = 0.0; vi[s][c] = 0.0; }
  }

  for (int r0 = 0; r0 < mm; r0 += SROWS) {
    const int nrow = min(SROWS, mm - r0);
    int pr[PER];
    double xr[PER], xi[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + i * ZLT, r = e / W;
      pr[i] = r < nrow ? perm[k0 + r0 + r] : 0;
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + i * ZLT, r = e / W, c = e % W;
      const bool ok = r < nrow && c < nc;
      const long long off = (long long)pr[i] * lda + k0 + c;
      xr[i] = ok ? ar[off] : 0.0;
      xi[i] = ok ? ai[off] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + i * ZLT;
      sr_[e] = xr[i];
      si_[e] = xi[i];
      if (e % W == 0 && e / W < nrow) s_ph[e / W] = pr[i];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int q = t + s * ZLT;
      if (q >= r0 && q < r0 + nrow) {
        ph[s] = s_ph[q - r0];
#pragma unroll
        for (int c = 0; c < W; ++c) { vr[s][c] = sr_[(q - r0) * W + c]; vi[s][c] = si_[(q - r0) * W + c]; }
      }
    }
    __syncthreads();
  }

  int first_zero = 0;
#pragma unroll
  for (int j = 0; j < W; ++j) {
    if (j >= nc) continue;
    const int par = j & 1;
    double best = -1.0;
    int bq = INT_MAX;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int q = t + s * ZLT;
      const double xv = fabs(vr[s][j]) + fabs(vi[s][j]);
      const bool ok = q >= j && q < mm && xv > best;
      best = ok ? xv : best;
      bq = ok ? q : bq;
    }
    double wbest;
    int wq;
    const int wl = wave_argmax(best, bq, wbest, wq);
    if (lane == wl) {
      const int s = (wq - t) / ZLT;
#pragma unroll
      for (int ss = 0; ss < R; ++ss)
        if (ss == s) {
#pragma unroll
          for (int c = 0; c < W; ++c) { s_crr[par][wv][c] = vr[ss][c]; s_cri[par][wv][c] = vi[ss][c]; }
          s_cph[par][wv] = ph[ss];
        }
    }
    if (lane == 0) { s_cv[par][wv] = wbest; s_ci[par][wv] = wq; }
    if ((j & (ZLT - 1)) == t) {
#pragma unroll
      for (int c = 0; c < W; ++c) { s_jr[par][c] = vr[j / ZLT][c]; s_ji[par][c] = vi[j / ZLT][c]; }
      s_jph[par] = ph[j / ZLT];
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
    const bool have = gw >= 0;
    const int p = have ? gq : j;
    double pwr[W], pwi[W];
#pragma unroll
    for (int c = 0; c < W; ++c) {
      pwr[c] = have ? s_crr[par][gw][c] : s_jr[par][c];
      pwi[c] = have ? s_cri[par][gw][c] : s_ji[par][c];
    }
    const int pph = have ? s_cph[par][gw] : s_jph[par];
    if (p != j) {
      if ((j & (ZLT - 1)) == t) {
#pragma unroll
        for (int c = 0; c < W; ++c) { vr[j / ZLT][c] = pwr[c]; vi[j / ZLT][c] = pwi[c]; }
        ph[j / ZLT] = pph;
      }
      if ((p & (ZLT - 1)) == t) {
#pragma unroll
        for (int ss = 0; ss < R; ++ss)
          if (ss == p / ZLT) {
#pragma unroll
            for (int c = 0; c < W; ++c) { vr[ss][c] = s_jr[par][c]; vi[ss][c] = s_ji[par][c]; }
            ph[ss] = s_jph[par];
          }
      }
    }
    const zc piv{pwr[j], pwi[j]};
    if (piv.r == 0.0 && piv.i == 0.0) {
      if (!first_zero) first_zero = k0 + j + 1;
    } else {
      const zc rp = zrecip(piv);
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const int q = t + s * ZLT;
        const bool below = q > j && q < mm;
        zc l = zmul(zc{vr[s][j], vi[s][j]}, rp);
        if (!below) l = zc{0.0, 0.0};
        if (below) { vr[s][j] = l.r; vi[s][j] = l.i; }
#pragma unroll
        for (int c = 0; c < W; ++c)
          if (c > j) {
            vr[s][c] -= l.r * pwr[c] - l.i * pwi[c];
            vi[s][c] -= l.r * pwi[c] + l.i * pwr[c];
          }
      }
    }
  }
  if (t == 0 && first_zero && *info == 0) *info = first_zero;

  for (int r0 = 0; r0 < mm; r0 += SROWS) {
    const int nrow = min(SROWS, mm - r0);
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int q = t + s * ZLT;
      if (q >= r0 && q < r0 + nrow) {
        s_ph[q - r0] = ph[s];
        perm[k0 + q] = ph[s];
#pragma unroll
        for (int c = 0; c < W; ++c) { sr_[(q - r0) * W + c] = vr[s][c]; si_[(q - r0) * W + c] = vi[s][c]; }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + i * ZLT, r = e / W, c = e % W;
      if (r < nrow && c < nc) {
        const long long off = (long long)s_ph[r] * lda + k0 + c;
        ar[off] = sr_[e];
        ai[off] = si_[e];
      }
    }
    __syncthreads();
  }

  if (n2 <= 0) return;
  const int cs = k0 + nc;
  for (int r0 = 0; r0 < mm; r0 += SROWS) {
    const int nrow = min(SROWS, mm - r0);
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int q = t + s * ZLT;
      if (q >= r0 && q < r0 + nrow) s_ph[q - r0] = ph[s];
    }
    __syncthreads();
    double xr[PER], xi[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + i * ZLT, r = e / W, c = e % W;
      const bool ok = r < nrow && c < n2;
      const long long off = ok ? (long long)s_ph[r] * lda + cs + c : 0;
      xr[i] = ok ? ar[off] : 0.0;
      xi[i] = ok ? ai[off] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) { sr_[t + i * ZLT] = xr[i]; si_[t + i * ZLT] = xi[i]; }
    __syncthreads();
    if (r0 == 0 && t < 64) {
#pragma unroll
      for (int k = 0; k < W; ++k) {
        if (k < nc) {
          if (t > k && t < nc) {
            const double lr = vr[0][k], li = vi[0][k];
#pragma unroll
            for (int c = 0; c < W; ++c) {
              const double ur = sr_[k * W + c], ui = si_[k * W + c];
              sr_[t * W + c] -= lr * ur - li * ui;
              si_[t * W + c] -= lr * ui + li * ur;
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      }
      for (int e = t; e < W * W; e += 64) {
        const bool ok = e / W < nc;
        s_ur[e / W][e % W] = ok ? sr_[e] : 0.0;
        s_ui[e / W][e % W] = ok ? si_[e] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int q = t + s * ZLT;
      if (q >= r0 && q < r0 + nrow && q >= nc) {
#pragma unroll
        for (int c = 0; c < W; ++c) {
          double accr = sr_[(q - r0) * W + c], acci = si_[(q - r0) * W + c];
#pragma unroll
          for (int k = 0; k < W; ++k)
            if (k < nc) {
              accr -= vr[s][k] * s_ur[k][c] - vi[s][k] * s_ui[k][c];
              acci -= vr[s][k] * s_ui[k][c] + vi[s][k] * s_ur[k][c];
            }
          sr_[(q - r0) * W + c] = accr;
          si_[(q - r0) * W + c] = acci;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + i * ZLT, r = e / W, c = e % W;
      if (r < nrow && c < n2) {
        const long long off = (long long)s_ph[r] * lda + cs + c;
        ar[off] = sr_[e];
        ai[off] = si_[e];
      }
    }
    __syncthreads();
  }
}

inline int zleaf_width(int mm) {
  const int R = ceil_div(mm, ZLT);
  if (R <= 2) return 8;
  if (R <= 4) return 4;
  if (R <= 8) return 2;
  if (R <= 16) return 1;
  return 0;
}

void zlaunch_leaf(hipStream_t s, double* ar, double* ai, int lda, int* perm, int k0, int mm, int nc, int n2,
                  int* info) {
  const int R = ceil_div(mm, ZLT);
  if (nc > zleaf_width(mm) || n2 > zleaf_width(mm)) throw std::runtime_error("getrf_z64: leaf wider than template");
  dim3 g(1), b(ZLT);
  if (R <= 1) hipLaunchKernelGGL((k_lu_leaf_z64<1, 8>), g, b, 0, s, ar, ai, lda, perm, k0, mm, nc, n2, info);
  else if (R <= 2) hipLaunchKernelGGL((k_lu_leaf_z64<2, 8>), g, b, 0, s, ar, ai, lda, perm, k0, mm, nc, n2, info);
  else if (R <= 4) hipLaunchKernelGGL((k_lu_leaf_z64<4, 4>), g, b, 0, s, ar, ai, lda, perm, k0, mm, nc, n2, info);
  else if (R <= 8) hipLaunchKernelGGL((k_lu_leaf_z64<8, 2>), g, b, 0, s, ar, ai, lda, perm, k0, mm, nc, n2, info);
  else if (R <= 16) hipLaunchKernelGGL((k_lu_leaf_z64<16, 1>), g, b, 0, s, ar, ai, lda, perm, k0, mm, nc, n2, info);
  else throw std::runtime_error("getrf_z64: matrix order above 16384 is not supported");
  FROB_LAUNCH_CHECK();
}

void zgetrf_rec(hipStream_t s, double* ar, double* ai, int lda, int* perm, int k0, int m, int n, int* info,
                double* work) {
  const int mm = m - k0;
  const int wmax = zleaf_width(mm);
  if (n <= wmax) {
    zlaunch_leaf(s, ar, ai, lda, perm, k0, mm, n, 0, info);
    return;
  }
  int n1 = (n / 2 + 3) / 4 * 4;
  if (n1 >= n) n1 = n / 2;
  const int n2 = n - n1;
  if (n1 <= wmax && n2 <= wmax) {
    zlaunch_leaf(s, ar, ai, lda, perm, k0, mm, n1, n2, info);
    zgetrf_rec(s, ar, ai, lda, perm, k0 + n1, m, n2, info, work);
    return;
  }
  zgetrf_rec(s, ar, ai, lda, perm, k0, m, n1, info, work);
  ZOp L11{ar + k0, ai + k0, lda, perm + k0};
  ZOut A12{ar + k0 + n1, ai + k0 + n1, lda, perm + k0, nullptr};
  trsm_z64(s, false, TRI_LOWER_UNIT, OP_N, n1, n2, L11, A12, work);
  ZOp L21{ar + k0, ai + k0, lda, perm + k0 + n1};
  ZOp U12{ar + k0 + n1, ai + k0 + n1, lda, perm + k0};
  ZOut A22{ar + k0 + n1, ai + k0 + n1, lda, perm + k0 + n1, nullptr};
  gemm_z64(s, OP_N, OP_N, m - k0 - n1, n2, n1, -1.0, L21, TRI_NONE, U12, TRI_NONE, 1.0, A22);
  zgetrf_rec(s, ar, ai, lda, perm, k0 + n1, m, n2, info, work);
}

}  // namespace

size_t getrf_z_work_elems(int n) { return trsm_z_work_elems(n / 2 + 8); }

void getrf_z64(hipStream_t s, int n, double* re, double* im, int lda, int* perm, int* info, double* work) {
  if (n <= 0) return;
  iota_i32(s, n, perm);
  zgetrf_rec(s, re, im, lda, perm, 0, n, n, info, work);
}

}  // namespace frob
