// lu_z64.hip -- complex (planar FP64) LU with partial pivoting for the
// complex-arithmetic baseline (Algorithm 4).  Same design as lu_f64.hip:
// recursive column splitting, register-resident leaf panels in one workgroup
// (512 or 1024 threads) with position-tracked rows, pivoting through the row-index array
// perm, one launch per bottom recursion node.  A complex value takes two
// registers, so a leaf holds half as many columns as the real one.  The pivot
// measure is |Re| + |Im| (LAPACK's izamax convention); ties go to the lowest
// row.
#include <algorithm>

#include "common.hpp"
#include "devutil.hpp"
#include "internal.hpp"
#include "tri_dev.hpp"

namespace frob {

namespace {

constexpr int ZLT = 512;   // threads of the leaf workgroup (twice that for 513 .. 4096 rows)

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

// the fused sibling update needs a second R x W block of registers
constexpr bool ZLEAF_SIBLING(int R) { return R <= 8; }
// leaves whose panel and sibling blocks move together, transposed through LDS
constexpr bool ZLEAF_JOINT(int W) { return W % 2 == 0 && W <= 8; }

// One workgroup factors an mm x nc complex panel (nc <= W) held in
// registers, thread t of NT owning panel rows q = t + s * NT (s < R).  The design
// is the real leaf's (lu_f64.hip): rows never move, each carries its logical
// position pos and a pivot step exchanges positions only; the candidate
// search runs on FP32 images of the pivot measure |Re| + |Im| with the exact
// FP64 comparison on ties; one barrier per column; rows are read and written
// by their owning threads straight from HBM; with n2 > 0 the kernel factors a
// whole bottom recursion node (the n2 columns to the right are updated with
// U12 = L11^{-1} A12, A22 -= L21 U12 and factored as panel columns
// nc .. nc + n2).
template <int R, int W, int NT = ZLT>
__global__ __launch_bounds__(NT) void k_lu_leaf_z64(double* __restrict__ ar, double* __restrict__ ai, int lda,
                                                    int* __restrict__ perm, int k0, int mm, int nc, int n2, int* info,
                                                    int* __restrict__ snap, int sfrom) {
  constexpr int NW = NT / 64;
  __shared__ double s_cv[2][NW];
  __shared__ int s_ck[2][NW];
  __shared__ double s_crr[2][NW][W], s_cri[2][NW][W];
  __shared__ double s_lr[W][W + 1], s_li[W][W + 1];
  __shared__ double s_ur[W][W + 1], s_ui[W][W + 1];
  // staging of the joint row segments (row pitch 2W + 2 doubles: 16-byte
  // aligned rows, consecutive rows on different banks)
  __shared__ __align__(16) double s_st[ZLEAF_JOINT(W) ? NW : 1][64][ZLEAF_JOINT(W) ? 2 * W + 2 : 2];
  __shared__ int s_sph[ZLEAF_JOINT(W) ? NW : 1][64];

  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const bool vbase = ((lda & 1) == 0) && ((reinterpret_cast<uintptr_t>(ar) & 15) == 0) &&
                     ((reinterpret_cast<uintptr_t>(ai) & 15) == 0);

  int ph[R], pos[R];
#pragma unroll
  for (int s = 0; s < R; ++s) ph[s] = perm[k0 + min(t + s * NT, mm - 1)];
#pragma unroll
  for (int s = 0; s < R; ++s) pos[s] = t + s * NT < mm ? t + s * NT : -1;

  // columns col0 .. col0 + ncol - 1 of this thread's rows (both planes), one
  // batch of unconditional loads at clamped addresses
  auto load_rows = [&](double (&xr)[R][W], double (&xi)[R][W], int col0, int ncol, bool mask = true) {
    if (W % 2 == 0 && vbase && ((col0 | ncol) & 1) == 0) {
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const long long o = (long long)ph[s] * lda + col0;
#pragma unroll
        for (int c = 0; c + 1 < W; c += 2) {
          const double2 yr = *reinterpret_cast<const double2*>(ar + o + min(c, ncol - 2));
          const double2 yi = *reinterpret_cast<const double2*>(ai + o + min(c, ncol - 2));
          xr[s][c] = yr.x; xr[s][c + 1] = yr.y;
          xi[s][c] = yi.x; xi[s][c + 1] = yi.y;
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const long long o = (long long)ph[s] * lda + col0;
#pragma unroll
        for (int c = 0; c < W; ++c) {
          xr[s][c] = ar[o + min(c, ncol - 1)];
          xi[s][c] = ai[o + min(c, ncol - 1)];
        }
      }
    }
    if (mask) {
#pragma unroll
      for (int s = 0; s < R; ++s)
#pragma unroll
        for (int c = 0; c < W; ++c) {
          xr[s][c] = c < ncol ? xr[s][c] : 0.0;
          xi[s][c] = c < ncol ? xi[s][c] : 0.0;
        }
    }
  };
  auto store_rows = [&](const double (&xr)[R][W], const double (&xi)[R][W], int col0, int ncol) {
    const bool vec = W % 2 == 0 && vbase && ((col0 | ncol) & 1) == 0;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      if (pos[s] < 0) continue;
      const long long o = (long long)ph[s] * lda + col0;
      if (vec) {
#pragma unroll
        for (int c = 0; c + 1 < W; c += 2)
          if (c < ncol) {
            *reinterpret_cast<double2*>(ar + o + c) = make_double2(xr[s][c], xr[s][c + 1]);
            *reinterpret_cast<double2*>(ai + o + c) = make_double2(xi[s][c], xi[s][c + 1]);
          }
      } else {
#pragma unroll
        for (int c = 0; c < W; ++c)
          if (c < ncol) {
            ar[o + c] = xr[s][c];
            ai[o + c] = xi[s][c];
          }
      }
    }
  };

  double vr[R][W], vi[R][W], xr[R][W], xi[R][W];
  // panel and sibling block together: row segments of W + n2 columns per plane
  const bool joint = W % 2 == 0 && ZLEAF_SIBLING(R) && n2 > 0 && nc == W && vbase && ((k0 | n2) & 1) == 0;
  // Joint segments transposed through LDS (as in the real leaf): W
  // consecutive lanes move one row segment of a plane (16 bytes each), so an
  // instruction touches 64 / W row segments instead of 64; the planes take
  // turns in one staging buffer, each wave staging its own 64 rows per slot.
  constexpr int RPI = 64 / (W > 1 ? W : 2);
  const int m = lane % W;
  auto stage_in = [&](const double (&y0)[W], const double (&y1)[W], double (&p)[W], double (&q)[W])
                      __attribute__((always_inline)) {
    __syncthreads();   // the previous contents have been read
#pragma unroll
    for (int i = 0; i < W; ++i)
      *reinterpret_cast<double2*>(&s_st[wv][i * RPI + lane / W][2 * m]) = make_double2(y0[i], y1[i]);
    __syncthreads();
#pragma unroll
    for (int c = 0; c + 1 < W; c += 2) {
      const double2 e = *reinterpret_cast<const double2*>(&s_st[wv][lane][c]);
      const double2 f = *reinterpret_cast<const double2*>(&s_st[wv][lane][W + c]);
      p[c] = e.x; p[c + 1] = e.y;
      q[c] = f.x; q[c + 1] = f.y;
    }
  };
  auto stage_out = [&](const double (&p)[W], const double (&q)[W], double* plane, int prs)
                       __attribute__((always_inline)) {
    __syncthreads();
    double* rb = &s_st[wv][lane][0];
#pragma unroll
    for (int c = 0; c + 1 < W; c += 2) {
      *reinterpret_cast<double2*>(rb + c) = make_double2(p[c], p[c + 1]);
      *reinterpret_cast<double2*>(rb + W + c) = make_double2(q[c], q[c + 1]);
    }
    s_sph[wv][lane] = prs;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < W; ++i) {
      const int r = i * RPI + lane / W;
      const double2 y = *reinterpret_cast<const double2*>(&s_st[wv][r][2 * m]);
      const int prow = s_sph[wv][r];
      if (prow >= 0 && 2 * m < W + n2) *reinterpret_cast<double2*>(plane + (long long)prow * lda + k0 + 2 * m) = y;
    }
  };
  if (ZLEAF_JOINT(W) && joint) {
    if constexpr (ZLEAF_JOINT(W)) {
      const int cm = k0 + min(2 * m, W + n2 - 2);
      double y0r[R][W], y1r[R][W], y0i[R][W], y1i[R][W];
#pragma unroll
      for (int s = 0; s < R; ++s)
#pragma unroll
        for (int i = 0; i < W; ++i) {
          const long long o = (long long)__shfl(ph[s], i * RPI + lane / W) * lda + cm;
          const double2 tr = *reinterpret_cast<const double2*>(ar + o);
          const double2 ti = *reinterpret_cast<const double2*>(ai + o);
          y0r[s][i] = tr.x; y1r[s][i] = tr.y;
          y0i[s][i] = ti.x; y1i[s][i] = ti.y;
        }
#pragma unroll
      for (int s = 0; s < R; ++s) {
        __builtin_amdgcn_sched_barrier(0);   // one slot at a time (register pressure)
        stage_in(y0r[s], y1r[s], vr[s], xr[s]);
        stage_in(y0i[s], y1i[s], vi[s], xi[s]);
      }
    }
  } else if (joint) {
    // the sibling's columns continue this thread's row segments: each row's
    // pairs are fetched right after the panel's, from the cache line the
    // first load brought in; they stay in flight during the first half and
    // are masked when first used
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const long long o = (long long)ph[s] * lda + k0;
#pragma unroll
      for (int c = 0; c + 1 < W; c += 2) {
        const double2 yr = *reinterpret_cast<const double2*>(ar + o + c);
        const double2 yi = *reinterpret_cast<const double2*>(ai + o + c);
        vr[s][c] = yr.x; vr[s][c + 1] = yr.y;
        vi[s][c] = yi.x; vi[s][c + 1] = yi.y;
      }
#pragma unroll
      for (int c = 0; c + 1 < W; c += 2) {
        const double2 yr = *reinterpret_cast<const double2*>(ar + o + W + min(c, n2 - 2));
        const double2 yi = *reinterpret_cast<const double2*>(ai + o + W + min(c, n2 - 2));
        xr[s][c] = yr.x; xr[s][c + 1] = yr.y;
        xi[s][c] = yi.x; xi[s][c + 1] = yi.y;
      }
    }
  } else {
    load_rows(vr, vi, k0, nc);
    // the sibling's columns are fetched now and stay in flight during the
    // first half (masked when first used, so nothing waits on them before)
    if (ZLEAF_SIBLING(R) && n2 > 0) load_rows(xr, xi, k0 + nc, n2, false);
  }

  int first_zero = 0;
  // one column step: register column jj of block (xr, xi), panel column off + jj
  auto column = [&](double (&xr)[R][W], double (&xi)[R][W], auto jc, int off, int ncols)
                    __attribute__((always_inline)) {
    constexpr int jj = decltype(jc)::value;
    if (jj >= ncols) return;  // uniform
    const int jp = off + jj;
    constexpr int par = jj & 1;
    auto meas = [&](int s) { return fabs(xr[s][jj]) + fabs(xi[s][jj]); };
    auto key = [&](int s) {
      const double m = meas(s);
      return (pos[s] >= jp && m == m) ? __float_as_int((float)m) : -1;
    };
    int kmax = key(0);
#pragma unroll
    for (int s = 1; s < R; ++s) kmax = max(kmax, key(s));
    double best = -1.0;
    int bq = INT_MAX, nt = 0;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const bool m = kmax >= 0 && key(s) == kmax;
      best = m ? meas(s) : best;
      bq = m ? pos[s] : bq;
      nt += m ? 1 : 0;
    }
    if (R > 1 && __ballot(nt > 1)) {
      best = -1.0;
      bq = INT_MAX;
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const double m = meas(s);
        const bool ok = kmax >= 0 && key(s) == kmax && (m > best || (m == best && pos[s] < bq));
        best = ok ? m : best;
        bq = ok ? pos[s] : bq;
      }
    }
    const int wmf = wave_max_key(kmax);
    if (wmf >= 0) {
      const unsigned long long tied = __ballot(kmax == wmf);
      const int wl = (__popcll(tied) == 1) ? __ffsll((long long)tied) - 1 : exact_argmax(tied, best, bq);
      if (lane == wl) {
#pragma unroll
        for (int s = 0; s < R; ++s)
          if (pos[s] == bq) {
#pragma unroll
            for (int c = 0; c < W; ++c) {
              s_crr[par][wv][c] = xr[s][c];
              s_cri[par][wv][c] = xi[s][c];
            }
          }
        s_cv[par][wv] = best;
        s_ck[par][wv] = bq;
      }
    } else if (lane == 0) {
      s_cv[par][wv] = -1.0;
      s_ck[par][wv] = INT_MAX;
    }
    __syncthreads();
    // (read unconditionally, then selected: no divergent branch around the LDS reads)
    const double sv0 = s_cv[par][lane & (NW - 1)];
    const int sk0 = s_ck[par][lane & (NW - 1)];
    const double sv = lane < NW ? sv0 : -2.0;
    const int sk = lane < NW ? sk0 : INT_MAX;
    const int sf = __float_as_int((float)sv);
    const int gmf = __builtin_amdgcn_readlane(row_max_key(sf), 15);
    int p;
    const double *prr, *pri;
    if (gmf >= 0) {
      const unsigned long long tied = __ballot(lane < NW && sf == gmf);
      const int gw = (__popcll(tied) == 1) ? __ffsll((long long)tied) - 1 : exact_argmax(tied, sv, sk);
      p = __builtin_amdgcn_readlane(sk, gw);
      prr = s_crr[par][gw];
      pri = s_cri[par][gw];
    } else {
      // every candidate is NaN: keep row jp in place (uniform slow path)
      p = jp;
#pragma unroll
      for (int s = 0; s < R; ++s)
        if (pos[s] == jp) {
#pragma unroll
          for (int c = 0; c < W; ++c) {
            s_crr[par][0][c] = xr[s][c];
            s_cri[par][0][c] = xi[s][c];
          }
        }
      __syncthreads();
      prr = s_crr[par][0];
      pri = s_cri[par][0];
    }
#pragma unroll
    for (int s = 0; s < R; ++s) pos[s] = pos[s] == p ? jp : (pos[s] == jp ? p : pos[s]);
    const zc piv{prr[jj], pri[jj]};
    const bool nz = piv.r != 0.0 || piv.i != 0.0;
    if (!nz && !first_zero) first_zero = k0 + jp + 1;
    const zc rp = nz ? zrecip(piv) : zc{0.0, 0.0};
    double pwr[W], pwi[W];
#pragma unroll
    for (int c = jj + 1; c < W; ++c) {
      pwr[c] = prr[c];
      pwi[c] = pri[c];
    }
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const bool below = nz && pos[s] > jp;
      const zc q = zmul(zc{xr[s][jj], xi[s][jj]}, rp);
      const double lr = below ? q.r : 0.0, li = below ? q.i : 0.0;
      xr[s][jj] = below ? q.r : xr[s][jj];
      xi[s][jj] = below ? q.i : xi[s][jj];
#pragma unroll
      for (int c = jj + 1; c < W; ++c) {
        xr[s][c] = fma(li, pwi[c], fma(-lr, pwr[c], xr[s][c]));
        xi[s][c] = fma(-li, pwr[c], fma(-lr, pwi[c], xi[s][c]));
      }
    }
  };
  StaticFor<0, W>::run([&](auto jc) __attribute__((always_inline)) { column(vr, vi, jc, 0, nc); });
  if (!(ZLEAF_JOINT(W) && joint)) store_rows(vr, vi, k0, nc);

  if (ZLEAF_SIBLING(R) && n2 > 0) {
    const int cs = k0 + nc;
#pragma unroll
    for (int s = 0; s < R; ++s)
#pragma unroll
      for (int c = 0; c < W; ++c) {
        xr[s][c] = c < n2 ? xr[s][c] : 0.0;
        xi[s][c] = c < n2 ? xi[s][c] : 0.0;
      }
#pragma unroll
    for (int s = 0; s < R; ++s)
      if (pos[s] >= 0 && pos[s] < nc) {
        const int i = pos[s];
#pragma unroll
        for (int k = 0; k < W; ++k) {
          s_lr[i][k] = vr[s][k];
          s_li[i][k] = vi[s][k];
          s_ur[i][k] = xr[s][k];
          s_ui[i][k] = xi[s][k];
        }
      }
    __syncthreads();
    if (t < n2) {
      // U12 = L11^{-1} A12, column t, by substitution in registers
      double ur[W], ui[W];
#pragma unroll
      for (int i = 0; i < W; ++i) {
        const double vr = s_ur[i][t], vi = s_ui[i][t];
        ur[i] = i < nc ? vr : 0.0;
        ui[i] = i < nc ? vi : 0.0;
      }
      StaticFor<1, W>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if (i >= nc) return;  // uniform
        double accr = ur[i], acci = ui[i];
#pragma unroll
        for (int k = 0; k < i; ++k) {
          const double lr = s_lr[i][k], li = s_li[i][k];
          accr = fma(li, ui[k], fma(-lr, ur[k], accr));
          acci = fma(-li, ur[k], fma(-lr, ui[k], acci));
        }
        ur[i] = accr;
        ui[i] = acci;
      });
#pragma unroll
      for (int i = 0; i < W; ++i)
        if (i < nc) {
          s_ur[i][t] = ur[i];
          s_ui[i][t] = ui[i];
        }
    }
    __syncthreads();
    // A22 -= L21 U12, one row of U12 at a time
    StaticFor<0, W>::run([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      if (k >= nc) return;  // uniform
      __builtin_amdgcn_sched_barrier(0);
      double ur[W], ui[W];
#pragma unroll
      for (int c = 0; c < W; ++c) {
        ur[c] = s_ur[k][c];
        ui[c] = s_ui[k][c];
      }
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const double lr = vr[s][k], li = vi[s][k];
#pragma unroll
        for (int c = 0; c < W; ++c) {
          xr[s][c] = fma(li, ui[c], fma(-lr, ur[c], xr[s][c]));
          xi[s][c] = fma(-li, ur[c], fma(-lr, ui[c], xi[s][c]));
        }
      }
    });
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const bool top = pos[s] >= 0 && pos[s] < nc;
      const int pi = top ? pos[s] : 0;
#pragma unroll
      for (int c = 0; c < W; ++c) {
        const double uvr = s_ur[pi][c], uvi = s_ui[pi][c];
        xr[s][c] = top ? uvr : xr[s][c];
        xi[s][c] = top ? uvi : xi[s][c];
      }
    }
    StaticFor<0, W>::run([&](auto jc) __attribute__((always_inline)) { column(xr, xi, jc, nc, n2); });
    if (ZLEAF_JOINT(W) && joint) {
      if constexpr (ZLEAF_JOINT(W)) {
#pragma unroll
        for (int s = 0; s < R; ++s) {
          const int prs = pos[s] >= 0 ? ph[s] : -1;
          stage_out(vr[s], xr[s], ar, prs);
          stage_out(vi[s], xi[s], ai, prs);
        }
      }
    } else {
      store_rows(xr, xi, cs, n2);
    }
  }
  if (t == 0 && first_zero && *info == 0) *info = first_zero;

#pragma unroll
  for (int s = 0; s < R; ++s)
    if (pos[s] >= 0) {
      perm[k0 + pos[s]] = ph[s];
      // copy of the trailing row order from position sfrom on (look-ahead)
      if (snap && k0 + pos[s] >= sfrom) snap[k0 + pos[s] - sfrom] = ph[s];
    }
}

// widest leaf for a panel with mm rows (R * W <= 16 complex values per thread)
inline int zleaf_width(int mm) {
  const int R = ceil_div(mm, ZLT);
  if (R <= 1) return 16;
  if (R <= 2) return 8;
  if (R <= 4) return 4;
  if (R <= 8) return 2;
  if (R <= 32) return 1;
  return 0;
}

void zlaunch_leaf(hipStream_t s, double* ar, double* ai, int lda, int* perm, int k0, int mm, int nc, int n2,
                  int* info, int* snap = nullptr, int sfrom = 0) {
  const int R = ceil_div(mm, ZLT);
  if (nc > zleaf_width(mm) || n2 > zleaf_width(mm)) throw std::runtime_error("getrf_z64: leaf wider than template");
  if (n2 > 0 && !ZLEAF_SIBLING(R)) throw std::runtime_error("getrf_z64: no fused sibling update for this leaf");
  // 1024 threads for 513 .. 4096 rows (half the rows per thread of a 512-thread
  // leaf of the same width), 512 otherwise
  void (*kern)(double*, double*, int, int*, int, int, int, int, int*, int*, int);
  int threads = 2 * ZLT;
  if (R <= 1) { kern = k_lu_leaf_z64<1, 16>; threads = ZLT; }
  else if (R <= 2) kern = k_lu_leaf_z64<1, 8, 2 * ZLT>;
  else if (R <= 4) kern = k_lu_leaf_z64<2, 4, 2 * ZLT>;
  else if (R <= 8) kern = k_lu_leaf_z64<4, 2, 2 * ZLT>;
  else if (R <= 16) { kern = k_lu_leaf_z64<16, 1>; threads = ZLT; }
  else if (R <= 32) { kern = k_lu_leaf_z64<32, 1>; threads = ZLT; }
  else throw std::runtime_error("getrf_z64: matrix order above 16384 is not supported");
  hipLaunchKernelGGL(kern, dim3(1), dim3(threads), 0, s, ar, ai, lda, perm, k0, mm, nc, n2, info, snap, sfrom);
  FROB_LAUNCH_CHECK();
}

// Solve L x = b in place for a unit lower complex triangle L of order
// 4 NBLK in LDS (planes Lr, Li, row stride LDL); the quad layout and
// sweeps of quad_lower_solve (tri_dev.hpp), in complex arithmetic.
template <int LDL, int NBLK>
__device__ __forceinline__ void zquad_unit_lower_solve(const double* __restrict__ Lr, const double* __restrict__ Li,
                                                       double (&xr)[NBLK], double (&xi)[NBLK], int g) {
  StaticFor<0, NBLK>::run([&](auto bc) {
    constexpr int b = decltype(bc)::value;
    double br = xr[b], bi = xi[b];
    double sr[4], si[4];
    StaticFor<0, 4>::run([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      sr[q] = quad_bcast<q>(br);
      si[q] = quad_bcast<q>(bi);
      if (q < 3 && g > q) {
        const double lr = Lr[(4 * b + g) * LDL + 4 * b + q], li = Li[(4 * b + g) * LDL + 4 * b + q];
        br = fma(li, si[q], fma(-lr, sr[q], br));
        bi = fma(-li, sr[q], fma(-lr, si[q], bi));
      }
    });
    xr[b] = br;
    xi[b] = bi;
    StaticFor<0, 4>::run([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      StaticFor<b + 1, NBLK>::run([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        const double lr = Lr[(4 * m + g) * LDL + 4 * b + q], li = Li[(4 * m + g) * LDL + 4 * b + q];
        xr[m] = fma(li, si[q], fma(-lr, sr[q], xr[m]));
        xi[m] = fma(-li, sr[q], fma(-lr, si[q], xi[m]));
      });
    });
  });
}

// Internal recursion node with n1, n2 <= NB (16 or 32) in one launch, the
// complex counterpart of the real node kernel (lu_f64.hip): every workgroup
// solves U12 = L11^{-1} A12 and updates its 64 rows of A22 -= L21 U12; the
// last workgroup to finish (counted on *cnt) writes U12 and resets the count.
constexpr int ZNODE_MAX = 32;
template <int NB>
__global__ __launch_bounds__(256) void k_lu_node_z64(double* __restrict__ ar, double* __restrict__ ai, int lda,
                                                     const int* __restrict__ perm, int k0, int mm, int n1, int n2,
                                                     int* cnt) {
  constexpr int ROWS = 64;
  constexpr int LD = NB + 1;
  constexpr int TPR = 256 / NB;
  constexpr int PL = NB * NB / 256;
  constexpr int PB = ROWS * NB / 256;
  constexpr int QB = NB / 4;
  constexpr int CJ = NB / 16;
  static_assert(PL >= 1 && NB % 16 == 0, "node shape");
  __shared__ double Lsr[ROWS * LD], Lsi[ROWS * LD];
  __shared__ double Usr[NB * LD], Usi[NB * LD];
  __shared__ int s_last;
  const int tid = threadIdx.x;
  const int cs = k0 + n1;
  const int r0 = n1 + blockIdx.x * ROWS;
  const int er = tid / NB, ec = tid % NB;
  const int c = tid >> 2, g = tid & 3;
  const int ti = tid >> 4, tj = tid & 15;
  // one batch of unconditional loads at clamped addresses
  int pl[PL], pb[PB], px[QB], qr[4];
#pragma unroll
  for (int u = 0; u < PL; ++u) pl[u] = perm[k0 + min(er + TPR * u, n1 - 1)];
#pragma unroll
  for (int u = 0; u < PB; ++u) pb[u] = perm[k0 + min(r0 + er + TPR * u, mm - 1)];
#pragma unroll
  for (int u = 0; u < QB; ++u) px[u] = perm[k0 + min(4 * u + g, n1 - 1)];
#pragma unroll
  for (int i = 0; i < 4; ++i) qr[i] = perm[k0 + min(r0 + ti + 16 * i, mm - 1)];
  double vlr[PL], vli[PL], vbr[PB], vbi[PB], xr[QB], xi[QB], accr[4][CJ], acci[4][CJ];
  {
    const int cl = k0 + min(ec, n1 - 1), cx = cs + min(c, n2 - 1);
#pragma unroll
    for (int u = 0; u < PL; ++u) {
      vlr[u] = ar[(long long)pl[u] * lda + cl];
      vli[u] = ai[(long long)pl[u] * lda + cl];
    }
#pragma unroll
    for (int u = 0; u < QB; ++u) {
      xr[u] = ar[(long long)px[u] * lda + cx];
      xi[u] = ai[(long long)px[u] * lda + cx];
    }
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      vbr[u] = ar[(long long)pb[u] * lda + cl];
      vbi[u] = ai[(long long)pb[u] * lda + cl];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < CJ; ++j) {
        const long long o = (long long)qr[i] * lda + cs + min(tj + 16 * j, n2 - 1);
        accr[i][j] = ar[o];
        acci[i][j] = ai[o];
      }
  }
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int r = er + TPR * u;
    const bool low = r < n1 && ec < r;
    Lsr[r * LD + ec] = low ? vlr[u] : (r == ec ? 1.0 : 0.0);
    Lsi[r * LD + ec] = low ? vli[u] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < QB; ++u) {
    const bool ok = 4 * u + g < n1 && c < n2;
    xr[u] = ok ? xr[u] : 0.0;
    xi[u] = ok ? xi[u] : 0.0;
  }
  __syncthreads();
  zquad_unit_lower_solve<LD, QB>(Lsr, Lsi, xr, xi, g);
  __syncthreads();   // every wave is done with L11
  if (c < NB) {
#pragma unroll
    for (int u = 0; u < QB; ++u) {
      Usr[(4 * u + g) * LD + c] = xr[u];
      Usi[(4 * u + g) * LD + c] = xi[u];
    }
  }
#pragma unroll
  for (int u = 0; u < PB; ++u) {
    const int r = er + TPR * u;
    const bool ok = r0 + r < mm && ec < n1;
    Lsr[r * LD + ec] = ok ? vbr[u] : 0.0;
    Lsi[r * LD + ec] = ok ? vbi[u] : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < n1; ++k) {
    double lr[4], li[4], ur[CJ], ui[CJ];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      lr[i] = Lsr[(ti + 16 * i) * LD + k];
      li[i] = Lsi[(ti + 16 * i) * LD + k];
    }
#pragma unroll
    for (int j = 0; j < CJ; ++j) {
      ur[j] = Usr[k * LD + tj + 16 * j];
      ui[j] = Usi[k * LD + tj + 16 * j];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < CJ; ++j) {
        accr[i][j] = fma(li[i], ui[j], fma(-lr[i], ur[j], accr[i][j]));
        acci[i][j] = fma(-li[i], ur[j], fma(-lr[i], ui[j], acci[i][j]));
      }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < CJ; ++j) {
      const int r = r0 + ti + 16 * i, cc = tj + 16 * j;
      if (r < mm && cc < n2) {
        const long long o = (long long)qr[i] * lda + cs + cc;
        ar[o] = accr[i][j];
        ai[o] = acci[i][j];
      }
    }
  // every read of A12 by this workgroup is complete
  if (tid == 0) s_last = atomicAdd(cnt, 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (s_last) {
#pragma unroll
    for (int u = 0; u < PL; ++u) {
      const int r = er + TPR * u;
      if (r < n1 && ec < n2) {
        const long long o = (long long)pl[u] * lda + cs + ec;
        ar[o] = Usr[r * LD + ec];
        ai[o] = Usi[r * LD + ec];
      }
    }
    if (tid == 0) atomicExch(cnt, 0);
  }
}

void zlaunch_node(hipStream_t s, double* ar, double* ai, int lda, const int* perm, int k0, int mm, int n1, int n2,
                  int* cnt) {
  const int rows = mm - n1;
  const dim3 g(rows > 0 ? ceil_div(rows, 64) : 1), b(256);
  const int w = max(n1, n2);
  if (w <= 16) hipLaunchKernelGGL(k_lu_node_z64<16>, g, b, 0, s, ar, ai, lda, perm, k0, mm, n1, n2, cnt);
  else if (w <= ZNODE_MAX) hipLaunchKernelGGL(k_lu_node_z64<32>, g, b, 0, s, ar, ai, lda, perm, k0, mm, n1, n2, cnt);
  else throw std::runtime_error("getrf_z64: node wider than the node kernel");
  FROB_LAUNCH_CHECK();
}

// snap (optional): the leaf that ends the recursion also writes
// perm[sfrom .. m) to snap[0 ..)
void zgetrf_rec(hipStream_t s, double* ar, double* ai, int lda, int* perm, int k0, int m, int n, int* info,
                double* work, int* cnt, int* snap = nullptr, int sfrom = 0) {
  const int mm = m - k0;
  const int wmax = zleaf_width(mm);
  if (n <= wmax) {
    zlaunch_leaf(s, ar, ai, lda, perm, k0, mm, n, 0, info, snap, sfrom);
    return;
  }
  int n1 = (n / 2 + 3) / 4 * 4;
  if (n1 >= n) n1 = n / 2;
  const int n2 = n - n1;
  if (n1 <= wmax && n2 <= wmax && ZLEAF_SIBLING(ceil_div(mm, ZLT))) {
    // bottom node: one leaf launch factors both halves
    zlaunch_leaf(s, ar, ai, lda, perm, k0, mm, n1, n2, info, snap, sfrom);
    return;
  }
  zgetrf_rec(s, ar, ai, lda, perm, k0, m, n1, info, work, cnt);
  if (n1 <= ZNODE_MAX && n2 <= ZNODE_MAX) {
    zlaunch_node(s, ar, ai, lda, perm, k0, m - k0, n1, n2, cnt);
    zgetrf_rec(s, ar, ai, lda, perm, k0 + n1, m, n2, info, work, cnt, snap, sfrom);
    return;
  }
  ZOp L11{ar + k0, ai + k0, lda, perm + k0};
  ZOut A12{ar + k0 + n1, ai + k0 + n1, lda, perm + k0, nullptr};
  trsm_z64(s, false, TRI_LOWER_UNIT, OP_N, n1, n2, L11, A12, work);
  ZOp L21{ar + k0, ai + k0, lda, perm + k0 + n1};
  ZOp U12{ar + k0 + n1, ai + k0 + n1, lda, perm + k0};
  ZOut A22{ar + k0 + n1, ai + k0 + n1, lda, perm + k0 + n1, nullptr};
  gemm_z64(s, OP_N, OP_N, m - k0 - n1, n2, n1, -1.0, L21, TRI_NONE, U12, TRI_NONE, 1.0, A22);
  zgetrf_rec(s, ar, ai, lda, perm, k0 + n1, m, n2, info, work, cnt, snap, sfrom);
}

// Panels of ZLA_NB columns with a look-ahead of one panel; the ordering and
// the snapshot of the trailing rows' indices are those of the real version
// (getrf_lookahead in lu_f64.hip).
void zgetrf_lookahead(hipStream_t s0, int n, double* ar, double* ai, int lda, int* perm, int* info, double* work,
                      int* cnt, const LookAhead& la) {
  hipStream_t s1 = la.s1;
  double* work0 = work;
  double* work1 = work0 + trsm_z_work_elems(n / 2 + 8);
  int* snap[2];
  snap[0] = reinterpret_cast<int*>(work1 + trsm_z_work_elems(ZLA_NB));
  snap[1] = snap[0] + n;
  auto evF = [&](int j) { return la.ev[j & 3]; };
  auto evR = [&](int j) { return la.ev[4 + (j & 3)]; };
  auto update = [&](hipStream_t st, int k0, int nb, int c, int w, const int* trows, double* wk) {
    ZOp L11{ar + k0, ai + k0, lda, perm + k0};
    ZOut A12{ar + c, ai + c, lda, perm + k0, nullptr};
    trsm_z64(st, false, TRI_LOWER_UNIT, OP_N, nb, w, L11, A12, wk);
    ZOp L21{ar + k0, ai + k0, lda, trows};
    ZOp U12{ar + c, ai + c, lda, perm + k0};
    ZOut A22{ar + c, ai + c, lda, trows, nullptr};
    gemm_z64(st, OP_N, OP_N, n - (k0 + nb), w, nb, -1.0, L21, TRI_NONE, U12, TRI_NONE, 1.0, A22);
  };
  const int np = ceil_div(n, ZLA_NB);
  int last_r = -1;
  for (int j = 0; j < np; ++j) {
    const int k0 = j * ZLA_NB, nb = min(ZLA_NB, n - k0);
    const int r0 = k0 + nb;
    int* sn = snap[j & 1];
    // the panel's last leaf also writes the snapshot perm[r0 .. n)
    zgetrf_rec(s0, ar, ai, lda, perm, k0, n, nb, info, work0, cnt, r0 < n ? sn : nullptr, r0);
    if (r0 >= n) break;
    FROB_HIP(hipEventRecord(evF(j), s0));
    const int c1 = r0, w1 = min(ZLA_NB, n - c1);
    if (j >= 1 && last_r == j - 1) FROB_HIP(hipStreamWaitEvent(s0, evR(j - 1), 0));
    // the next panel's update is a recursion node when it is narrow enough
    if (nb <= ZNODE_MAX && w1 <= ZNODE_MAX) zlaunch_node(s0, ar, ai, lda, perm, k0, n - k0, nb, w1, cnt);
    else update(s0, k0, nb, c1, w1, perm + r0, work0);
    const int c2 = c1 + w1, w2 = n - c2;
    if (w2 > 0) {
      FROB_HIP(hipStreamWaitEvent(s1, evF(j), 0));
      GridCapScope cap(LA_GRID_CAP);   // leave compute units to the panel chain
      update(s1, k0, nb, c2, w2, sn, work1);
      FROB_HIP(hipEventRecord(evR(j), s1));
      last_r = j;
    }
  }
  if (last_r >= 0) FROB_HIP(hipStreamWaitEvent(s0, evR(last_r), 0));
}

}  // namespace

size_t getrf_z_work_elems(int n) {
  return 64 + trsm_z_work_elems(n / 2 + 8) + trsm_z_work_elems(ZLA_NB) + (size_t)n;
}

void getrf_z64(hipStream_t s, int n, double* re, double* im, int lda, int* perm, int* info, double* work,
               const LookAhead* la) {
  if (n <= 0) return;
  iota_i32(s, n, perm);
  // the node kernels' workgroup counter lives in the first 64 doubles of work
  int* cnt = reinterpret_cast<int*>(work);
  fill_i32(s, 1, 0, cnt);
  if (getrf_lookahead_on(n, la)) zgetrf_lookahead(s, n, re, im, lda, perm, info, work + 64, cnt, *la);
  else zgetrf_rec(s, re, im, lda, perm, 0, n, n, info, work + 64, cnt);
}

}  // namespace frob
