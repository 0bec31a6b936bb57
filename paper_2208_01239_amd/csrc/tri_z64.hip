// tri_z64.hip -- complex (planar FP64) triangular solves and inverses for the
// complex-arithmetic baselines.  Same structure as tri_f64.hip:
//  * base case: a triangle of order <= 32 in LDS, one right-hand side per lane
//    in registers (a column of B on the left side, a row of B on the right
//    side), substitution with broadcast LDS reads of the triangle;
//  * diagonal-block inverses by one batched base-case launch plus two batched
//    complex GEMMs per doubling level;
//  * blocked solves: in-place GEMM leaves with the 64x64 diagonal inverses and
//    one GEMM update per inner node of the recursion.
// op(T) may be T, T^T or T^H (conjugate transpose).
#include "common.hpp"
#include "internal.hpp"

namespace frob {

namespace {

constexpr int TZ = 32;   // base-case triangle order
constexpr int DZ = 64;   // diagonal block order of the blocked solve

__host__ __device__ inline bool zlower(int tri) { return tri == TRI_LOWER || tri == TRI_LOWER_UNIT; }
__host__ __device__ inline bool zunit(int tri) { return tri == TRI_LOWER_UNIT || tri == TRI_UPPER_UNIT; }
__host__ __device__ inline int zflip(int tri) {
  switch (tri) {
    case TRI_LOWER: return TRI_UPPER;
    case TRI_LOWER_UNIT: return TRI_UPPER_UNIT;
    case TRI_UPPER: return TRI_LOWER;
    case TRI_UPPER_UNIT: return TRI_LOWER_UNIT;
    default: return tri;
  }
}

// Solve T' X' = B' where (left) T' = op(T), lane = column c of B; or (right,
// X op(T) = B) T' = op(T)^T, lane = row c of B.  Triangle order nt <= NT.
template <int NT, bool RIGHT>
__device__ __forceinline__ void ztrsm_reg_body(int tri, int opT, int nt, int nr, const ZOp& T, const ZOut& B,
                                               int identity, int c0) {
  __shared__ double Tr[NT][NT + 1];
  __shared__ double Ti[NT][NT + 1];
  const int lane = threadIdx.x;
  const int triP = RIGHT ? zflip(tri) : tri;
  // T'(i,k) = stored(k,i) if tT; conjugated if cj
  const bool tT = RIGHT ? (opT == OP_N) : (opT != OP_N);
  const bool cj = opT == OP_C;
  const bool lower = zlower(triP), unit = zunit(triP);
  for (int e = lane; e < NT * NT; e += 64) {
    const int r = e / NT, cc = e % NT;
    const int i = tT ? cc : r, k = tT ? r : cc;
    double vr = 0.0, vi = 0.0;
    if (i < nt && k < nt && (lower ? k <= i : k >= i)) {
      if (unit && i == k) vr = 1.0;
      else {
        const int pr = T.rows ? T.rows[r] : r;
        vr = T.re[(long long)pr * T.ld + cc];
        vi = T.im[(long long)pr * T.ld + cc];
        if (cj) vi = -vi;
      }
    }
    Tr[i][k] = vr;
    Ti[i][k] = vi;
  }
  const int c = c0 + lane;
  const bool act = c < nr;
  double xr[NT], xi[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    double vr = 0.0, vi = 0.0;
    if (i < nt && act) {
      if (identity) vr = (i == c) ? 1.0 : 0.0;
      else if (!RIGHT) {
        const int pr = B.rows ? B.rows[i] : i;
        vr = B.re[(long long)pr * B.ld + c];
        vi = B.im[(long long)pr * B.ld + c];
      } else {
        const int pr = B.rows ? B.rows[c] : c;
        vr = B.re[(long long)pr * B.ld + i];
        vi = B.im[(long long)pr * B.ld + i];
      }
    }
    xr[i] = vr;
    xi[i] = vi;
  }
  __syncthreads();
  auto finish = [&](int k) {
    if (!unit) {
      const double dr = Tr[k][k], di = Ti[k][k];
      const double den = dr * dr + di * di;
      const double ar = xr[k], ai = xi[k];
      xr[k] = (ar * dr + ai * di) / den;
      xi[k] = (ai * dr - ar * di) / den;
    }
  };
  if (lower) {
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      if (k < nt) {
        finish(k);
#pragma unroll
        for (int i = k + 1; i < NT; ++i)
          if (i < nt) {
            const double tr = Tr[i][k], ti = Ti[i][k];
            xr[i] -= tr * xr[k] - ti * xi[k];
            xi[i] -= tr * xi[k] + ti * xr[k];
          }
      }
    }
  } else {
#pragma unroll
    for (int k = NT - 1; k >= 0; --k) {
      if (k < nt) {
        finish(k);
#pragma unroll
        for (int i = 0; i < k; ++i) {
          const double tr = Tr[i][k], ti = Ti[i][k];
          xr[i] -= tr * xr[k] - ti * xi[k];
          xi[i] -= tr * xi[k] + ti * xr[k];
        }
      }
    }
  }
  if (act) {
#pragma unroll
    for (int i = 0; i < NT; ++i)
      if (i < nt) {
        long long off;
        if (!RIGHT) {
          const int pr = B.rows ? B.rows[i] : i;
          off = (long long)pr * B.ld + (B.cols ? B.cols[c] : c);
        } else {
          const int pr = B.rows ? B.rows[c] : c;
          off = (long long)pr * B.ld + (B.cols ? B.cols[i] : i);
        }
        B.re[off] = xr[i];
        B.im[off] = xi[i];
      }
  }
}

template <bool RIGHT>
__global__ __launch_bounds__(64) void k_ztrsm_small(int tri, int opT, int nt, int nr, ZOp T, ZOut B, int identity) {
  ztrsm_reg_body<TZ, RIGHT>(tri, opT, nt, nr, T, B, identity, blockIdx.x * 64);
}

// inverse of every TZ x TZ diagonal block of op(T), block y written on the
// diagonal of D (ld ldd) at offset TZ*y
__global__ __launch_bounds__(64) void k_ztri_inv_blocks(int tri, int opT, int n, ZOp T, double* Dre, double* Dim,
                                                       int ldd) {
  const int d = blockIdx.y * TZ;
  const int nt = min(TZ, n - d);
  ZOp Tb = T;
  const long long off = d + (T.rows ? 0 : (long long)d * T.ld);
  Tb.re = T.re + off;
  Tb.im = T.im + off;
  Tb.rows = T.rows ? T.rows + d : nullptr;
  const long long od = (long long)d * ldd + d;
  ZOut Db{Dre + od, Dim + od, ldd, nullptr, nullptr};
  ztrsm_reg_body<TZ, false>(tri, opT, nt, nt, Tb, Db, 1, 0);
}

inline ZOp zsub(ZOp T, int r, int c) {
  ZOp o = T;
  const long long off = c + (T.rows ? 0 : (long long)r * T.ld);
  o.re = T.re + off;
  o.im = T.im + off;
  o.rows = T.rows ? T.rows + r : nullptr;
  return o;
}
inline ZOp zopsub(ZOp T, int opT, int r, int c) { return opT != OP_N ? zsub(T, c, r) : zsub(T, r, c); }
inline ZOut zosub(ZOut B, int r, int c) {
  ZOut o = B;
  const long long off = (B.cols ? 0 : c) + (B.rows ? 0 : (long long)r * B.ld);
  o.re = B.re + off;
  o.im = B.im + off;
  o.rows = B.rows ? B.rows + r : nullptr;
  o.cols = B.cols ? B.cols + c : nullptr;
  return o;
}
inline ZOp zas_op(ZOut B) {
  ZOp o;
  o.re = B.re;
  o.im = B.im;
  o.ld = B.ld;
  o.rows = B.rows;
  return o;
}

// inverses of the diagonal blocks of op(T) of order nb (power of two >= TZ),
// written on the diagonal of D (n x n, ld ldd); tmp holds n*nb/4 + 64 doubles per plane (x2)
void zdinv(hipStream_t s, int tri, int opT, int n, ZOp T, int nb, double* Dre, double* Dim, int ldd, double* tmp) {
  hipLaunchKernelGGL(k_ztri_inv_blocks, dim3(1, ceil_div(n, TZ)), dim3(64), 0, s, tri, opT, n, T, Dre, Dim, ldd);
  FROB_LAUNCH_CHECK();
  const bool lower = zlower(tri);
  const int triW = lower ? TRI_LOWER : TRI_UPPER;
  const bool tT = opT != OP_N;
  const size_t half = (size_t)n * (nb / 4) + 64;
  double* tre = tmp;
  double* tim = tmp + half;
  for (int sz = TZ; 2 * sz <= nb && sz < n; sz *= 2) {
    const int st = 2 * sz;
    const int nfull = n / st;
    const long long sD = (long long)st * ldd + st;
    const long long sT = (long long)sz * sz;
    if (nfull > 0) {
      ZOp W11{Dre, Dim, ldd, nullptr};
      ZOp W22{Dre + (long long)sz * ldd + sz, Dim + (long long)sz * ldd + sz, ldd, nullptr};
      ZOut Tm{tre, tim, sz, nullptr, nullptr};
      ZOp Tmo{tre, tim, sz, nullptr};
      // stored block of op(T) at logical (r, c), stepping st along the diagonal
      auto strided = [&](int r, int c, long long& sp, int& sr) {
        const int srr = tT ? c : r, scc = tT ? r : c;
        ZOp o = zsub(T, srr, scc);
        if (T.rows) { sp = st; sr = st; }
        else { sp = (long long)st * T.ld + st; sr = 0; }
        return o;
      };
      long long sp;
      int sr;
      if (lower) {
        ZOp T21 = strided(sz, 0, sp, sr);
        gemm_z64_batched(s, opT, OP_N, sz, sz, sz, 1.0, T21, TRI_NONE, W11, triW, 0.0, Tm, false, nfull, sp, sD, sT,
                         sr, 0, 0);
        gemm_z64_batched(s, OP_N, OP_N, sz, sz, sz, -1.0, W22, triW, Tmo, TRI_NONE, 0.0,
                         ZOut{Dre + (long long)sz * ldd, Dim + (long long)sz * ldd, ldd, nullptr, nullptr}, false,
                         nfull, sD, sT, sD, 0, 0, 0);
      } else {
        ZOp T12 = strided(0, sz, sp, sr);
        gemm_z64_batched(s, opT, OP_N, sz, sz, sz, 1.0, T12, TRI_NONE, W22, triW, 0.0, Tm, false, nfull, sp, sD, sT,
                         sr, 0, 0);
        gemm_z64_batched(s, OP_N, OP_N, sz, sz, sz, -1.0, W11, triW, Tmo, TRI_NONE, 0.0,
                         ZOut{Dre + sz, Dim + sz, ldd, nullptr, nullptr}, false, nfull, sD, sT, sD, 0, 0, 0);
      }
    }
    const int r0 = nfull * st;
    if (r0 + sz < n) {
      const int s2 = n - r0 - sz;
      const long long ob = (long long)r0 * ldd + r0;
      double* Wr = Dre + ob;
      double* Wi = Dim + ob;
      ZOp W11{Wr, Wi, ldd, nullptr};
      ZOp W22{Wr + (long long)sz * ldd + sz, Wi + (long long)sz * ldd + sz, ldd, nullptr};
      if (lower) {
        gemm_z64(s, opT, OP_N, s2, sz, sz, 1.0, zopsub(T, opT, r0 + sz, r0), TRI_NONE, W11, triW, 0.0,
                 ZOut{tre, tim, sz, nullptr, nullptr});
        gemm_z64(s, OP_N, OP_N, s2, sz, s2, -1.0, W22, triW, ZOp{tre, tim, sz, nullptr}, TRI_NONE, 0.0,
                 ZOut{Wr + (long long)sz * ldd, Wi + (long long)sz * ldd, ldd, nullptr, nullptr});
      } else {
        gemm_z64(s, opT, OP_N, sz, s2, s2, 1.0, zopsub(T, opT, r0, r0 + sz), TRI_NONE, W22, triW, 0.0,
                 ZOut{tre, tim, s2, nullptr, nullptr});
        gemm_z64(s, OP_N, OP_N, sz, s2, sz, -1.0, W11, triW, ZOp{tre, tim, s2, nullptr}, TRI_NONE, 0.0,
                 ZOut{Wr + sz, Wi + sz, ldd, nullptr, nullptr});
      }
    }
  }
}

void ztrsm_rec(hipStream_t s, bool right, bool lower, int opT, int r0, int nt, int nr, ZOp T, ZOut B,
               const double* Dre, const double* Dim, int ldd) {
  if (nt <= DZ) {
    const long long od = (long long)r0 * ldd + r0;
    ZOp Di{Dre + od, Dim + od, ldd, nullptr};
    const int triD = lower ? TRI_LOWER : TRI_UPPER;
    if (!right)
      gemm_z64(s, OP_N, OP_N, nt, nr, nt, 1.0, Di, triD, zas_op(B), TRI_NONE, 0.0, B, false, GEMM_NEED_FULL_M);
    else
      gemm_z64(s, OP_N, OP_N, nr, nt, nt, 1.0, zas_op(B), TRI_NONE, Di, triD, 0.0, B, false, GEMM_NEED_FULL_N);
    return;
  }
  const int nblk = ceil_div(nt, DZ);
  const int n1 = (nblk / 2) * DZ, n2 = nt - n1;
  ZOp T21 = zopsub(T, opT, r0 + n1, r0), T12 = zopsub(T, opT, r0, r0 + n1);
  if (!right) {
    ZOut B1 = zosub(B, 0, 0), B2 = zosub(B, n1, 0);
    if (lower) {
      ztrsm_rec(s, false, lower, opT, r0, n1, nr, T, B1, Dre, Dim, ldd);
      gemm_z64(s, opT, OP_N, n2, nr, n1, -1.0, T21, TRI_NONE, zas_op(B1), TRI_NONE, 1.0, B2);
      ztrsm_rec(s, false, lower, opT, r0 + n1, n2, nr, T, B2, Dre, Dim, ldd);
    } else {
      ztrsm_rec(s, false, lower, opT, r0 + n1, n2, nr, T, B2, Dre, Dim, ldd);
      gemm_z64(s, opT, OP_N, n1, nr, n2, -1.0, T12, TRI_NONE, zas_op(B2), TRI_NONE, 1.0, B1);
      ztrsm_rec(s, false, lower, opT, r0, n1, nr, T, B1, Dre, Dim, ldd);
    }
  } else {
    ZOut B1 = zosub(B, 0, 0), B2 = zosub(B, 0, n1);
    if (lower) {
      ztrsm_rec(s, true, lower, opT, r0 + n1, n2, nr, T, B2, Dre, Dim, ldd);
      gemm_z64(s, OP_N, opT, nr, n1, n2, -1.0, zas_op(B2), TRI_NONE, T21, TRI_NONE, 1.0, B1);
      ztrsm_rec(s, true, lower, opT, r0, n1, nr, T, B1, Dre, Dim, ldd);
    } else {
      ztrsm_rec(s, true, lower, opT, r0, n1, nr, T, B1, Dre, Dim, ldd);
      gemm_z64(s, OP_N, opT, nr, n2, n1, -1.0, zas_op(B1), TRI_NONE, T12, TRI_NONE, 1.0, B2);
      ztrsm_rec(s, true, lower, opT, r0 + n1, n2, nr, T, B2, Dre, Dim, ldd);
    }
  }
}

}  // namespace

void trsm_small_z64(hipStream_t s, bool right, int tri, int opT, int nt, int nr, ZOp T, ZOut B, bool identity) {
  if (nt <= 0 || nr <= 0) return;
  if (nt > TZ) throw std::runtime_error("trsm_small_z64: triangle larger than 32");
  if (B.cols && !identity) throw std::runtime_error("trsm_small_z64: column scatter needs identity mode");
  const int grid = ceil_div(nr, 64);
  if (right)
    hipLaunchKernelGGL(k_ztrsm_small<true>, dim3(grid), dim3(64), 0, s, tri, opT, nt, nr, T, B, identity ? 1 : 0);
  else
    hipLaunchKernelGGL(k_ztrsm_small<false>, dim3(grid), dim3(64), 0, s, tri, opT, nt, nr, T, B, identity ? 1 : 0);
  FROB_LAUNCH_CHECK();
}

size_t trsm_z_work_elems(int nt) { return 2 * ((size_t)nt * nt + (size_t)nt * (DZ / 4) + 4096); }

void trsm_z64(hipStream_t s, bool right, int tri, int opT, int nt, int nr, ZOp T, ZOut B, double* work) {
  if (nt <= 0 || nr <= 0) return;
  if (nt <= TZ) {
    trsm_small_z64(s, right, tri, opT, nt, nr, T, B, false);
    return;
  }
  if (B.cols) throw std::runtime_error("trsm_z64: column scatter not supported");
  double* Dre = work;
  double* Dim = work + (size_t)nt * nt;
  double* tmp = work + 2 * (size_t)nt * nt;
  zdinv(s, tri, opT, nt, T, DZ, Dre, Dim, nt, tmp);
  ztrsm_rec(s, right, zlower(tri), opT, 0, nt, nr, T, B, Dre, Dim, nt);
}

size_t trtri_z_tmp_elems(int n) {
  int nb = TZ;
  while (nb < n) nb *= 2;
  return 2 * ((size_t)n * (nb / 4) + 64) + 4096;
}

void trtri_z64(hipStream_t s, int tri, int opT, int n, ZOp T, double* Wre, double* Wim, int ldw, double* tmp) {
  if (n <= 0) return;
  int nb = TZ;
  while (nb < n) nb *= 2;
  fill_f64(s, n, n, 0.0, Wre, ldw);
  fill_f64(s, n, n, 0.0, Wim, ldw);
  zdinv(s, tri, opT, n, T, nb, Wre, Wim, ldw, tmp);
}

}  // namespace frob
