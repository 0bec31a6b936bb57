// tri_f64.hip -- triangular solves and triangular inverses in FP64.
//
// The base case keeps a triangle of order <= 64 in LDS together with a
// 64-column strip of the right-hand side and runs substitution there; the
// four lanes that share a right-hand-side column sit in one wave, so a step of
// the substitution needs only wave-level ordering, not a workgroup barrier.
// Larger triangles are handled recursively: halve the triangle, solve one
// half, update the other half's right-hand side with one GEMM, solve the
// second half.  Triangular inverses use the same recursion with
// W21 = -W22 (T21 W11) (lower) or W12 = -W11 (T12 W22) (upper).
#include "common.hpp"
#include "internal.hpp"

namespace frob {

namespace {

constexpr int TS = 64;  // order of the LDS-resident triangle

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bool tri_is_lower(int tri) { return tri == TRI_LOWER || tri == TRI_LOWER_UNIT; }
__device__ __forceinline__ bool tri_is_unit(int tri) { return tri == TRI_LOWER_UNIT || tri == TRI_UPPER_UNIT; }
__device__ __forceinline__ int tri_flip(int tri) {
  switch (tri) {
    case TRI_LOWER: return TRI_UPPER;
    case TRI_LOWER_UNIT: return TRI_UPPER_UNIT;
    case TRI_UPPER: return TRI_LOWER;
    case TRI_UPPER_UNIT: return TRI_LOWER_UNIT;
    default: return tri;
  }
}

// Solve T' X' = B' for a 64-column strip, where (left side)  T' = op(T), X' = X,
// or (right side) T' = op(T)^T, X' = X^T, B' = B^T.
template <bool RIGHT>
__device__ __forceinline__ void trsm_small_body(int tri, int trans, int nt, int nr, const DOp& T, const DOut& B,
                                                int identity, int c0) {
  __shared__ double Ts[TS][TS + 1];
  __shared__ double Xs[TS][TS + 1];
  const int tid = threadIdx.x;
  const int triP = RIGHT ? tri_flip(tri) : tri;   // triangle of T'
  const bool tT = (trans != 0) != RIGHT;          // T'(i,k) = stored(k,i) if tT
  const bool lower = tri_is_lower(triP);
  const bool unit = tri_is_unit(triP);

  // T' into LDS (masked to its triangle; unit diagonal read as one)
  for (int e = tid; e < TS * TS; e += 256) {
    const int r = e / TS, cc = e % TS;          // stored coordinates (coalesced reads)
    const int i = tT ? cc : r, k = tT ? r : cc;  // logical coordinates in T'
    double v = 0.0;
    if (i < nt && k < nt) {
      const bool in = lower ? (k <= i) : (k >= i);
      if (in) {
        if (unit && i == k) v = 1.0;
        else {
          const int pr = T.rows ? T.rows[r] : r;
          v = T.p[(long long)pr * T.ld + cc];
        }
      }
    }
    Ts[i][k] = v;
  }
  // B' strip into LDS: Xs[k][c] = B'(k, c0 + c)
  for (int e = tid; e < TS * TS; e += 256) {
    int k, c;
    if (!RIGHT) { k = e / TS; c = e % TS; } else { c = e / TS; k = e % TS; }
    const int gc = c0 + c;
    double v = 0.0;
    if (k < nt && gc < nr) {
      if (identity) v = (k == gc) ? 1.0 : 0.0;
      else if (!RIGHT) {
        const int pr = B.rows ? B.rows[k] : k;
        v = B.p[(long long)pr * B.ld + gc];
      } else {
        const int pr = B.rows ? B.rows[gc] : gc;
        v = B.p[(long long)pr * B.ld + k];
      }
    }
    Xs[k][c] = v;
  }
  __syncthreads();

  // wave w owns columns [16w, 16w + 16); lane group g = lane / 16 owns rows = g (mod 4)
  const int lane = tid & 63;
  const int c = (tid >> 6) * 16 + (lane & 15);
  const int g = lane >> 4;
  if (lower) {
    for (int k = 0; k < nt; ++k) {
      if ((k & 3) == g && !unit) Xs[k][c] = Xs[k][c] / Ts[k][k];
      wave_sync();
      const double xk = Xs[k][c];
      for (int i = k + 1 + ((g - (k + 1)) & 3); i < nt; i += 4) Xs[i][c] -= Ts[i][k] * xk;
      wave_sync();
    }
  } else {
    for (int k = nt - 1; k >= 0; --k) {
      if ((k & 3) == g && !unit) Xs[k][c] = Xs[k][c] / Ts[k][k];
      wave_sync();
      const double xk = Xs[k][c];
      for (int i = g; i < k; i += 4) Xs[i][c] -= Ts[i][k] * xk;
      wave_sync();
    }
  }
  __syncthreads();

  for (int e = tid; e < TS * TS; e += 256) {
    int k, cc;
    if (!RIGHT) { k = e / TS; cc = e % TS; } else { cc = e / TS; k = e % TS; }
    const int gc = c0 + cc;
    if (k < nt && gc < nr) {
      if (!RIGHT) {
        const int pr = B.rows ? B.rows[k] : k;
        B.p[(long long)pr * B.ld + (B.cols ? B.cols[gc] : gc)] = Xs[k][cc];
      } else {
        const int pr = B.rows ? B.rows[gc] : gc;
        B.p[(long long)pr * B.ld + (B.cols ? B.cols[k] : k)] = Xs[k][cc];
      }
    }
  }
}

template <bool RIGHT>
__global__ __launch_bounds__(256) void k_trsm_small_f64(int tri, int trans, int nt, int nr, DOp T, DOut B,
                                                        int identity) {
  trsm_small_body<RIGHT>(tri, trans, nt, nr, T, B, identity, blockIdx.x * TS);
}

// Left solve op(T) X = B with a triangle of order nt <= NT held in LDS and one
// right-hand-side column per lane held in registers (x[NT], fully unrolled):
// step k finalizes x_k and subtracts T(i,k) x_k from the rows below (above);
// T(i,k) is the same for every lane, so each LDS read is a broadcast.
template <int NT>
__device__ __forceinline__ void trsm_left_reg_body(int tri, int trans, int nt, int nr, const DOp& T, const DOut& B,
                                                   int identity, int c0) {
  __shared__ double Ts[NT][NT + 1];
  const int lane = threadIdx.x;
  const bool lower = tri_is_lower(tri), unit = tri_is_unit(tri);
  for (int e = lane; e < NT * NT; e += 64) {
    const int r = e / NT, cc = e % NT;           // stored coordinates (coalesced)
    const int i = trans ? cc : r, k = trans ? r : cc;
    double v = 0.0;
    if (i < nt && k < nt && (lower ? k <= i : k >= i)) {
      if (unit && i == k) v = 1.0;
      else {
        const int pr = T.rows ? T.rows[r] : r;
        v = T.p[(long long)pr * T.ld + cc];
      }
    }
    Ts[i][k] = v;
  }
  const int c = c0 + lane;
  const bool act = c < nr;
  double x[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    double v = 0.0;
    if (i < nt && act) {
      if (identity) v = (i == c) ? 1.0 : 0.0;
      else {
        const int pr = B.rows ? B.rows[i] : i;
        v = B.p[(long long)pr * B.ld + c];
      }
    }
    x[i] = v;
  }
  __syncthreads();
  if (lower) {
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      if (k < nt) {
        if (!unit) x[k] = x[k] / Ts[k][k];
#pragma unroll
        for (int i = k + 1; i < NT; ++i)
          if (i < nt) x[i] -= Ts[i][k] * x[k];
      }
    }
  } else {
#pragma unroll
    for (int k = NT - 1; k >= 0; --k) {
      if (k < nt) {
        if (!unit) x[k] = x[k] / Ts[k][k];
#pragma unroll
        for (int i = 0; i < k; ++i) x[i] -= Ts[i][k] * x[k];
      }
    }
  }
  if (act) {
#pragma unroll
    for (int i = 0; i < NT; ++i)
      if (i < nt) {
        const int pr = B.rows ? B.rows[i] : i;
        B.p[(long long)pr * B.ld + (B.cols ? B.cols[c] : c)] = x[i];
      }
  }
}

template <int NT>
__global__ __launch_bounds__(64) void k_trsm_left_reg_f64(int tri, int trans, int nt, int nr, DOp T, DOut B,
                                                          int identity) {
  trsm_left_reg_body<NT>(tri, trans, nt, nr, T, B, identity, blockIdx.x * 64);
}

// Inverse of every 64x64 diagonal block of op(T) (order n), block y written to
// D + 64y * ldd + 64y (identity right-hand side, register-resident columns).
__global__ __launch_bounds__(64) void k_tri_inv64_reg_f64(int tri, int trans, int n, DOp T, double* D, int ldd) {
  const int d = blockIdx.y * TS;
  const int nt = min(TS, n - d);
  DOp Tb = T;
  Tb.p = T.p + d + (T.rows ? 0 : (long long)d * T.ld);
  Tb.rows = T.rows ? T.rows + d : nullptr;
  DOut Db{D + (long long)d * ldd + d, ldd, nullptr, nullptr};
  trsm_left_reg_body<TS>(tri, trans, nt, nt, Tb, Db, 1, 0);
}

inline bool host_lower(int tri) { return tri == TRI_LOWER || tri == TRI_LOWER_UNIT; }

// sub-block helpers: operand block starting at logical (r, c) of the stored matrix
inline DOp dsub(DOp T, int r, int c) {
  DOp o = T;
  o.p = T.p + c + (T.rows ? 0 : (long long)r * T.ld);
  o.rows = T.rows ? T.rows + r : nullptr;
  return o;
}
// block of op(T) at logical (r, c)
inline DOp dopsub(DOp T, bool trans, int r, int c) { return trans ? dsub(T, c, r) : dsub(T, r, c); }
inline DOut osub(DOut B, int r, int c) {
  DOut o = B;
  o.p = B.p + (B.cols ? 0 : c) + (B.rows ? 0 : (long long)r * B.ld);
  o.rows = B.rows ? B.rows + r : nullptr;
  o.cols = B.cols ? B.cols + c : nullptr;
  return o;
}
inline DOp as_op(DOut B) {
  DOp o;
  o.p = B.p;
  o.ld = B.ld;
  o.rows = B.rows;
  return o;
}

}  // namespace

void trsm_small_f64(hipStream_t s, bool right, int tri, bool trans, int nt, int nr, DOp T, DOut B, bool identity) {
  if (nt <= 0 || nr <= 0) return;
  if (nt > TS) throw std::runtime_error("trsm_small_f64: triangle larger than 64");
  if (B.cols && !identity) throw std::runtime_error("trsm_small_f64: column scatter needs identity mode");
  const int grid = ceil_div(nr, TS);
  if (right) {
    hipLaunchKernelGGL(k_trsm_small_f64<true>, dim3(grid), dim3(256), 0, s, tri, trans ? 1 : 0, nt, nr, T, B,
                       identity ? 1 : 0);
  } else if (nt <= 16) {
    hipLaunchKernelGGL(k_trsm_left_reg_f64<16>, dim3(grid), dim3(64), 0, s, tri, trans ? 1 : 0, nt, nr, T, B,
                       identity ? 1 : 0);
  } else if (nt <= 32) {
    hipLaunchKernelGGL(k_trsm_left_reg_f64<32>, dim3(grid), dim3(64), 0, s, tri, trans ? 1 : 0, nt, nr, T, B,
                       identity ? 1 : 0);
  } else {
    hipLaunchKernelGGL(k_trsm_left_reg_f64<64>, dim3(grid), dim3(64), 0, s, tri, trans ? 1 : 0, nt, nr, T, B,
                       identity ? 1 : 0);
  }
  FROB_LAUNCH_CHECK();
}

// ------------------------------------------------------------------------
// Diagonal-block inverses.  Level 0 inverts all 64x64 diagonal blocks in one
// launch; each further level doubles the block order with two batched GEMMs
// over all blocks of that level (uniform stride along the diagonal):
//   lower:  W21 = -W22 (T21 W11)      upper:  W12 = -W11 (T12 W22)
// ------------------------------------------------------------------------
namespace {

// stored-block operand at logical op(T) block (r, c), batched along the diagonal
// with step `st` (in logical rows/cols) -> (pointer stride, rows stride)
struct Strided {
  DOp op;
  long long sp;
  int sr;
};
inline Strided diag_strided(DOp T, bool trans, int r, int c, int st) {
  const int sr = trans ? c : r, sc = trans ? r : c;  // stored coordinates
  Strided o;
  o.op = dsub(T, sr, sc);
  if (T.rows) { o.sp = st; o.sr = st; }
  else { o.sp = (long long)st * T.ld + st; o.sr = 0; }
  return o;
}

}  // namespace

void dinv_f64(hipStream_t s, int tri, bool trans, int n, DOp T, int nb, double* D, int ldd, double* tmp) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_tri_inv64_reg_f64, dim3(1, ceil_div(n, TS)), dim3(64), 0, s, tri, trans ? 1 : 0, n, T, D, ldd);
  FROB_LAUNCH_CHECK();
  const bool lower = host_lower(tri);
  const int triW = lower ? TRI_LOWER : TRI_UPPER;
  for (int sz = TS; 2 * sz <= nb && sz < n; sz *= 2) {
    const int st = 2 * sz;
    const int nfull = n / st;
    const long long sD = (long long)st * ldd + st;
    // full parents: z = 0 .. nfull-1 at diagonal offset r0 = st * z
    if (nfull > 0) {
      DOp W11{D, ldd, nullptr}, W22{D + (long long)sz * ldd + sz, ldd, nullptr};
      DOut Tm{tmp, sz, nullptr, nullptr};
      DOp Tmo{tmp, sz, nullptr};
      const long long sT = (long long)sz * sz;
      if (lower) {
        Strided T21 = diag_strided(T, trans, sz, 0, st);
        gemm_f64_batched(s, trans, false, sz, sz, sz, 1.0, T21.op, TRI_NONE, W11, triW, 0.0, Tm, false, nfull, T21.sp,
                         sD, sT, T21.sr, 0, 0);
        gemm_f64_batched(s, false, false, sz, sz, sz, -1.0, W22, triW, Tmo, TRI_NONE, 0.0,
                         DOut{D + (long long)sz * ldd, ldd, nullptr, nullptr}, false, nfull, sD, sT, sD, 0, 0, 0);
      } else {
        Strided T12 = diag_strided(T, trans, 0, sz, st);
        gemm_f64_batched(s, trans, false, sz, sz, sz, 1.0, T12.op, TRI_NONE, W22, triW, 0.0, Tm, false, nfull, T12.sp,
                         sD, sT, T12.sr, 0, 0);
        gemm_f64_batched(s, false, false, sz, sz, sz, -1.0, W11, triW, Tmo, TRI_NONE, 0.0,
                         DOut{D + sz, ldd, nullptr, nullptr}, false, nfull, sD, sT, sD, 0, 0, 0);
      }
    }
    // trailing parent with a partial second child
    const int r0 = nfull * st;
    if (r0 + sz < n) {
      const int s2 = n - r0 - sz;
      double* Wb = D + (long long)r0 * ldd + r0;
      DOp W11{Wb, ldd, nullptr}, W22{Wb + (long long)sz * ldd + sz, ldd, nullptr};
      if (lower) {
        gemm_f64(s, trans, false, s2, sz, sz, 1.0, dopsub(T, trans, r0 + sz, r0), TRI_NONE, W11, triW, 0.0,
                 DOut{tmp, sz, nullptr, nullptr});
        gemm_f64(s, false, false, s2, sz, s2, -1.0, W22, triW, DOp{tmp, sz, nullptr}, TRI_NONE, 0.0,
                 DOut{Wb + (long long)sz * ldd, ldd, nullptr, nullptr});
      } else {
        gemm_f64(s, trans, false, sz, s2, s2, 1.0, dopsub(T, trans, r0, r0 + sz), TRI_NONE, W22, triW, 0.0,
                 DOut{tmp, s2, nullptr, nullptr});
        gemm_f64(s, false, false, sz, s2, sz, -1.0, W11, triW, DOp{tmp, s2, nullptr}, TRI_NONE, 0.0,
                 DOut{Wb + sz, ldd, nullptr, nullptr});
      }
    }
  }
}

// ------------------------------------------------------------------------
// Blocked triangular solve.  The inverses of the 128x128 diagonal blocks of
// op(T) are formed first (dinv_f64); the recursion then needs only GEMMs: a
// leaf is X_b = inv(T_bb) B_b computed in place by one GEMM whose block row
// (or block column) covers the whole leaf, and each inner node updates the
// other half's right-hand side with one GEMM.
// ------------------------------------------------------------------------
namespace {
constexpr int DNB = 128;

void trsm_rec(hipStream_t s, bool right, bool lower, bool trans, int r0, int nt, int nr, DOp T, DOut B, const double* D,
              int ldd) {
  if (nt <= DNB) {
    DOp Di{D + (long long)r0 * ldd + r0, ldd, nullptr};
    const int triD = lower ? TRI_LOWER : TRI_UPPER;
    if (!right)
      gemm_f64(s, false, false, nt, nr, nt, 1.0, Di, triD, as_op(B), TRI_NONE, 0.0, B, false, 1, 0, 0, 0,
               GEMM_NEED_FULL_M);
    else
      gemm_f64(s, false, false, nr, nt, nt, 1.0, as_op(B), TRI_NONE, Di, triD, 0.0, B, false, 1, 0, 0, 0,
               GEMM_NEED_FULL_N);
    return;
  }
  const int nblk = ceil_div(nt, DNB);
  const int n1 = (nblk / 2) * DNB, n2 = nt - n1;
  DOp T21 = dopsub(T, trans, r0 + n1, r0), T12 = dopsub(T, trans, r0, r0 + n1);
  if (!right) {
    DOut B1 = osub(B, 0, 0), B2 = osub(B, n1, 0);
    if (lower) {
      trsm_rec(s, false, lower, trans, r0, n1, nr, T, B1, D, ldd);
      gemm_f64(s, trans, false, n2, nr, n1, -1.0, T21, TRI_NONE, as_op(B1), TRI_NONE, 1.0, B2);
      trsm_rec(s, false, lower, trans, r0 + n1, n2, nr, T, B2, D, ldd);
    } else {
      trsm_rec(s, false, lower, trans, r0 + n1, n2, nr, T, B2, D, ldd);
      gemm_f64(s, trans, false, n1, nr, n2, -1.0, T12, TRI_NONE, as_op(B2), TRI_NONE, 1.0, B1);
      trsm_rec(s, false, lower, trans, r0, n1, nr, T, B1, D, ldd);
    }
  } else {
    DOut B1 = osub(B, 0, 0), B2 = osub(B, 0, n1);
    if (lower) {
      trsm_rec(s, true, lower, trans, r0 + n1, n2, nr, T, B2, D, ldd);
      gemm_f64(s, false, trans, nr, n1, n2, -1.0, as_op(B2), TRI_NONE, T21, TRI_NONE, 1.0, B1);
      trsm_rec(s, true, lower, trans, r0, n1, nr, T, B1, D, ldd);
    } else {
      trsm_rec(s, true, lower, trans, r0, n1, nr, T, B1, D, ldd);
      gemm_f64(s, false, trans, nr, n2, n1, -1.0, as_op(B1), TRI_NONE, T12, TRI_NONE, 1.0, B2);
      trsm_rec(s, true, lower, trans, r0 + n1, n2, nr, T, B2, D, ldd);
    }
  }
}
}  // namespace

size_t trsm_work_elems(int nt) { return (size_t)nt * nt + (size_t)nt * (DNB / 4) + 4096; }

void trsm_f64(hipStream_t s, bool right, int tri, bool trans, int nt, int nr, DOp T, DOut B, double* work) {
  if (nt <= 0 || nr <= 0) return;
  if (nt <= TS) {
    trsm_small_f64(s, right, tri, trans, nt, nr, T, B, false);
    return;
  }
  if (B.cols) throw std::runtime_error("trsm_f64: column scatter not supported");
  double* D = work;
  double* tmp = work + (size_t)nt * nt;
  dinv_f64(s, tri, trans, nt, T, DNB, D, nt, tmp);
  trsm_rec(s, right, host_lower(tri), trans, 0, nt, nr, T, B, D, nt);
}

size_t trtri_tmp_elems(int n) {
  int nb = TS;
  while (nb < n) nb *= 2;
  return (size_t)n * (nb / 4) + 4096;
}

void trtri_f64(hipStream_t s, int tri, bool trans, int n, DOp T, double* W, int ldw, double* tmp) {
  if (n <= 0) return;
  int nb = TS;
  while (nb < n) nb *= 2;
  fill_f64(s, n, n, 0.0, W, ldw);
  dinv_f64(s, tri, trans, n, T, nb, W, ldw, tmp);
}

}  // namespace frob
