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
__global__ __launch_bounds__(256) void k_trsm_small_f64(int tri, int trans, int nt, int nr, DOp T, DOut B,
                                                        int identity) {
  __shared__ double Ts[TS][TS + 1];
  __shared__ double Xs[TS][TS + 1];
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * TS;
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

inline int split64(int n) {
  int h = (n / 2 + TS - 1) / TS * TS;
  if (h >= n) h = n - TS;
  return h;
}

}  // namespace

void trsm_small_f64(hipStream_t s, bool right, int tri, bool trans, int nt, int nr, DOp T, DOut B, bool identity) {
  if (nt <= 0 || nr <= 0) return;
  if (nt > TS) throw std::runtime_error("trsm_small_f64: triangle larger than 64");
  if (B.cols && !identity) throw std::runtime_error("trsm_small_f64: column scatter needs identity mode");
  const int grid = ceil_div(nr, TS);
  if (right)
    hipLaunchKernelGGL(k_trsm_small_f64<true>, dim3(grid), dim3(256), 0, s, tri, trans ? 1 : 0, nt, nr, T, B,
                       identity ? 1 : 0);
  else
    hipLaunchKernelGGL(k_trsm_small_f64<false>, dim3(grid), dim3(256), 0, s, tri, trans ? 1 : 0, nt, nr, T, B,
                       identity ? 1 : 0);
  FROB_LAUNCH_CHECK();
}

void trsm_f64(hipStream_t s, bool right, int tri, bool trans, int nt, int nr, DOp T, DOut B) {
  if (nt <= 0 || nr <= 0) return;
  if (nt <= TS) {
    trsm_small_f64(s, right, tri, trans, nt, nr, T, B, false);
    return;
  }
  const int n1 = split64(nt), n2 = nt - n1;
  const bool lower = host_lower(tri);
  DOp T11 = dopsub(T, trans, 0, 0), T22 = dopsub(T, trans, n1, n1);
  DOp T21 = dopsub(T, trans, n1, 0), T12 = dopsub(T, trans, 0, n1);
  if (!right) {
    DOut B1 = osub(B, 0, 0), B2 = osub(B, n1, 0);
    if (lower) {
      trsm_f64(s, false, tri, trans, n1, nr, T11, B1);
      gemm_f64(s, trans, false, n2, nr, n1, -1.0, T21, TRI_NONE, as_op(B1), TRI_NONE, 1.0, B2);
      trsm_f64(s, false, tri, trans, n2, nr, T22, B2);
    } else {
      trsm_f64(s, false, tri, trans, n2, nr, T22, B2);
      gemm_f64(s, trans, false, n1, nr, n2, -1.0, T12, TRI_NONE, as_op(B2), TRI_NONE, 1.0, B1);
      trsm_f64(s, false, tri, trans, n1, nr, T11, B1);
    }
  } else {
    DOut B1 = osub(B, 0, 0), B2 = osub(B, 0, n1);
    if (lower) {
      trsm_f64(s, true, tri, trans, n2, nr, T22, B2);
      gemm_f64(s, false, trans, nr, n1, n2, -1.0, as_op(B2), TRI_NONE, T21, TRI_NONE, 1.0, B1);
      trsm_f64(s, true, tri, trans, n1, nr, T11, B1);
    } else {
      trsm_f64(s, true, tri, trans, n1, nr, T11, B1);
      gemm_f64(s, false, trans, nr, n2, n1, -1.0, as_op(B1), TRI_NONE, T12, TRI_NONE, 1.0, B2);
      trsm_f64(s, true, tri, trans, n2, nr, T22, B2);
    }
  }
}

void trtri_f64(hipStream_t s, int tri, bool trans, int n, DOp T, DOut W, double* tmp, int ldtmp) {
  if (n <= 0) return;
  if (n <= TS) {
    trsm_small_f64(s, false, tri, trans, n, n, T, W, true);
    return;
  }
  const int n1 = split64(n), n2 = n - n1;
  const bool lower = host_lower(tri);
  const int triW = lower ? TRI_LOWER : TRI_UPPER;   // W's diagonal is stored explicitly
  trtri_f64(s, tri, trans, n1, dopsub(T, trans, 0, 0), osub(W, 0, 0), tmp, ldtmp);
  trtri_f64(s, tri, trans, n2, dopsub(T, trans, n1, n1), osub(W, n1, n1), tmp, ldtmp);
  DOut Tm{tmp, ldtmp, nullptr, nullptr};
  DOp Tmo{tmp, ldtmp, nullptr};
  // the block of W outside the triangle is exactly zero
  {
    DOut Z = lower ? osub(W, 0, n1) : osub(W, n1, 0);
    if (Z.rows || Z.cols) throw std::runtime_error("trtri_f64: W must be a plain buffer");
    if (lower) fill_f64(s, n1, n2, 0.0, Z.p, Z.ld);
    else fill_f64(s, n2, n1, 0.0, Z.p, Z.ld);
  }
  if (lower) {
    // Tmp (n2 x n1) = T21 W11 ; W21 = -W22 Tmp
    gemm_f64(s, trans, false, n2, n1, n1, 1.0, dopsub(T, trans, n1, 0), TRI_NONE, as_op(osub(W, 0, 0)), triW, 0.0,
             Tm);
    gemm_f64(s, false, false, n2, n1, n2, -1.0, as_op(osub(W, n1, n1)), triW, Tmo, TRI_NONE, 0.0, osub(W, n1, 0));
  } else {
    // Tmp (n1 x n2) = T12 W22 ; W12 = -W11 Tmp
    gemm_f64(s, trans, false, n1, n2, n2, 1.0, dopsub(T, trans, 0, n1), TRI_NONE, as_op(osub(W, n1, n1)), triW,
             0.0, Tm);
    gemm_f64(s, false, false, n1, n2, n1, -1.0, as_op(osub(W, 0, 0)), triW, Tmo, TRI_NONE, 0.0, osub(W, 0, n1));
  }
}

}  // namespace frob
