// tri_f64.hip -- triangular solves and triangular inverses in FP64.
//
// Base case (triangle of order <= 64): one workgroup loads the triangle into
// LDS and solves for a 64-wide strip of the right-hand side by substitution,
// four threads per right-hand side (the quad substitution of tri_dev.hpp).
// Larger triangles: the 64x64 diagonal blocks are inverted by the same
// kernel (identity right-hand sides), doubled to 128 by batched GEMMs (W21 = -W22 (T21 W11) for lower,
// W12 = -W11 (T12 W22) for upper), and the solve recursion then needs only
// GEMMs.
#include "common.hpp"
#include "internal.hpp"
#include "tri_dev.hpp"

namespace frob {

namespace {

constexpr int TS = 64;   // order of the LDS-resident triangle
constexpr int LS = TS + 1;  // LDS row stride (odd: column reads are conflict-free)

__device__ __forceinline__ bool tri_is_lower(int tri) { return tri == TRI_LOWER || tri == TRI_LOWER_UNIT; }
__device__ __forceinline__ bool tri_is_unit(int tri) { return tri == TRI_LOWER_UNIT || tri == TRI_UPPER_UNIT; }

// Modes of the base-case kernel.
enum : int { SM_LEFT = 0, SM_RIGHT = 1, SM_INV = 2 };

// Base case, 256 threads, triangle of order nt <= 64:
//   SM_LEFT : B(:, strip) <- op(T)^{-1} B(:, strip)      (B is nt x nr)
//   SM_RIGHT: B(strip, :) <- B(strip, :) op(T)^{-1}      (B is nr x nt)
//   SM_INV  : D block y <- op(T_yy)^{-1}, T_yy the y-th 64x64 diagonal block
// Each is M x = b for 64 columns x at once: M = op(T) with x the columns of
// the strip (left, inverse: b = identity columns), or M = op(T)^T with x the
// rows of the strip (right).  An upper M is solved as J M J (J reverses the
// order of the first nt indices), which is lower.
template <int MODE>
__global__ __launch_bounds__(256) void k_trsm64_f64(int tri, int trans, int n, int nr, DOp T, DOut B, double* D,
                                                   int ldd) {
  __shared__ double Ls[TS * LS];
  __shared__ double rd[TS];
  const int tid = threadIdx.x;
  const bool unit = tri_is_unit(tri);
  const bool right = MODE == SM_RIGHT;
  const bool mLower = tri_is_lower(tri) != right;           // `tri` describes op(T); M = op(T)^T on the right
  const bool sT = (trans != 0) != right;                    // M(i,k) = stored(k,i)
  int nt = n, d0 = 0;
  if (MODE == SM_INV) {
    d0 = blockIdx.y * TS;
    nt = min(TS, n - d0);
  }
  auto rv = [&](int i) { return (mLower || i >= nt) ? i : nt - 1 - i; };   // solve index <-> logical index
  // Global loads: in-range (clamped) addresses, issued unconditionally in
  // unrolled batches so that they overlap; out-of-range values are replaced.
  const int wr = tid >> 6, lc = tid & 63;      // T: a wave reads stored rows wr + 4u, columns lc
  const int c = tid >> 2, g = tid & 3;         // quad layout of the solve
  const int s0 = blockIdx.x * TS;
  double tv[16], x[16];
  int prx[16];                                 // left: physical rows of x
  double* bpr = nullptr;                       // right: the strip row of this thread's x
  {
    const int cc = min(lc, nt - 1);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = min(wr + 4 * u, nt - 1);
      const int pr = T.rows ? T.rows[d0 + r] : d0 + r;
      tv[u] = T.p[(long long)pr * T.ld + d0 + cc];
    }
    if (MODE == SM_LEFT) {
      const int col = s0 + min(c, nr - 1);
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int li = min(rv(4 * m + g), nt - 1);
        prx[m] = B.rows ? B.rows[li] : li;
      }
#pragma unroll
      for (int m = 0; m < 16; ++m) x[m] = B.p[(long long)prx[m] * B.ld + col];
    } else if (MODE == SM_RIGHT) {
      const int row = s0 + min(c, nr - 1);
      bpr = B.p + (long long)(B.rows ? B.rows[row] : row) * B.ld;
#pragma unroll
      for (int m = 0; m < 16; ++m) x[m] = bpr[min(rv(4 * m + g), nt - 1)];
    }
  }
  // ---- M into LDS in solve coordinates, padded with the identity ----
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int r = wr + 4 * u, cc = lc;           // stored coordinates
    const int i = sT ? cc : r, k = sT ? r : cc;  // logical M(i, k)
    const int si = rv(i), sk = rv(k);            // solve coordinates
    const bool in = i < nt && k < nt && (sk < si || (i == k && !unit));
    Ls[si * LS + sk] = in ? tv[u] : (si == sk ? 1.0 : 0.0);
  }
  __syncthreads();
  if (tid < TS) rd[tid] = 1.0 / Ls[tid * LS + tid];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int si = 4 * m + g, li = rv(si);
    if (MODE == SM_INV) x[m] = (si == c) ? 1.0 : 0.0;
    else x[m] = (li < nt && s0 + c < nr) ? x[m] : 0.0;
  }
  __syncthreads();
  quad_lower_solve<LS>(Ls, rd, x, g, MODE == SM_INV ? (tid >> 6) * 4 : opaque_zero());

  // ---- results ----
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int si = 4 * m + g, li = rv(si);
    if (MODE == SM_INV) {
      // column c of (J M J)^{-1} is column rv(c) of M^{-1}, row si is row li
      if (li < nt && c < nt) D[(long long)(d0 + li) * ldd + d0 + rv(c)] = x[m];
    } else if (li < nt && s0 + c < nr) {
      if (MODE == SM_LEFT) B.p[(long long)prx[m] * B.ld + s0 + c] = x[m];
      else bpr[li] = x[m];
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

}  // namespace

void trsm_small_f64(hipStream_t s, bool right, int tri, bool trans, int nt, int nr, DOp T, DOut B) {
  if (nt <= 0 || nr <= 0) return;
  if (nt > TS) throw std::runtime_error("trsm_small_f64: triangle larger than 64");
  if (B.cols) throw std::runtime_error("trsm_small_f64: column scatter not supported");
  const int grid = ceil_div(nr, TS);
  if (right)
    hipLaunchKernelGGL(k_trsm64_f64<SM_RIGHT>, dim3(grid), dim3(256), 0, s, tri, trans ? 1 : 0, nt, nr, T, B,
                       (double*)nullptr, 0);
  else
    hipLaunchKernelGGL(k_trsm64_f64<SM_LEFT>, dim3(grid), dim3(256), 0, s, tri, trans ? 1 : 0, nt, nr, T, B,
                       (double*)nullptr, 0);
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
  hipLaunchKernelGGL(k_trsm64_f64<SM_INV>, dim3(1, ceil_div(n, TS)), dim3(256), 0, s, tri, trans ? 1 : 0, n, 0, T,
                     DOut{nullptr, 0, nullptr, nullptr}, D, ldd);
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
// Blocked triangular solve.  The inverses of the diagonal blocks of op(T) are
// formed first (dinv_f64); the recursion then needs only GEMMs: a leaf is
// X_b = inv(T_bb) B_b, and each inner node updates the other half's
// right-hand side with one GEMM.  Leaves of DNB = 128 are computed in place
// by one GEMM whose block row (or block column) covers the whole leaf.  Left
// solves with no row indirection on B and nr <= nt take leaves of DNB_OUT =
// 512 instead, computed out of place into a scratch block and copied back: a
// quarter of the leaf launches and of the small inner-node GEMMs.
// ------------------------------------------------------------------------
namespace {
constexpr int DNB = 128;
constexpr int DNB_OUT = 512;

void trsm_rec(hipStream_t s, bool right, bool lower, bool trans, int r0, int nt, int nr, DOp T, DOut B, const double* D,
              int ldd, int dnb, double* sx) {
  if (nt <= dnb) {
    DOp Di{D + (long long)r0 * ldd + r0, ldd, nullptr};
    const int triD = lower ? TRI_LOWER : TRI_UPPER;
    if (sx) {
      // left solve, out of place: sx = inv(T_bb) B_b (nt x nr, ld nr), then B_b = sx
      gemm_f64(s, false, false, nt, nr, nt, 1.0, Di, triD, as_op(B), TRI_NONE, 0.0, DOut{sx, nr, nullptr, nullptr});
      copy_f64(s, nt, nr, sx, nr, nullptr, B.p, B.ld);
    } else if (!right) {
      gemm_f64(s, false, false, nt, nr, nt, 1.0, Di, triD, as_op(B), TRI_NONE, 0.0, B, false, 1, 0, 0, 0,
               GEMM_NEED_FULL_M);
    } else {
      gemm_f64(s, false, false, nr, nt, nt, 1.0, as_op(B), TRI_NONE, Di, triD, 0.0, B, false, 1, 0, 0, 0,
               GEMM_NEED_FULL_N);
    }
    return;
  }
  const int nblk = ceil_div(nt, dnb);
  const int n1 = (nblk / 2) * dnb, n2 = nt - n1;
  DOp T21 = dopsub(T, trans, r0 + n1, r0), T12 = dopsub(T, trans, r0, r0 + n1);
  if (!right) {
    DOut B1 = osub(B, 0, 0), B2 = osub(B, n1, 0);
    if (lower) {
      trsm_rec(s, false, lower, trans, r0, n1, nr, T, B1, D, ldd, dnb, sx);
      gemm_f64(s, trans, false, n2, nr, n1, -1.0, T21, TRI_NONE, as_op(B1), TRI_NONE, 1.0, B2);
      trsm_rec(s, false, lower, trans, r0 + n1, n2, nr, T, B2, D, ldd, dnb, sx);
    } else {
      trsm_rec(s, false, lower, trans, r0 + n1, n2, nr, T, B2, D, ldd, dnb, sx);
      gemm_f64(s, trans, false, n1, nr, n2, -1.0, T12, TRI_NONE, as_op(B2), TRI_NONE, 1.0, B1);
      trsm_rec(s, false, lower, trans, r0, n1, nr, T, B1, D, ldd, dnb, sx);
    }
  } else {
    DOut B1 = osub(B, 0, 0), B2 = osub(B, 0, n1);
    if (lower) {
      trsm_rec(s, true, lower, trans, r0 + n1, n2, nr, T, B2, D, ldd, dnb, sx);
      gemm_f64(s, false, trans, nr, n1, n2, -1.0, as_op(B2), TRI_NONE, T21, TRI_NONE, 1.0, B1);
      trsm_rec(s, true, lower, trans, r0, n1, nr, T, B1, D, ldd, dnb, sx);
    } else {
      trsm_rec(s, true, lower, trans, r0, n1, nr, T, B1, D, ldd, dnb, sx);
      gemm_f64(s, false, trans, nr, n2, n1, -1.0, as_op(B1), TRI_NONE, T12, TRI_NONE, 1.0, B2);
      trsm_rec(s, true, lower, trans, r0 + n1, n2, nr, T, B2, D, ldd, dnb, sx);
    }
  }
}
}  // namespace

// D (nt x nt), the doubling scratch of dinv_f64 and the out-of-place leaf block
size_t trsm_work_elems(int nt) {
  return (size_t)nt * nt + (size_t)nt * (DNB_OUT / 4) + (size_t)DNB_OUT * nt + 4096;
}

void trsm_f64(hipStream_t s, bool right, int tri, bool trans, int nt, int nr, DOp T, DOut B, double* work) {
  if (nt <= 0 || nr <= 0) return;
  if (nt <= TS) {
    trsm_small_f64(s, right, tri, trans, nt, nr, T, B);
    return;
  }
  if (B.cols) throw std::runtime_error("trsm_f64: column scatter not supported");
  const bool out = !right && !B.rows && nr <= nt && nt > DNB;
  const int dnb = out ? DNB_OUT : DNB;
  double* D = work;
  double* tmp = work + (size_t)nt * nt;
  double* sx = out ? tmp + (size_t)nt * (DNB_OUT / 4) + 4096 : nullptr;
  dinv_f64(s, tri, trans, nt, T, dnb, D, nt, tmp);
  trsm_rec(s, right, host_lower(tri), trans, 0, nt, nr, T, B, D, nt, dnb, sx);
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
