// lu_f64.hip -- LU factorization with partial pivoting (GEPP) in FP64.
//
// Recursive column splitting: factor the left half, solve U12 = L11^{-1} A12,
// update A22 -= L21 U12 with one matrix-core GEMM, factor the right half.  The
// recursion stops at a "leaf" panel narrow enough to live in the registers of
// one workgroup of 512 or 1024 threads (rows-per-thread x columns <= 32
// doubles per thread and block), where the pivot search is a DPP
// max-reduction per wave followed by a reduction over the waves' slots, with
// the lowest row index winning ties.
//
// Pivoting never moves data: rows are addressed through the index array perm
// (logical row i of P A lives in physical row perm[i]), so a row interchange
// is a swap of two integers and the stored multipliers of earlier columns
// follow automatically.  An exactly-zero pivot column is recorded in *info
// (1-based, first occurrence) and factoring continues, as LAPACK does.
#include <algorithm>
#include <climits>

#include "common.hpp"
#include "devutil.hpp"
#include "handle.hpp"
#include "internal.hpp"
#include "tri_dev.hpp"

namespace frob {

namespace {

constexpr int LEAF_NT = 512;        // threads of the leaf workgroup (twice that for 513 .. 4096 rows)

// One workgroup of NT threads factors an mm x nc panel (nc <= W) held in
// registers.  Thread t owns panel rows q = t + s * NT (s < R).  Rows never move: each row
// carries its current logical position pos (GEPP's row interchanges act on
// these integers only), so a pivot step exchanges no data between threads.
// Per column j:
//   - every lane takes its best candidate (largest |a_qj| among rows with
//     pos >= j, lowest pos on ties) by an integer maximum over FP32 images of
//     |a_qj| (rounding is monotone, so the exact maximum is among the rows
//     that attain the largest image; exact FP64 comparison only when several
//     rows of one lane attain it);
//   - the wave maximum of the images is found with single-instruction DPP
//     steps; a ballot then settles the winner exactly in FP64 (one lane in the
//     usual case, an exact FP64 comparison among the tied lanes otherwise);
//   - the wave's winner writes (|value|, pos, row) to a parity-double-
//     buffered LDS slot; one barrier; every wave reduces the eight slots the
//     same way and reads the pivot row from the winning slot;
//   - positions are exchanged and every row below is scaled and updated
//     (branch-free: rows above are updated with a zero multiplier).
// Each thread reads and writes its own rows straight from and to HBM (rows
// are scattered through perm, so a row's W contiguous doubles are its own
// memory transactions either way): one batch of unconditional loads at
// clamped addresses, one memory latency per panel.
//
// With n2 > 0 the kernel factors a whole bottom recursion node: after its nc
// columns it loads the n2 <= W columns to the right, applies the
// factorization to them (U12 = L11^{-1} A12 by substitution, A22 -= L21 U12
// with L21 still in registers) and factors them as panel columns nc .. nc+n2.
// the fused sibling update needs a second R x W block of registers; the
// tallest leaves (more than 16 rows per thread) leave it to a node kernel
constexpr bool LEAF_SIBLING(int R) { return R <= 16; }
// leaves whose panel and sibling blocks are written back together through LDS
constexpr bool LEAF_JOINT_STORE(int W) { return W <= 8; }

template <int R, int W, int NT = LEAF_NT>
__global__ __launch_bounds__(NT) void k_lu_leaf_f64(double* __restrict__ a, int lda, int* __restrict__ perm, int k0,
                                                    int mm, int nc, int n2, int* info, int* __restrict__ snap,
                                                    int sfrom) {
  constexpr int NW = NT / 64;
  static_assert(W % 2 == 0 && NW <= 16, "leaf shape");
  __shared__ double s_cv[2][NW];
  __shared__ int s_ck[2][NW];
  __shared__ __align__(16) double s_crow[2][NW][W];
  __shared__ double s_l[W][W + 1];
  __shared__ double s_u[W][W + 1];
  // staging of the joint write-back (row pitch 2W + 2 doubles: 16-byte aligned
  // rows, consecutive rows on different banks)
  __shared__ __align__(16) double s_st[LEAF_JOINT_STORE(W) ? NW : 1][64][LEAF_JOINT_STORE(W) ? 2 * W + 2 : 2];
  __shared__ int s_sph[LEAF_JOINT_STORE(W) ? NW : 1][64];

  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const bool vbase = ((lda & 1) == 0) && ((reinterpret_cast<uintptr_t>(a) & 15) == 0);

  // ---- this thread's rows q = t + s NT: physical row ph, logical position pos
  //      (padding rows q >= mm: pos -1, never candidates, never stored) ----
  int ph[R], pos[R];
#pragma unroll
  for (int s = 0; s < R; ++s) ph[s] = perm[k0 + min(t + s * NT, mm - 1)];
#pragma unroll
  for (int s = 0; s < R; ++s) pos[s] = t + s * NT < mm ? t + s * NT : -1;

  // Columns col0 .. col0 + ncol - 1 of this thread's rows, straight from HBM:
  // one batch of unconditional loads at clamped addresses (16-byte pairs
  // when rows are 16-byte aligned and the extent is even), columns beyond
  // ncol zeroed afterwards.
  auto load_rows = [&](double (&x)[R][W], int col0, int ncol, bool mask = true) {
    if (vbase && ((col0 | ncol) & 1) == 0) {
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const double* row = a + (long long)ph[s] * lda + col0;
#pragma unroll
        for (int c = 0; c < W; c += 2) {
          const double2 y = *reinterpret_cast<const double2*>(row + min(c, ncol - 2));
          x[s][c] = y.x;
          x[s][c + 1] = y.y;
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const double* row = a + (long long)ph[s] * lda + col0;
#pragma unroll
        for (int c = 0; c < W; ++c) x[s][c] = row[min(c, ncol - 1)];
      }
    }
    if (mask) {
#pragma unroll
      for (int s = 0; s < R; ++s)
#pragma unroll
        for (int c = 0; c < W; ++c) x[s][c] = c < ncol ? x[s][c] : 0.0;
    }
  };
  auto store_rows = [&](const double (&x)[R][W], int col0, int ncol) {
    const bool vec = vbase && ((col0 | ncol) & 1) == 0;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      if (pos[s] < 0) continue;
      double* row = a + (long long)ph[s] * lda + col0;
      if (vec) {
#pragma unroll
        for (int c = 0; c < W; c += 2)
          if (c < ncol) *reinterpret_cast<double2*>(row + c) = make_double2(x[s][c], x[s][c + 1]);
      } else {
#pragma unroll
        for (int c = 0; c < W; ++c)
          if (c < ncol) row[c] = x[s][c];
      }
    }
  };

  double v[R][W], x[R][W];
  // panel and sibling block together: row segments of W + n2 columns
  const bool joint = LEAF_SIBLING(R) && n2 > 0 && nc == W && vbase && ((k0 | n2) & 1) == 0;
  if (LEAF_JOINT_STORE(W) && joint) {
    // Joint row segments read transposed: W consecutive lanes fetch one row's
    // W + n2 contiguous columns (16 bytes each, so a load instruction touches
    // 64 / W row segments instead of 64), staged per slot through LDS into
    // the row-per-thread layout.  All loads are issued before the first is
    // staged; columns past n2 are masked when first used.
    if constexpr (LEAF_JOINT_STORE(W)) {
      constexpr int RPI = 64 / W;
      const int m = lane % W;
      const int cm = k0 + min(2 * m, W + n2 - 2);
      double y0[R][W], y1[R][W];
#pragma unroll
      for (int s = 0; s < R; ++s)
#pragma unroll
        for (int i = 0; i < W; ++i) {
          const int prow = __shfl(ph[s], i * RPI + lane / W);
          const double2 t2 = *reinterpret_cast<const double2*>(a + (long long)prow * lda + cm);
          y0[s][i] = t2.x;
          y1[s][i] = t2.y;
        }
#pragma unroll
      for (int s = 0; s < R; ++s) {
        __builtin_amdgcn_sched_barrier(0);   // one slot at a time (register pressure)
        __syncthreads();   // the previous slot's staged rows have been read
#pragma unroll
        for (int i = 0; i < W; ++i)
          *reinterpret_cast<double2*>(&s_st[wv][i * RPI + lane / W][2 * m]) = make_double2(y0[s][i], y1[s][i]);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < W; c += 2) {
          const double2 p = *reinterpret_cast<const double2*>(&s_st[wv][lane][c]);
          const double2 q = *reinterpret_cast<const double2*>(&s_st[wv][lane][W + c]);
          v[s][c] = p.x; v[s][c + 1] = p.y;
          x[s][c] = q.x; x[s][c + 1] = q.y;
        }
      }
    }
  } else if (joint) {
    // The sibling's columns continue this thread's row segments: they are
    // fetched now, each row's pairs right after the panel's, so both halves
    // of a row come from the cache line its first load brought in (a row is
    // its own line; the line fetches, not the bytes, bound this load).  They
    // stay in flight during the first half and are masked when first used.
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const double* row = a + (long long)ph[s] * lda + k0;
#pragma unroll
      for (int c = 0; c < W; c += 2) {
        const double2 y = *reinterpret_cast<const double2*>(row + c);
        v[s][c] = y.x;
        v[s][c + 1] = y.y;
      }
#pragma unroll
      for (int c = 0; c < W; c += 2) {
        const double2 y = *reinterpret_cast<const double2*>(row + W + min(c, n2 - 2));
        x[s][c] = y.x;
        x[s][c + 1] = y.y;
      }
    }
  } else {
    load_rows(v, k0, nc);
    // the sibling's columns are fetched now and stay in flight during the
    // first half (masked when first used, so nothing waits on them before)
    if (LEAF_SIBLING(R) && n2 > 0) load_rows(x, k0 + nc, n2, false);
  }

  // ---- factor ----
  int first_zero = 0;
  // One column step: register column jj (compile time, so every register
  // index is static) of block x, panel column jp = off + jj.
  auto column = [&](double (&x)[R][W], auto jc, int off, int ncols) __attribute__((always_inline)) {
    constexpr int jj = decltype(jc)::value;
    if (jj >= ncols) return;  // uniform
    const int jp = off + jj;
    constexpr int par = jj & 1;
    // FP32 image of |a_qj| as an integer key (-1: not a candidate; NaN never
    // is); the conversion is monotone, so the exact maximum is among the rows
    // that attain the largest key
    auto key = [&](int s) {
      const double xv = fabs(x[s][jj]);
      return (pos[s] >= jp && xv == xv) ? __float_as_int((float)xv) : -1;
    };
    int kmax = key(0);
#pragma unroll
    for (int s = 1; s < R; ++s) kmax = max(kmax, key(s));
    double best = -1.0;
    int bq = INT_MAX, nt = 0;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const bool m = kmax >= 0 && key(s) == kmax;
      best = m ? fabs(x[s][jj]) : best;
      bq = m ? pos[s] : bq;
      nt += m ? 1 : 0;
    }
    if (R > 1 && __ballot(nt > 1)) {
      // several rows of a lane share the largest key: exact comparison
      best = -1.0;
      bq = INT_MAX;
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const double xv = fabs(x[s][jj]);
        const bool ok = kmax >= 0 && key(s) == kmax && (xv > best || (xv == best && pos[s] < bq));
        best = ok ? xv : best;
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
            for (int c = 0; c < W; c += 2)
              *reinterpret_cast<double2*>(&s_crow[par][wv][c]) = make_double2(x[s][c], x[s][c + 1]);
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
    const double* prow;
    if (gmf >= 0) {
      const unsigned long long tied = __ballot(lane < NW && sf == gmf);
      const int gw = (__popcll(tied) == 1) ? __ffsll((long long)tied) - 1 : exact_argmax(tied, sv, sk);
      p = __builtin_amdgcn_readlane(sk, gw);
      prow = s_crow[par][gw];
    } else {
      // every candidate is NaN: keep row jp in place (uniform slow path)
      p = jp;
#pragma unroll
      for (int s = 0; s < R; ++s)
        if (pos[s] == jp) {
#pragma unroll
          for (int c = 0; c < W; ++c) s_crow[par][0][c] = x[s][c];
        }
      __syncthreads();
      prow = s_crow[par][0];
    }
    // row interchange jp <-> p on the positions only
#pragma unroll
    for (int s = 0; s < R; ++s) pos[s] = pos[s] == p ? jp : (pos[s] == jp ? p : pos[s]);
    const double piv = prow[jj];
    if (piv == 0.0 && !first_zero) first_zero = k0 + jp + 1;
    // scale by the reciprocal unless it would overflow (as LAPACK's getf2
    // does); a zero pivot leaves the (all-zero) column and the rows as they are
    const bool nz = piv != 0.0;
    double pr[W];
#pragma unroll
    for (int c = jj + 1; c < W; ++c) pr[c] = prow[c];
    auto update = [&](auto scale) {
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const bool below = nz && pos[s] > jp;
        const double q = scale(x[s][jj]);
        const double l = below ? q : 0.0;
        x[s][jj] = below ? q : x[s][jj];
#pragma unroll
        for (int c = jj + 1; c < W; ++c) x[s][c] = fma(-l, pr[c], x[s][c]);
      }
    };
    if (fabs(piv) >= 2.2250738585072014e-308) {   // uniform
      const double rp = 1.0 / piv;
      update([rp](double x) { return x * rp; });
    } else {
      update([piv](double x) { return x / piv; });
    }
  };
  StaticFor<0, W>::run([&](auto jc) __attribute__((always_inline)) { column(v, jc, 0, nc); });
  if (!(LEAF_JOINT_STORE(W) && joint)) store_rows(v, k0, nc);

  if (LEAF_SIBLING(R) && n2 > 0) {
    // ---- sibling update: columns cs .. cs + n2 - 1 ----
    const int cs = k0 + nc;
#pragma unroll
    for (int s = 0; s < R; ++s)
#pragma unroll
      for (int c = 0; c < W; ++c) x[s][c] = c < n2 ? x[s][c] : 0.0;
#pragma unroll
    for (int s = 0; s < R; ++s)
      if (pos[s] >= 0 && pos[s] < nc) {
        const int i = pos[s];
#pragma unroll
        for (int k = 0; k < W; ++k) s_l[i][k] = v[s][k];
#pragma unroll
        for (int c = 0; c < W; ++c) s_u[i][c] = x[s][c];
      }
    __syncthreads();
    if (t < n2) {
      // U12 = L11^{-1} A12, column t, by substitution in registers
      double u[W];
#pragma unroll
      for (int i = 0; i < W; ++i) u[i] = s_u[i][t];
#pragma unroll
      for (int i = 0; i < W; ++i) u[i] = i < nc ? u[i] : 0.0;
      StaticFor<1, W>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if (i >= nc) return;  // uniform
        double acc = u[i];
#pragma unroll
        for (int k = 0; k < i; ++k) acc = fma(-s_l[i][k], u[k], acc);
        u[i] = acc;
      });
#pragma unroll
      for (int i = 0; i < W; ++i)
        if (i < nc) s_u[i][t] = u[i];
    }
    __syncthreads();
    // A22 -= L21 U12, one row of U12 at a time (the scheduling barrier keeps
    // the LDS reads of later rows from being hoisted into registers)
    StaticFor<0, W>::run([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      if (k >= nc) return;  // uniform
      __builtin_amdgcn_sched_barrier(0);
      double u[W];
#pragma unroll
      for (int c = 0; c < W; ++c) u[c] = s_u[k][c];
#pragma unroll
      for (int s = 0; s < R; ++s)
#pragma unroll
        for (int c = 0; c < W; ++c) x[s][c] = fma(-v[s][k], u[c], x[s][c]);
    });
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const bool top = pos[s] >= 0 && pos[s] < nc;
      const int pi = top ? pos[s] : 0;
#pragma unroll
      for (int c = 0; c < W; ++c) {
        const double uv = s_u[pi][c];
        x[s][c] = top ? uv : x[s][c];
      }
    }
    // ---- factor the sibling's columns too (panel columns nc .. nc + n2) ----
    StaticFor<0, W>::run([&](auto jc) __attribute__((always_inline)) { column(x, jc, nc, n2); });
    if constexpr (LEAF_JOINT_STORE(W)) {
      if (joint) {
        // Both blocks are written back together, transposed through LDS so
        // that W consecutive lanes write one row's W + n2 contiguous columns
        // (16 bytes each): a store instruction then touches 64 / W row
        // segments instead of 64, and the store rate is set by the segments
        // touched.  Each wave stages its own 64 rows per slot s.
#pragma unroll
        for (int s = 0; s < R; ++s) {
          __syncthreads();   // the previous slot's staged rows have been read
          double* rb = &s_st[wv][lane][0];
#pragma unroll
          for (int c = 0; c < W; c += 2) *reinterpret_cast<double2*>(rb + c) = make_double2(v[s][c], v[s][c + 1]);
#pragma unroll
          for (int c = 0; c < W; c += 2)
            *reinterpret_cast<double2*>(rb + W + c) = make_double2(x[s][c], x[s][c + 1]);
          s_sph[wv][lane] = pos[s] >= 0 ? ph[s] : -1;
          __syncthreads();
          constexpr int RPI = 64 / W;   // rows per store instruction
          const int m = lane % W;       // 16-byte chunk of the row segment
#pragma unroll
          for (int i = 0; i < W; ++i) {
            const int r = i * RPI + lane / W;
            const double2 y = *reinterpret_cast<const double2*>(&s_st[wv][r][2 * m]);
            const int prow = s_sph[wv][r];
            if (prow >= 0 && 2 * m < W + n2) *reinterpret_cast<double2*>(a + (long long)prow * lda + k0 + 2 * m) = y;
          }
        }
      } else {
        store_rows(x, cs, n2);
      }
    } else {
      store_rows(x, cs, n2);
    }
  }
  if (t == 0 && first_zero && *info == 0) *info = first_zero;

  // ---- the new row order ----
#pragma unroll
  for (int s = 0; s < R; ++s)
    if (pos[s] >= 0) {
      perm[k0 + pos[s]] = ph[s];
      // copy of the trailing row order from position sfrom on (look-ahead)
      if (snap && k0 + pos[s] >= sfrom) snap[k0 + pos[s] - sfrom] = ph[s];
    }
}

// widest leaf for a panel with mm rows (R * W <= 32 doubles per thread keeps
// the panel, the prefetched sibling block and the pivot row within 256 VGPRs)
inline int leaf_width(int mm) {
  const int R = ceil_div(mm, LEAF_NT);
  if (R <= 1) return 32;
  if (R <= 2) return 16;
  if (R <= 4) return 8;
  if (R <= 8) return 4;
  if (R <= 32) return 2;
  return 0;
}

void launch_leaf(hipStream_t s, double* a, int lda, int* perm, int k0, int mm, int nc, int n2, int* info,
                 int* snap = nullptr, int sfrom = 0) {
  const int R = ceil_div(mm, LEAF_NT);
  if (nc > leaf_width(mm) || n2 > leaf_width(mm)) throw std::runtime_error("getrf_f64: leaf wider than its template");
  if (n2 > 0 && !LEAF_SIBLING(R)) throw std::runtime_error("getrf_f64: no fused sibling update for this leaf");
  // 1024 threads for 513 .. 4096 rows (half the rows per thread of a 512-thread
  // leaf of the same width), 512 otherwise
  void (*kern)(double*, int, int*, int, int, int, int, int*, int*, int);
  int threads = 2 * LEAF_NT;
  if (R <= 1) { kern = k_lu_leaf_f64<1, 32>; threads = LEAF_NT; }
  else if (R <= 2) kern = k_lu_leaf_f64<1, 16, 2 * LEAF_NT>;
  else if (R <= 4) kern = k_lu_leaf_f64<2, 8, 2 * LEAF_NT>;
  else if (R <= 8) kern = k_lu_leaf_f64<4, 4, 2 * LEAF_NT>;
  else if (R <= 16) { kern = k_lu_leaf_f64<16, 2>; threads = LEAF_NT; }
  else if (R <= 32) { kern = k_lu_leaf_f64<32, 2>; threads = LEAF_NT; }
  else throw std::runtime_error("getrf_f64: matrix order above 16384 is not supported");
  hipLaunchKernelGGL(kern, dim3(1), dim3(threads), 0, s, a, lda, perm, k0, mm, nc, n2, info, snap, sfrom);
  FROB_LAUNCH_CHECK();
}

// Internal recursion node with n1, n2 <= NB (16, 32 or 64) in one launch
// (replaces a triangular-solve launch and a GEMM launch): every workgroup
// solves U12 = L11^{-1} A12 (quad substitution on an LDS copy of the unit
// lower L11), then updates its 64 rows of A22 -= L21 U12.  A12 may be
// overwritten with U12 only after every workgroup has read it: the workgroups
// count themselves on *cnt and the last one writes U12 and resets the counter.
constexpr int NODE_MAX = 64;
constexpr int NODE_ROWS = 64;   // rows of A22 per workgroup
constexpr int NODE_RI = NODE_ROWS / 16;   // rows per thread in the product
template <int NB>
__global__ __launch_bounds__(256) void k_lu_node_f64(double* __restrict__ a, int lda, const int* __restrict__ perm,
                                                     int k0, int mm, int n1, int n2, int* cnt) {
  constexpr int LD = NB + 1;
  constexpr int TPR = 256 / NB;               // rows per pass of the NB-wide element mapping
  constexpr int PL = NB * NB / 256;           // L11 / U12 elements per thread
  constexpr int PB = NODE_ROWS * NB / 256;    // L21 / A22 elements per thread
  constexpr int QB = NB / 4;                  // blocks of four rows in the solve
  static_assert(PL >= 1 && NB % 4 == 0, "node shape");
  __shared__ double Ls[NODE_ROWS * LD];       // L11, then the block of L21
  __shared__ double Us[NB * LD];              // U12
  __shared__ double rd[NB];
  __shared__ int s_last;
  const int tid = threadIdx.x;
  const int cs = k0 + n1;                     // first column of A12 / A22
  const int r0 = n1 + blockIdx.x * NODE_ROWS; // this workgroup's first row of L21 / A22
  const int er = tid / NB, ec = tid % NB;     // element (er + TPR u, ec)
  const int c = tid >> 2, g = tid & 3;        // quad layout of the solve
  // Every global load has an in-range (clamped) address and is issued
  // unconditionally in one batch, so the loads overlap (one memory latency);
  // out-of-range values are replaced afterwards.  L21 and A22 are fetched up
  // front and wait in registers while U12 is solved.
  // the product: thread (ti, tj) owns rows ti + 16 i (i < NODE_RI), columns tj + 16 j (j < CJ)
  constexpr int CJ = NB / 16;
  const int ti = tid >> 4, tj = tid & 15;
  int pl[PL], pb[PB], px[QB], qr[NODE_RI];
#pragma unroll
  for (int u = 0; u < PL; ++u) pl[u] = perm[k0 + min(er + TPR * u, n1 - 1)];
#pragma unroll
  for (int u = 0; u < PB; ++u) pb[u] = perm[k0 + min(r0 + er + TPR * u, mm - 1)];
#pragma unroll
  for (int u = 0; u < QB; ++u) px[u] = perm[k0 + min(4 * u + g, n1 - 1)];
#pragma unroll
  for (int i = 0; i < NODE_RI; ++i) qr[i] = perm[k0 + min(r0 + ti + 16 * i, mm - 1)];
  double vl[PL], vb[PB], x[QB], acc[NODE_RI][CJ];
  {
    const int cl = k0 + min(ec, n1 - 1), cx = cs + min(c, n2 - 1);
#pragma unroll
    for (int u = 0; u < PL; ++u) vl[u] = a[(long long)pl[u] * lda + cl];
#pragma unroll
    for (int u = 0; u < QB; ++u) x[u] = a[(long long)px[u] * lda + cx];
#pragma unroll
    for (int u = 0; u < PB; ++u) vb[u] = a[(long long)pb[u] * lda + cl];
#pragma unroll
    for (int i = 0; i < NODE_RI; ++i)
#pragma unroll
      for (int j = 0; j < CJ; ++j) acc[i][j] = a[(long long)qr[i] * lda + cs + min(tj + 16 * j, n2 - 1)];
  }
#pragma unroll
  for (int u = 0; u < PL; ++u) {
    const int r = er + TPR * u;
    Ls[r * LD + ec] = (r < n1 && ec < r) ? vl[u] : (r == ec ? 1.0 : 0.0);
  }
#pragma unroll
  for (int u = 0; u < QB; ++u) x[u] = (4 * u + g < n1 && c < n2) ? x[u] : 0.0;
  if (tid < NB) rd[tid] = 1.0;
  __syncthreads();
  quad_lower_solve<LD, QB>(Ls, rd, x, g, opaque_zero());
  __syncthreads();   // every wave is done with L11
  if (c < NB) {
#pragma unroll
    for (int u = 0; u < QB; ++u) Us[(4 * u + g) * LD + c] = x[u];
  }
#pragma unroll
  for (int u = 0; u < PB; ++u) {
    const int r = er + TPR * u;
    Ls[r * LD + ec] = (r0 + r < mm && ec < n1) ? vb[u] : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < n1; ++k) {
    double lv[NODE_RI], uv[CJ];
#pragma unroll
    for (int i = 0; i < NODE_RI; ++i) lv[i] = Ls[(ti + 16 * i) * LD + k];
#pragma unroll
    for (int j = 0; j < CJ; ++j) uv[j] = Us[k * LD + tj + 16 * j];
#pragma unroll
    for (int i = 0; i < NODE_RI; ++i)
#pragma unroll
      for (int j = 0; j < CJ; ++j) acc[i][j] = fma(-lv[i], uv[j], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < NODE_RI; ++i)
#pragma unroll
    for (int j = 0; j < CJ; ++j) {
      const int r = r0 + ti + 16 * i, cc = tj + 16 * j;
      if (r < mm && cc < n2) a[(long long)qr[i] * lda + cs + cc] = acc[i][j];
    }
  // every read of A12 by this workgroup is complete (its values fed the solve)
  if (tid == 0) s_last = atomicAdd(cnt, 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (s_last) {
#pragma unroll
    for (int u = 0; u < PL; ++u) {
      const int r = er + TPR * u;
      if (r < n1 && ec < n2) a[(long long)pl[u] * lda + cs + ec] = Us[r * LD + ec];
    }
    if (tid == 0) atomicExch(cnt, 0);
  }
}

void launch_node(hipStream_t s, double* a, int lda, const int* perm, int k0, int mm, int n1, int n2, int* cnt) {
  const int rows = mm - n1;
  const dim3 g(rows > 0 ? ceil_div(rows, NODE_ROWS) : 1), b(256);
  const int w = max(n1, n2);
  if (w <= 16) hipLaunchKernelGGL(k_lu_node_f64<16>, g, b, 0, s, a, lda, perm, k0, mm, n1, n2, cnt);
  else if (w <= 32) hipLaunchKernelGGL(k_lu_node_f64<32>, g, b, 0, s, a, lda, perm, k0, mm, n1, n2, cnt);
  else if (w <= NODE_MAX) hipLaunchKernelGGL(k_lu_node_f64<64>, g, b, 0, s, a, lda, perm, k0, mm, n1, n2, cnt);
  else throw std::runtime_error("getrf_f64: node wider than the node kernel");
  FROB_LAUNCH_CHECK();
}

// factor columns [k0, k0 + n) over logical rows [k0, m)
// snap (optional): the leaf that ends the recursion, the last to write perm,
// also writes perm[sfrom .. m) to snap[0 ..)
void getrf_rec(hipStream_t s, double* a, int lda, int* perm, int k0, int m, int n, int* info, double* work, int* cnt,
               int* snap = nullptr, int sfrom = 0) {
  const int mm = m - k0;
  const int wmax = leaf_width(mm);
  if (n <= wmax) {
    launch_leaf(s, a, lda, perm, k0, mm, n, 0, info, snap, sfrom);
    return;
  }
  int n1 = (n / 2 + 7) / 8 * 8;
  if (n1 >= n) n1 = n / 2;
  const int n2 = n - n1;
  if (n1 <= wmax && n2 <= wmax && LEAF_SIBLING(ceil_div(mm, LEAF_NT))) {
    // bottom node: one leaf launch factors both halves
    launch_leaf(s, a, lda, perm, k0, mm, n1, n2, info, snap, sfrom);
    return;
  }
  getrf_rec(s, a, lda, perm, k0, m, n1, info, work, cnt);
  if (n1 <= NODE_MAX && n2 <= NODE_MAX) {
    launch_node(s, a, lda, perm, k0, m - k0, n1, n2, cnt);
    getrf_rec(s, a, lda, perm, k0 + n1, m, n2, info, work, cnt, snap, sfrom);
    return;
  }
  // U12 = L11^{-1} A12 (unit lower), rows through perm
  DOp L11{a + k0, lda, perm + k0};
  DOut A12{a + k0 + n1, lda, perm + k0, nullptr};
  trsm_f64(s, false, TRI_LOWER_UNIT, false, n1, n2, L11, A12, work);
  // A22 -= L21 U12
  DOp L21{a + k0, lda, perm + k0 + n1};
  DOp U12{a + k0 + n1, lda, perm + k0};
  DOut A22{a + k0 + n1, lda, perm + k0 + n1, nullptr};
  gemm_f64(s, false, false, m - k0 - n1, n2, n1, -1.0, L21, TRI_NONE, U12, TRI_NONE, 1.0, A22);
  getrf_rec(s, a, lda, perm, k0 + n1, m, n2, info, work, cnt, snap, sfrom);
}

// Panels of la.nb (default LA_NB) columns with a look-ahead of one panel (see internal.hpp),
// grouped into super-panels of LA_SUPER panels.
// Row interchanges only permute `perm` among the trailing positions, so a
// trailing update may run while a later panel pivots, provided it addresses
// its rows through a copy of perm taken when its panel was finished (the set
// of trailing physical rows is the same; their order does not matter to a
// row-wise update); the panel's last leaf writes that copy beside perm.
// Inside a super-panel each panel updates only the super-panel's columns:
//   s0: panel j (with the snapshot) -> event F_j -> [wait R_{j-1}] update of
//       panel j+1's columns (one node launch) -> panel j+1 ...
//   s1: [wait F_j] rank-LA_NB update of the super-panel's columns right of
//       panel j+1 -> event R_j
// Columns right of the super-panel receive its LA_SUPER panels at once, as
// one rank-(LA_SUPER * LA_NB) update (a deeper, more efficient GEMM):
//   s0: [wait G_{s-1}] the next super-panel's columns -> its first panel ...
//   s1: [wait F_j] every column further right -> event G_s
// The next super-panel's columns wait for G_{s-1}, the previous far update
// of those columns.  Snapshots: panel j's (within a super-panel) is rewritten
// at panel j + 2, after s0 has waited for R_j; a super-panel's (written by its
// last panel, read by the far updates) at super-panel s + 2, after s0 has
// waited for G_s.
void getrf_lookahead(hipStream_t s0, int n, int q, double* a, int lda, int* perm, int* info, double* work, int* cnt,
                     const LookAhead& la) {
  const int nt = n + q;   // the q columns right of the matrix take every update and no pivot search
  // panel width: the caller's choice (a multiple of 16 up to LA_NB, the width
  // the scratch below is sized for)
  const int PW = (la.nb >= 16 && la.nb <= LA_NB && la.nb % 16 == 0) ? la.nb : LA_NB;
  const int SW = PW * LA_SUPER;   // super-panel width
  hipStream_t s1 = la.s1;
  double* work0 = work;
  double* work1 = work0 + trsm_work_elems(n / 2 + 8);
  int* snap[2];
  int* snapF[2];
  snap[0] = reinterpret_cast<int*>(work1 + trsm_work_elems(SW));
  snap[1] = snap[0] + n;
  snapF[0] = snap[1] + n;
  snapF[1] = snapF[0] + n;
  auto evF = [&](int j) { return la.ev[j & 3]; };
  auto evR = [&](int j) { return la.ev[4 + (j & 1)]; };
  auto evG = [&](int sp) { return la.ev[6 + (sp & 1)]; };
  // columns c .. c + w - 1 of the trailing matrix, updated with the factored
  // columns k0 .. k0 + nb (rows of the update through trows)
  auto update = [&](hipStream_t st, int k0, int nb, int c, int w, const int* trows, double* wk, bool timed) {
    DOp L11{a + k0, lda, perm + k0};
    DOut A12{a + c, lda, perm + k0, nullptr};
    trsm_f64(st, false, TRI_LOWER_UNIT, false, nb, w, L11, A12, wk);
    const int m = n - (k0 + nb);
    if (m <= 0) return;
    DOp L21{a + k0, lda, trows};
    DOp U12{a + c, lda, perm + k0};
    DOut A22{a + c, lda, trows, nullptr};
    // algorithmic bytes: L21 and U12 read once, A22 read and written
    ProfScope ps(timed ? la.prof : nullptr, PROF_TRAIL_GEMM, 2.0 * m * (double)w * nb, st,
                 8.0 * ((double)m * nb + (double)nb * w + 2.0 * m * w));
    gemm_f64(st, false, false, m, w, nb, -1.0, L21, TRI_NONE, U12, TRI_NONE, 1.0, A22);
  };
  const int np = ceil_div(n, PW);
  int last_r = -1, last_g = -1;
  for (int j = 0; j < np; ++j) {
    const int k0 = j * PW, nb = min(PW, n - k0);
    const int r0 = k0 + nb;
    const int sp = j / LA_SUPER;
    const int K0 = sp * SW;                        // first column of this super-panel
    const int spend = min(n, K0 + SW);             // end of this super-panel's columns
    const bool last_in_sp = r0 >= spend;
    int* sn = last_in_sp ? snapF[sp & 1] : snap[j & 1];
    // the panel's last leaf also writes the snapshot perm[r0 .. n)
    getrf_rec(s0, a, lda, perm, k0, n, nb, info, work0, cnt, r0 < n ? sn : nullptr, r0);
    if (!last_in_sp) {
      FROB_HIP(hipEventRecord(evF(j), s0));
      const int c1 = r0, w1 = min(PW, spend - c1);
      if (j >= 1 && last_r == j - 1) FROB_HIP(hipStreamWaitEvent(s0, evR(j - 1), 0));
      // the next panel's update is a recursion node (solve and update in one launch)
      if (nb <= NODE_MAX && w1 <= NODE_MAX) launch_node(s0, a, lda, perm, k0, n - k0, nb, w1, cnt);
      else update(s0, k0, nb, c1, w1, perm + r0, work0, false);
      const int c2 = c1 + w1, w2 = spend - c2;
      if (w2 > 0) {
        FROB_HIP(hipStreamWaitEvent(s1, evF(j), 0));
        GridCapScope cap(LA_GRID_CAP);   // leave compute units to the panel chain
        update(s1, k0, nb, c2, w2, sn, work1, true);
        FROB_HIP(hipEventRecord(evR(j), s1));
        last_r = j;
      }
      continue;
    }
    // the super-panel is factored: its rank-(r0 - K0) update of the columns
    // right of it (the extra columns included)
    const int KB = r0 - K0;
    if (r0 >= n) {
      // no rows below: the extra columns' rows of this super-panel only (U12)
      if (q > 0) {
        if (last_g >= 0) FROB_HIP(hipStreamWaitEvent(s0, evG(last_g), 0));
        update(s0, K0, KB, n, q, perm + r0, work0, false);
      }
      break;
    }
    FROB_HIP(hipEventRecord(evF(j), s0));
    if (last_g == sp - 1 && sp >= 1) FROB_HIP(hipStreamWaitEvent(s0, evG(sp - 1), 0));
    const int c1 = r0, w1 = min(SW, n - c1);
    if (KB <= NODE_MAX && w1 <= NODE_MAX) launch_node(s0, a, lda, perm, K0, n - K0, KB, w1, cnt);
    else update(s0, K0, KB, c1, w1, sn, work0, false);
    const int c2 = c1 + w1, w2 = nt - c2;
    if (w2 > 0) {
      FROB_HIP(hipStreamWaitEvent(s1, evF(j), 0));
      GridCapScope cap(LA_GRID_CAP);
      update(s1, K0, KB, c2, w2, sn, work1, true);
      FROB_HIP(hipEventRecord(evG(sp), s1));
      last_g = sp;
    }
  }
  if (last_g >= 0) FROB_HIP(hipStreamWaitEvent(s0, evG(last_g), 0));
  if (last_r >= 0) FROB_HIP(hipStreamWaitEvent(s0, evR(last_r), 0));
}

}  // namespace

size_t getrf_work_elems(int n) {
  // node counter, recursion and look-ahead scratch of s0, solve scratch of the
  // second stream, four snapshots of n row indices; or the solve of extra
  // columns without the look-ahead
  return 64 + std::max(trsm_work_elems(n / 2 + 8) + trsm_work_elems(LA_NB * LA_SUPER) + 2 * (size_t)n,
                       trsm_work_elems(n));
}

bool getrf_lookahead_on(int n, const LookAhead* la) { return la && la->s1 && n >= LA_MIN; }

void getrf_f64(hipStream_t s, int n, double* a, int lda, int* perm, int* info, double* work, const LookAhead* la,
               int q) {
  if (n <= 0) return;
  iota_i32(s, n, perm);
  // the node kernels' workgroup counter lives in the first 64 doubles of work
  int* cnt = reinterpret_cast<int*>(work);
  fill_i32(s, 1, 0, cnt);
  if (getrf_lookahead_on(n, la)) {
    getrf_lookahead(s, n, q, a, lda, perm, info, work + 64, cnt, *la);
  } else {
    getrf_rec(s, a, lda, perm, 0, n, n, info, work + 64, cnt);
    if (q > 0)
      trsm_f64(s, false, TRI_LOWER_UNIT, false, n, q, DOp{a, lda, perm}, DOut{a + n, lda, perm, nullptr}, work + 64);
  }
}

}  // namespace frob
