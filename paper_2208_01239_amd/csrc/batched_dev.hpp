// batched_dev.hpp -- the workgroup-level building blocks of the batched
// inversion (one workgroup of BT threads inverts one matrix at a time) and the
// body of the persistent kernel.
//
// The code is written against a handful of primitives that the including file
// supplies before including this header, inside namespace frob::bat:
//   BB_FN                      qualifier of the out-of-line building blocks
//   BB_IN                      qualifier of the small inline helpers
//   int  bb_tid()              thread index within the workgroup
//   void bb_sync()             workgroup barrier (with workgroup memory fence)
//   template <class V> V bb_shfl_xor(V v, int mask)   lane exchange in a wave of 64
//   int  bb_first(int v)       the value held by the wave's first lane
//   d4   bb_mfma(double a, double b, d4 c)   16x16x4 FP64 matrix-core product
//   f4   bb_mfma(float a, float b, f4 c)     16x16x4 FP32 matrix-core product
//   int  bb_atomic_add(int* p, int v)        atomic fetch-and-add
//   BB_GLOBAL                  address-space qualifier of device-memory pointers
//                              (global memory on the GPU: loads and stores of
//                              their own kind, counted apart from LDS accesses)
// and the vector types frob::d4 / frob::f4.  batched.hip maps them to the
// gfx950 intrinsics; the test suite maps them to a cooperative CPU emulation of
// one or more workgroups that checks every barrier is reached by every thread
// in the same order (tests/emu/batched_emu.cpp).
#pragma once

#include <climits>
#include <cmath>

namespace frob {
namespace bat {

constexpr int BT = 256;          // threads per workgroup
constexpr int BNMAX = 512;       // largest order handled in-workgroup
constexpr int PNB = 16;          // largest LU panel width
constexpr int PP = PNB + 1;      // LDS pitch of panel rows (odd in 8-byte words: rows fall on different banks)
// The panel buffer holds an LU panel (BNMAX x PP), a triangular or Cholesky
// diagonal block, the staged interchange gather (2 PNB x BT), or the GEMM's two
// operand stages of the widest tile (16 x (20 + 260) each); 70 KiB in FP64,
// so that two workgroups fit a compute unit's 160 KiB of LDS.
constexpr int PANEL_ELEMS = 8960;
static_assert(PANEL_ELEMS >= BNMAX * PP && PANEL_ELEMS >= 2 * PNB * BT, "panel buffer too small");
constexpr int XNB = 16;          // diagonal blocks solved by register substitution (triangular solves, Cholesky)
constexpr int GK = 16;           // GEMM k-step
// Element-wise passes keep SU loads per thread in flight before their stores:
// the matrices are reached through generic pointers, so the compiler cannot
// move a load above an earlier store, and a pass of dependent load-store
// pairs would wait one memory latency per element.
constexpr int SU = 8;

BB_IN int imin(int a, int b) { return a < b ? a : b; }
BB_IN int imax(int a, int b) { return a > b ? a : b; }

// Output layout of the 16x16x4 products: lane l holds column l % 16 of four
// rows.  Input layout: lane l supplies A(l % 16, l / 16) and B(l / 16, l % 16).
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef d4 acc;
  BB_IN static acc op(double a, double b, acc c) { return bb_mfma(a, b, c); }
  BB_IN static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef f4 acc;
  BB_IN static acc op(float a, float b, acc c) { return bb_mfma(a, b, c); }
  BB_IN static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <typename T>
struct Smem {
  T panel[PANEL_ELEMS];      // LU panel / Cholesky diagonal block / triangular diagonal block;
                             // the GEMM's double-buffered operand tiles when none of those is live
  T slot_v[2][BT / 64];       // LU panel: each wave's pivot candidate by column parity: |value|,
  int slot_p[2][BT / 64];     //   position,
  int slot_q[2][BT / 64];     //   and row in the panel buffer
  int bcast[4];
  int perm[BNMAX];           // LU: original row now at each row position
  int rowpos[BNMAX];         // LU panel: final position of each panel row
  int tl_dst[2 * PNB];       // LU panel: rows changed by the panel's interchanges,
  int tl_src[2 * PNB];       //   and the rows their new content comes from
  int tl_n;
};

// Scalar arguments of the out-of-line building blocks arrive in vector
// registers; re-reading them through the first lane makes every loop bound and
// branch condition derived from them uniform to the compiler (they are uniform
// in value), so barrier-containing regions are never entered with a partial or
// empty exec mask.
BB_IN int uni(int v) { return bb_first(v); }
BB_IN bool uni(bool v) { return bb_first((int)v) != 0; }

// ---------------------------------------------------------------- GEMM
// C (M x N) = alpha op(A) op(B) + beta C; op(A) is M x K (A stored K x M if ta).
// Output tiles of TM x TN = (WM * BA * 16) x (WN * BB * 16): 4 waves in a
// WM x WN grid, each owning BA x BB blocks of 16 x 16 (16x16x4 matrix-core
// products).  Operand tiles are staged k-major in LDS, double-buffered in the
// panel buffer (the callers hold nothing live there during a product): the
// next k-step's global loads are in flight during the current products and
// one barrier separates the k-steps.  Edges: loads at clamped in-range
// addresses, values outside the matrix zeroed when staged.
template <typename T, int WM, int WN, int BA, int BB>
BB_FN void wg_gemm_tiles(Smem<T>& sm, int M, int N, int K, T alpha, BB_GLOBAL const T* A, int lda, bool ta,
                         BB_GLOBAL const T* B, int ldb, bool tb, T beta, BB_GLOBAL T* C, int ldc, bool lower) {
  typedef typename Mfma<T>::acc acc_t;
  constexpr int TM = WM * BA * 16, TN = WN * BB * 16;
  constexpr int PA = TM + 4, PB = TN + 4;          // LDS pitches of the k-major tiles
  constexpr int BUF = GK * (PA + PB);              // one stage: A tile then B tile
  static_assert(2 * BUF <= PANEL_ELEMS, "GEMM stages exceed the panel buffer");
  constexpr int EA = (TM * GK + BT - 1) / BT, EB = (TN * GK + BT - 1) / BT;
  const int tid = bb_tid(), lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / WN) * (BA * 16), wn = (wave % WN) * (BB * 16);
  const int tilesN = (N + TN - 1) / TN;
  const int tiles = ((M + TM - 1) / TM) * tilesN;
  const int nk = (K + GK - 1) / GK;
  T* lds = sm.panel;
  for (int t = 0; t < tiles; ++t) {
    const int tm = (t / tilesN) * TM, tn = (t % tilesN) * TN;
    if (lower && tn > tm + TM - 1) continue;   // entirely above the diagonal (uniform)
    acc_t acc[BA][BB];
#pragma unroll
    for (int a = 0; a < BA; ++a)
#pragma unroll
      for (int b = 0; b < BB; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
    T ra[EA], rb[EB];
    auto load = [&](int k0) {
#pragma unroll
      for (int u = 0; u < EA; ++u) {
        const int e = imin(tid + BT * u, TM * GK - 1);
        int i, k;
        if (!ta) { i = e / GK; k = e % GK; } else { k = e / TM; i = e % TM; }
        const int gi = imin(tm + i, M - 1), gk = imin(k0 + k, K - 1);
        ra[u] = ta ? A[(long long)gk * lda + gi] : A[(long long)gi * lda + gk];
      }
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        const int e = imin(tid + BT * u, TN * GK - 1);
        int k, j;
        if (!tb) { k = e / TN; j = e % TN; } else { j = e / GK; k = e % GK; }
        const int gk = imin(k0 + k, K - 1), gj = imin(tn + j, N - 1);
        rb[u] = tb ? B[(long long)gj * ldb + gk] : B[(long long)gk * ldb + gj];
      }
    };
    auto store = [&](int k0, T* st) {
#pragma unroll
      for (int u = 0; u < EA; ++u) {
        const int e = tid + BT * u;
        if (e < TM * GK) {
          int i, k;
          if (!ta) { i = e / GK; k = e % GK; } else { k = e / TM; i = e % TM; }
          st[k * PA + i] = (tm + i < M && k0 + k < K) ? ra[u] : T(0);
        }
      }
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        const int e = tid + BT * u;
        if (e < TN * GK) {
          int k, j;
          if (!tb) { k = e / TN; j = e % TN; } else { j = e / GK; k = e % GK; }
          st[GK * PA + k * PB + j] = (tn + j < N && k0 + k < K) ? rb[u] : T(0);
        }
      }
    };
    if (nk > 0) {
      load(0);
      store(0, lds);
    }
    bb_sync();
    for (int it = 0; it < nk; ++it) {
      if (it + 1 < nk) load((it + 1) * GK);
      const T* sa = lds + (it & 1) * BUF;
      const T* sb = sa + GK * PA;
#pragma unroll
      for (int kk = 0; kk < GK; kk += 4) {
        T fa[BA], fb[BB];
#pragma unroll
        for (int a = 0; a < BA; ++a) fa[a] = sa[(kk + (lane >> 4)) * PA + wm + 16 * a + (lane & 15)];
#pragma unroll
        for (int b = 0; b < BB; ++b) fb[b] = sb[(kk + (lane >> 4)) * PB + wn + 16 * b + (lane & 15)];
#pragma unroll
        for (int a = 0; a < BA; ++a)
#pragma unroll
          for (int b = 0; b < BB; ++b) acc[a][b] = Mfma<T>::op(fa[a], fb[b], acc[a][b]);
      }
      if (it + 1 < nk) store((it + 1) * GK, lds + ((it + 1) & 1) * BUF);
      bb_sync();
    }
    // epilogue, one block row at a time: its reads of C are all issued
    // before its writes.  Interior tiles take branch-free code: a store under
    // a per-lane condition sits in a block of its own, and the compiler then
    // waits for every earlier memory operation before it.
    if (tm + TM <= M && tn + TN <= N) {   // uniform
#pragma unroll
      for (int a = 0; a < BA; ++a) {
        T cv[4][BB];
        if (beta != T(0)) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int b = 0; b < BB; ++b)
              cv[v][b] = C[(long long)(tm + wm + 16 * a + Mfma<T>::row(lane, v)) * ldc + tn + wn + 16 * b + (lane & 15)];
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int b = 0; b < BB; ++b) cv[v][b] = T(0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int b = 0; b < BB; ++b)
            C[(long long)(tm + wm + 16 * a + Mfma<T>::row(lane, v)) * ldc + tn + wn + 16 * b + (lane & 15)] =
                alpha * acc[a][b][v] + beta * cv[v][b];
      }
      continue;
    }
#pragma unroll
    for (int a = 0; a < BA; ++a) {
      T cv[4][BB];
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int b = 0; b < BB; ++b) {
          const int i = imin(tm + wm + 16 * a + Mfma<T>::row(lane, v), M - 1);
          const int j = imin(tn + wn + 16 * b + (lane & 15), N - 1);
          cv[v][b] = beta != T(0) ? C[(long long)i * ldc + j] : T(0);
        }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = tm + wm + 16 * a + Mfma<T>::row(lane, v);
#pragma unroll
        for (int b = 0; b < BB; ++b) {
          const int j = tn + wn + 16 * b + (lane & 15);
          if (i < M && j < N) C[(long long)i * ldc + j] = alpha * acc[a][b][v] + beta * cv[v][b];
        }
      }
    }
  }
  bb_sync();
}

// The tile shape follows the product's shape: large tiles for full products
// (128 x 128 in FP32, 128 x 64 in FP64), wide ones for the short updates of
// the triangular solves, tall ones for the narrow column updates of the
// factorizations.
// lower: only tiles that meet the lower triangle (diagonal included) are
// formed; entries above the diagonal in those tiles are written too.
template <typename T>
BB_FN void wg_gemm(Smem<T>& sm, int M, int N, int K, T alpha, const T* A, int lda, bool ta, const T* B, int ldb,
                   bool tb, T beta, T* C, int ldc, bool lower = false) {
  M = uni(M); N = uni(N); K = uni(K); lda = uni(lda); ldb = uni(ldb); ldc = uni(ldc); ta = uni(ta); tb = uni(tb);
  lower = uni(lower);
  // device-memory pointers for the tiles: their loads and stores are then
  // global accesses, counted apart from the LDS accesses of the k-loop, so
  // the next k-step's loads stay in flight while its fragments are read
  BB_GLOBAL const T* gA = (BB_GLOBAL const T*)A;
  BB_GLOBAL const T* gB = (BB_GLOBAL const T*)B;
  BB_GLOBAL T* gC = (BB_GLOBAL T*)C;
  if (M <= 0 || N <= 0) {
    bb_sync();
    return;
  }
  if (M <= 16 && N > 64)
    wg_gemm_tiles<T, 1, 4, 1, 4>(sm, M, N, K, alpha, gA, lda, ta, gB, ldb, tb, beta, gC, ldc, lower);      // 16 x 256
  else if (M <= 32 && N > 64)
    wg_gemm_tiles<T, 2, 2, 1, 4>(sm, M, N, K, alpha, gA, lda, ta, gB, ldb, tb, beta, gC, ldc, lower);      // 32 x 128
  else if (N <= 16 && M > 64)
    wg_gemm_tiles<T, 4, 1, 4, 1>(sm, M, N, K, alpha, gA, lda, ta, gB, ldb, tb, beta, gC, ldc, lower);      // 256 x 16
  else if (N <= 32 && M > 64)
    wg_gemm_tiles<T, 2, 2, 4, 1>(sm, M, N, K, alpha, gA, lda, ta, gB, ldb, tb, beta, gC, ldc, lower);      // 128 x 32
  else if (M > 64 && N > 64 && sizeof(T) == 8)
    // FP64: 128 x 64; the 128 x 128 tile's accumulators and prefetch registers
    // exceed the register share of two waves per SIMD and spill in the k-loop
    wg_gemm_tiles<T, 2, 2, 4, 2>(sm, M, N, K, alpha, gA, lda, ta, gB, ldb, tb, beta, gC, ldc, lower);
  else if (M > 64 && N > 64)
    wg_gemm_tiles<T, 2, 2, 4, 4>(sm, M, N, K, alpha, gA, lda, ta, gB, ldb, tb, beta, gC, ldc, lower);      // 128 x 128
  else
    wg_gemm_tiles<T, 2, 2, 2, 2>(sm, M, N, K, alpha, gA, lda, ta, gB, ldb, tb, beta, gC, ldc, lower);      // 64 x 64
}

// ------------------------------------------------------- triangular solves
// op(T) X = B in place (B is n x nrhs), op(T) triangular:
//   mode 0: T lower, op(T) = T   (forward substitution; unit diagonal if `unit`)
//   mode 1: T lower, op(T) = T^T (backward)
//   mode 2: T upper, op(T) = T   (backward)
// idrhs (mode 0 only): B holds the identity on entry, so the solution T^{-1}
// is lower triangular and only the columns left of each block are touched.
// Leaves of nb <= 16 rows are solved by register substitution (one thread per
// right-hand side); the updates follow the order of the recursive algorithm
// (solve the first half, update the second half with a product of depth
// n / 2, solve the second half), flattened: when a leaf completes a group of
// g = lowbit(leaves done) leaves, the next g leaves' rows are updated by the
// group's solution, a product of depth g * nb.  Every row of B is thus
// rewritten about log2(n / nb) times instead of n / nb times, and the deep
// products near the root do most of the work.
template <typename T>
BB_FN void wg_trsm(Smem<T>& sm, int mode, int n, int nrhs, const T* L, int ldl, bool unit, T* B, int ldb, int nb,
                   bool idrhs = false) {
  mode = uni(mode); n = uni(n); nrhs = uni(nrhs); ldl = uni(ldl); ldb = uni(ldb); unit = uni(unit);
  idrhs = uni(idrhs) && mode == 0;
  const int tid = bb_tid();
  nb = imax(imin(uni(nb), XNB), 1);
  const int nblk = (n + nb - 1) / nb;
  const bool fwd = mode == 0;
  for (int t = 0; t < nblk; ++t) {
    const int blk = fwd ? t : nblk - 1 - t;
    const int k0 = blk * nb, kb = imin(nb, n - k0);
    // diagonal block of op(T) into LDS: D(i, k) = op(T)(k0 + i, k0 + k)
    T* D = sm.panel;
    for (int e = tid; e < kb * kb; e += BT) {
      const int i = e / kb, k = e % kb;
      const int r = mode == 1 ? k : i, c = mode == 1 ? i : k;   // stored coordinates within the block
      const bool in = mode == 2 ? c >= r : c <= r;
      D[i * PP + k] = in ? L[(long long)(k0 + r) * ldl + k0 + c] : T(0);
    }
    // A leaf that completes a group of one (t even) also applies its update
    // to the next leaf's rows, a product of depth kb, in registers: each
    // thread subtracts E x from the next rows of its columns, with
    // E(i, k) = op(T)(e0 + i, k0 + k) staged after the diagonal block.
    const bool g1 = (t & 1) == 0;
    const int e0 = fwd ? k0 + kb : imax(0, k0 - nb);
    const int ne = !g1 ? 0 : fwd ? imin(nb, n - e0) : k0 - e0;
    T* E = sm.panel + XNB * PP;
    for (int e = tid; e < ne * kb; e += BT) {
      const int i = e / kb, k = e % kb;
      E[i * PP + k] = mode == 1 ? L[(long long)(k0 + k) * ldl + e0 + i] : L[(long long)(e0 + i) * ldl + k0 + k];
    }
    bb_sync();
    // B = I (idrhs): the solution is lower triangular, so rows k0 .. k0 + kb
    // have nonzeros only in the columns left of k0 + kb
    const int jend = idrhs ? imin(nrhs, k0 + kb) : nrhs;
    for (int j = tid; j < jend; j += BT) {
      T x[XNB];
#pragma unroll
      for (int i = 0; i < XNB; ++i) x[i] = B[(long long)(k0 + imin(i, kb - 1)) * ldb + j];
      if (fwd) {
#pragma unroll
        for (int i = 0; i < XNB; ++i)
          if (i < kb) {
            T v = x[i];
#pragma unroll
            for (int k = 0; k < i; ++k) v -= D[i * PP + k] * x[k];
            x[i] = unit ? v : v / D[i * PP + i];
          }
      } else {
#pragma unroll
        for (int i = XNB - 1; i >= 0; --i)
          if (i < kb) {
            T v = x[i];
#pragma unroll
            for (int k = i + 1; k < XNB; ++k)
              if (k < kb) v -= D[i * PP + k] * x[k];
            x[i] = unit ? v : v / D[i * PP + i];
          }
      }
#pragma unroll
      for (int i = 0; i < XNB; ++i)
        if (i < kb) B[(long long)(k0 + i) * ldb + j] = x[i];
      for (int i0 = 0; i0 < ne; i0 += 4) {   // four rows at a time (registers)
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = B[(long long)(e0 + imin(i0 + u, ne - 1)) * ldb + j];
#pragma unroll
        for (int k = 0; k < XNB; ++k)
          if (k < kb) {
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] -= E[imin(i0 + u, ne - 1) * PP + k] * x[k];
          }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 + u < ne) B[(long long)(e0 + i0 + u) * ldb + j] = v[u];
      }
    }
    bb_sync();
    const int g = (t + 1) & -(t + 1);   // leaves in the group this leaf completes
    if (g == 1) continue;               // applied above
    if (fwd) {
      // done: rows [c0, c1); next: rows [c1, r1) -= op(T)[c1:r1, c0:c1] X[c0:c1]
      const int c1 = k0 + kb, c0 = c1 - imin(g * nb, c1), r1 = imin(c1 + g * nb, n);
      if (c1 < n)
        wg_gemm<T>(sm, r1 - c1, idrhs ? imin(nrhs, c1) : nrhs, c1 - c0, T(-1), L + (long long)c1 * ldl + c0, ldl, false,
                   B + (long long)c0 * ldb, ldb, false, T(1), B + (long long)c1 * ldb, ldb);
    } else {
      // done: rows [k0, c1); next: rows [r0, k0) -= op(T)[r0:k0, k0:c1] X[k0:c1]
      const int c1 = imin(k0 + g * nb, n), r0 = imax(0, k0 - g * nb);
      if (k0 > 0) {
        if (mode == 1)
          wg_gemm<T>(sm, k0 - r0, nrhs, c1 - k0, T(-1), L + (long long)k0 * ldl + r0, ldl, true,
                     B + (long long)k0 * ldb, ldb, false, T(1), B + (long long)r0 * ldb, ldb);
        else
          wg_gemm<T>(sm, k0 - r0, nrhs, c1 - k0, T(-1), L + (long long)r0 * ldl + k0, ldl, false,
                     B + (long long)k0 * ldb, ldb, false, T(1), B + (long long)r0 * ldb, ldb);
      }
    }
  }
}

// The update of the next nb <= PNB columns [c1, c1 + n2) by a finished LU
// panel [k0, k0 + kb) (a group of one in the recursive order), on the vector
// units: U12 = L11^{-1} A12 (L11 unit lower) on the panel's rows, then
// A22 -= L21 U12 below them.  Inline: an out-of-line product call would save
// and restore the callee-saved registers for a depth-kb update.
template <typename T>
BB_IN void wg_lu_update1(Smem<T>& sm, int n, T* A, int lda, int k0, int kb, int c1, int n2) {
  const int tid = bb_tid();
  T* Ls = sm.panel;               // L11, pitch PP
  T* Us = sm.panel + PNB * PP;    // A12, then U12
  {
    const int i = tid / PNB, c = tid % PNB;   // kb x PNB <= BT entries: one per thread
    if (i < kb) {
      if (c < kb) Ls[i * PP + c] = A[(long long)(k0 + i) * lda + k0 + c];
      if (c < n2) Us[i * PP + c] = A[(long long)(k0 + i) * lda + c1 + c];
    }
  }
  bb_sync();
  if (tid < n2) {
    T x[PNB];
#pragma unroll
    for (int i = 0; i < PNB; ++i) x[i] = Us[imin(i, kb - 1) * PP + tid];
#pragma unroll
    for (int i = 0; i < PNB; ++i)
      if (i < kb) {
        T v = x[i];
#pragma unroll
        for (int k = 0; k < i; ++k) v -= Ls[i * PP + k] * x[k];
        x[i] = v;
      }
#pragma unroll
    for (int i = 0; i < PNB; ++i)
      if (i < kb) {
        Us[i * PP + tid] = x[i];
        A[(long long)(k0 + i) * lda + c1 + tid] = x[i];
      }
  }
  bb_sync();
  for (int r = c1 + tid; r < n; r += BT) {
    T l[PNB];
    const T* lrow = A + (long long)r * lda + k0;
#pragma unroll
    for (int k = 0; k < PNB; ++k) l[k] = lrow[imin(k, kb - 1)];
    T* arow = A + (long long)r * lda + c1;
    for (int cb = 0; cb < n2; cb += 8) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = arow[imin(cb + u, n2 - 1)];
#pragma unroll
      for (int k = 0; k < PNB; ++k)
        if (k < kb) {
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] -= l[k] * Us[k * PP + imin(cb + u, n2 - 1)];
        }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (cb + u < n2) arow[cb + u] = v[u];
    }
  }
  bb_sync();
}

// ------------------------------------------------------------- LU (GEPP)
// P A = L U in place; perm_out[r] = the row of A that row r of P A is.
// Panels of nb <= PNB columns are factored in LDS.  Thread t owns the panel
// rows q = t + s BT (s < PR): only it writes them, and each row keeps its
// place in LDS while its logical position pos within the panel lives in the
// owner's registers (GEPP's interchanges act on these integers only).  Per
// column j, one barrier:
//   - every thread takes its best candidate (largest |a_qj| among its rows
//     with pos >= j, lowest pos on ties, NaN below every number), the wave
//     reduces (value, pos) by lane exchanges, and the lane holding the winner
//     publishes (value, pos, row) in the wave's slot (double-buffered by
//     column parity);
//   - after the barrier every thread reduces the slots the same way,
//     exchanges positions j and p, and updates its rows with pos > j from the
//     pivot row, read in place (its owner never writes it again).
// The panel is then written to its rows' final positions; the rows the
// panel's interchanges change in the columns outside it are rewritten by one
// gather per column, loads in flight before the stores.  Trailing updates in
// recursive order (below).  Returns the first zero pivot column + 1, or 0.
// nb >= 1 (the caller clamps).
constexpr int PR = BNMAX / BT;   // panel rows per thread
constexpr int RG = BT / PNB;     // rows moved together by the panel load and store
template <typename T>
BB_FN int wg_getrf(Smem<T>& sm, int n, T* A, int lda, int* perm_out, int nb) {
  n = uni(n); lda = uni(lda); nb = imin(uni(nb), PNB);
  const int tid = bb_tid(), lane = tid & 63, wave = tid >> 6;
  int info = 0;
  for (int r = tid; r < n; r += BT) sm.perm[r] = r;
  for (int k0 = 0, t = 0; k0 < n; k0 += nb, ++t) {
    const int kb = imin(nb, n - k0), m = n - k0;
    // panel (rows k0.., columns k0..k0+kb) into LDS: P[r][c]; thread t
    // moves column t % PNB of rows t / PNB + i RG
    T* P = sm.panel;
    const int pc = tid % PNB, pr0 = tid / PNB;
    const bool pcol = pc < kb;
    for (int rb = pr0; rb < m; rb += SU * RG) {
      T v[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) v[u] = A[(long long)(k0 + imin(rb + u * RG, m - 1)) * lda + k0 + imin(pc, kb - 1)];
#pragma unroll
      for (int u = 0; u < SU; ++u)
        if (pcol && rb + u * RG < m) P[(rb + u * RG) * PP + pc] = v[u];
    }
    int pos[PR];
#pragma unroll
    for (int s = 0; s < PR; ++s) pos[s] = tid + s * BT < m ? tid + s * BT : -1;
    if (tid == 0) sm.tl_n = 0;
    bb_sync();
    for (int j = 0; j < kb; ++j) {
      const int par = j & 1;
      // candidate among this thread's rows
      T bv = T(-2);
      int bp = INT_MAX, bq = 0;
#pragma unroll
      for (int s = 0; s < PR; ++s)
        if (pos[s] >= j) {
          const int q = tid + s * BT;
          const T a0 = std::fabs(P[q * PP + j]);
          const T a = a0 == a0 ? a0 : T(-1);
          const bool take = (a > bv) | ((a == bv) & (pos[s] < bp));
          bv = take ? a : bv;
          bp = take ? pos[s] : bp;
          bq = take ? q : bq;
        }
      // wave reduction; the lane holding the winner publishes it
      T wv = bv;
      int wp = bp;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const T ov = bb_shfl_xor(wv, off);
        const int op = bb_shfl_xor(wp, off);
        const bool take = (ov > wv) | ((ov == wv) & (op < wp));
        wv = take ? ov : wv;
        wp = take ? op : wp;
      }
      if (wp == INT_MAX) {
        if (lane == 0) {
          sm.slot_v[par][wave] = T(-2);
          sm.slot_p[par][wave] = INT_MAX;
        }
      } else if (bp == wp) {   // positions are distinct: exactly one lane
        sm.slot_v[par][wave] = wv;
        sm.slot_p[par][wave] = wp;
        sm.slot_q[par][wave] = bq;
      }
      bb_sync();
      T gv = sm.slot_v[par][0];
      int gp = sm.slot_p[par][0], gq = sm.slot_q[par][0];
#pragma unroll
      for (int w = 1; w < BT / 64; ++w) {
        const T ov = sm.slot_v[par][w];
        const int op = sm.slot_p[par][w], oq = sm.slot_q[par][w];
        const bool take = (ov > gv) | ((ov == gv) & (op < gp));
        gv = take ? ov : gv;
        gp = take ? op : gp;
        gq = take ? oq : gq;
      }
      // the row at position j is always a candidate, so gp < INT_MAX
      const int p = gp;
#pragma unroll
      for (int s = 0; s < PR; ++s) pos[s] = pos[s] == p ? j : (pos[s] == j ? p : pos[s]);
      const T* prow = P + gq * PP;
      const T d = prow[j];
      if (d == T(0)) {
        if (!info) info = k0 + j + 1;
      } else {
        // row segments pass through registers eight columns at a time, so
        // the LDS reads of a chunk are in flight together before its writes
        const T rd = T(1) / d;
#pragma unroll
        for (int s = 0; s < PR; ++s)
          if (pos[s] > j) {
            T* row = P + (tid + s * BT) * PP;
            const T l = row[j] * rd;
            row[j] = l;
            for (int c0 = j + 1; c0 < kb; c0 += 8) {
              T rv[8], pv[8];
#pragma unroll
              for (int u = 0; u < 8; ++u) {
                const int c = imin(c0 + u, kb - 1);
                rv[u] = row[c];
                pv[u] = prow[c];
              }
#pragma unroll
              for (int u = 0; u < 8; ++u)
                if (c0 + u < kb) row[c0 + u] = rv[u] - l * pv[u];
            }
          }
      }
    }
    // final positions: the store below reads them; the permutation and the
    // list of moved rows (at most 2 kb) follow from them
    int op[PR];
#pragma unroll
    for (int s = 0; s < PR; ++s) op[s] = pos[s] >= 0 ? sm.perm[k0 + tid + s * BT] : 0;
#pragma unroll
    for (int s = 0; s < PR; ++s)
      if (pos[s] >= 0) sm.rowpos[tid + s * BT] = pos[s];
    bb_sync();
#pragma unroll
    for (int s = 0; s < PR; ++s) {
      const int q = tid + s * BT;
      if (pos[s] >= 0 && pos[s] != q) {
        sm.perm[k0 + pos[s]] = op[s];
        const int e = bb_atomic_add(&sm.tl_n, 1);
        if (e < 2 * PNB) {
          sm.tl_dst[e] = k0 + pos[s];
          sm.tl_src[e] = k0 + q;
        }
      }
    }
    for (int rb = pr0; rb < m; rb += SU * RG) {
      T v[SU];
      int dr[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int r = imin(rb + u * RG, m - 1);
        v[u] = P[r * PP + pc];
        dr[u] = sm.rowpos[r];
      }
#pragma unroll
      for (int u = 0; u < SU; ++u)
        if (pcol && rb + u * RG < m) A[(long long)(k0 + dr[u]) * lda + k0 + pc] = v[u];
    }
    bb_sync();
    // each thread moves its own columns, staged in the (now free) panel
    // buffer: all loads of a column are issued, SU at a time, before any of
    // its stores
    const int cnt = imin(uni(sm.tl_n), 2 * PNB);
    for (int c = tid; c < n; c += BT) {
      if (c >= k0 && c < k0 + kb) continue;
      T* S = P;   // 2 PNB rows x BT columns fit the buffer; a thread's second column reuses its slots
      for (int e0 = 0; e0 < cnt; e0 += SU) {
        T v[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) v[u] = A[(long long)sm.tl_src[imin(e0 + u, cnt - 1)] * lda + c];
#pragma unroll
        for (int u = 0; u < SU; ++u)
          if (e0 + u < cnt) S[(e0 + u) * BT + tid] = v[u];
      }
      for (int e0 = 0; e0 < cnt; e0 += SU) {
        T v[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) v[u] = S[imin(e0 + u, cnt - 1) * BT + tid];
#pragma unroll
        for (int u = 0; u < SU; ++u)
          if (e0 + u < cnt) A[(long long)sm.tl_dst[e0 + u] * lda + c] = v[u];
      }
    }
    bb_sync();
    // Updates in the order of the recursive algorithm (factor the left half,
    // update the right half, factor the right half), flattened: panel t
    // completes a group of g = lowbit(t + 1) panels, columns [c0, c1), whose
    // interchanges every column has already received; the next g panels'
    // columns [c1, r1) take U12 = L11^{-1} A12 on the group's rows and
    // A22 -= L21 U12 below them, a product of depth c1 - c0.  Columns further
    // right wait for a larger group, so the trailing matrix is rewritten about
    // log2(n / nb) times instead of n / nb times.
    const int g = (t + 1) & -(t + 1);
    const int c1 = k0 + kb, c0 = c1 - imin(g * nb, c1), r1 = imin(c1 + g * nb, n);
    if (c1 < n && g == 1) {
      wg_lu_update1<T>(sm, n, A, lda, k0, kb, c1, r1 - c1);
    } else if (c1 < n) {
      wg_trsm<T>(sm, 0, c1 - c0, r1 - c1, A + (long long)c0 * lda + c0, lda, true, A + (long long)c0 * lda + c1, lda,
                 nb);
      wg_gemm<T>(sm, n - c1, r1 - c1, c1 - c0, T(-1), A + (long long)c1 * lda + c0, lda, false,
                 A + (long long)c0 * lda + c1, lda, false, T(1), A + (long long)c1 * lda + c1, lda);
    }
  }
  for (int r = tid; r < n; r += BT) perm_out[r] = sm.perm[r];
  bb_sync();
  return info;
}

// dst = P src: row r of dst is row perm[r] of src (n x ncols)
template <typename T>
BB_IN void wg_gather_rows(int n, int ncols, const T* src, int lds, const int* perm, T* dst, int ldd) {
  n = uni(n); ncols = uni(ncols); lds = uni(lds); ldd = uni(ldd);
  const int total = n * ncols;
  for (int base = bb_tid(); base < total; base += SU * BT) {
    T v[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = imin(base + u * BT, total - 1), r = e / ncols;
      v[u] = src[(long long)perm[r] * lds + (e - r * ncols)];
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = base + u * BT, r = e / ncols;
      if (e < total) dst[(long long)r * ldd + (e - r * ncols)] = v[u];
    }
  }
  bb_sync();
}

// dst = src P (n x n): column perm[r] of dst is column r of src
template <typename T>
BB_IN void wg_scatter_cols(int n, const T* src, const int* perm, T* dst) {
  n = uni(n);
  const int total = n * n;
  for (int base = bb_tid(); base < total; base += SU * BT) {
    T v[SU];
    int pc[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = imin(base + u * BT, total - 1);
      v[u] = src[e];
      pc[u] = perm[e % n];
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = base + u * BT;
      if (e < total) dst[(long long)(e / n) * n + pc[u]] = v[u];
    }
  }
  bb_sync();
}

// a[j][i] = sign a[i][j] above the diagonal (i > j), from the lower triangle
// (the entries read and the entries written are disjoint)
template <typename T>
BB_IN void wg_mirror(int n, T* a, T sign) {
  n = uni(n);
  const int total = n * n;
  for (int base = bb_tid(); base < total; base += SU * BT) {
    T v[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = imin(base + u * BT, total - 1), i = e / n;
      v[u] = e - i * n < i ? a[e] : T(0);
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int e = base + u * BT, i = e / n, j = e - i * n;
      if (e < total && j < i) a[(long long)j * n + i] = sign * v[u];
    }
  }
  bb_sync();
}

// The update of the next nb <= XNB block column [c1, c1 + n2) by a finished
// Cholesky block column [k0, k0 + kb) (a group of one in the recursive order),
// on the vector units: A[c1:, c1:c1+n2] -= L[c1:, k0:c1] L[c1:c1+n2, k0:c1]^T
// (entries above the diagonal included, never read).
template <typename T>
BB_IN void wg_chol_update1(Smem<T>& sm, int n, T* A, int lda, int k0, int kb, int c1, int n2) {
  const int tid = bb_tid();
  T* Lb = sm.panel;   // L[c1 + c][k0 + k] at Lb[c * PP + k]
  {
    const int c = tid / XNB, k = tid % XNB;   // n2 x XNB <= BT entries: one per thread
    if (c < n2 && k < kb) Lb[c * PP + k] = A[(long long)(c1 + c) * lda + k0 + k];
  }
  bb_sync();
  for (int r = c1 + tid; r < n; r += BT) {
    T l[XNB];
    const T* lrow = A + (long long)r * lda + k0;
#pragma unroll
    for (int k = 0; k < XNB; ++k) l[k] = lrow[imin(k, kb - 1)];
    T* arow = A + (long long)r * lda + c1;
    for (int cb = 0; cb < n2; cb += 8) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = arow[imin(cb + u, n2 - 1)];
#pragma unroll
      for (int k = 0; k < XNB; ++k)
        if (k < kb) {
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] -= l[k] * Lb[imin(cb + u, n2 - 1) * PP + k];
        }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (cb + u < n2) arow[cb + u] = v[u];
    }
  }
  bb_sync();
}

// ------------------------------------------------------------ Cholesky
// A = L L^T in place (lower triangle).  Returns the first non-positive pivot's
// column (1-based), or 0.  nb >= 1 (the caller clamps).
template <typename T>
BB_FN int wg_potrf(Smem<T>& sm, int n, T* A, int lda, int nb) {
  n = uni(n); lda = uni(lda);
  const int tid = bb_tid();
  nb = imin(uni(nb), XNB);
  int bad = 0;
  for (int k0 = 0, t = 0; k0 < n; k0 += nb, ++t) {
    const int kb = imin(nb, n - k0);
    T* D = sm.panel;
    for (int e = tid; e < kb * kb; e += BT) {
      const int i = e / kb, k = e % kb;
      D[i * PP + k] = (k <= i) ? A[(long long)(k0 + i) * lda + k0 + k] : T(0);
    }
    bb_sync();
    for (int j = 0; j < kb; ++j) {
      const T d = D[j * PP + j];
      // a non-positive pivot is recorded and the factorization runs on (its
      // square root is NaN): the control flow never depends on the data
      if (!bad && !(d > T(0))) bad = k0 + j + 1;
      const T ljj = std::sqrt(d);
      bb_sync();
      if (tid == 0) D[j * PP + j] = ljj;
      for (int i = j + 1 + tid; i < kb; i += BT) D[i * PP + j] /= ljj;
      bb_sync();
      for (int e = tid; e < kb * kb; e += BT) {
        const int i = e / kb, c = e % kb;
        if (i > j && c > j && c <= i) D[i * PP + c] -= D[i * PP + j] * D[c * PP + j];
      }
      bb_sync();
    }
    for (int e = tid; e < kb * kb; e += BT) {
      const int i = e / kb, k = e % kb;
      if (k <= i) A[(long long)(k0 + i) * lda + k0 + k] = D[i * PP + k];
    }
    bb_sync();
    const int rest = n - k0 - kb;
    if (rest > 0) {
      // L21 = A21 L11^{-T}: row r solves L11 x = a_r
      for (int r = tid; r < rest; r += BT) {
        T* row = A + (long long)(k0 + kb + r) * lda + k0;
        T x[XNB];
#pragma unroll
        for (int i = 0; i < XNB; ++i) x[i] = row[imin(i, kb - 1)];
#pragma unroll
        for (int i = 0; i < XNB; ++i)
          if (i < kb) {
            T v = x[i];
#pragma unroll
            for (int k = 0; k < i; ++k) v -= D[i * PP + k] * x[k];
            x[i] = v / D[i * PP + i];
          }
#pragma unroll
        for (int i = 0; i < XNB; ++i)
          if (i < kb) row[i] = x[i];
      }
      bb_sync();
      // trailing update in the order of the recursive algorithm (as in
      // wg_getrf): the group of g = lowbit(t + 1) finished block columns
      // [c0, c1) updates the next g block columns [c1, r1) below the
      // diagonal, A[c1:, c1:r1] -= L[c1:, c0:c1] L[c1:r1, c0:c1]^T (the
      // entries above the diagonal of that block are updated too and never read)
      const int g = (t + 1) & -(t + 1);
      const int c1 = k0 + kb, c0 = c1 - imin(g * nb, c1), r1 = imin(c1 + g * nb, n);
      if (g == 1)
        wg_chol_update1<T>(sm, n, A, lda, k0, kb, c1, r1 - c1);
      else
        wg_gemm<T>(sm, n - c1, r1 - c1, c1 - c0, T(-1), A + (long long)c1 * lda + c0, lda, false,
                   A + (long long)c1 * lda + c0, lda, true, T(1), A + (long long)c1 * lda + c1, lda);
    }
  }
  return bad;
}

template <typename T>
BB_IN void wg_copy(int n, const T* src, T* dst) {
  n = uni(n);
  const int total = n * n;
  for (int base = bb_tid(); base < total; base += SU * BT) {
    T v[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) v[u] = src[imin(base + u * BT, total - 1)];
#pragma unroll
    for (int u = 0; u < SU; ++u)
      if (base + u * BT < total) dst[base + u * BT] = v[u];
  }
  bb_sync();
}
template <typename T>
BB_IN void wg_identity(int n, T* dst) {
  n = uni(n);
  for (int e = bb_tid(); e < n * n; e += BT) dst[e] = (e / n == e % n) ? T(1) : T(0);
  bb_sync();
}

struct BatchArgs {
  int count;
  const int* n;         // per-matrix order
  const int* kind;      // 0 general, 1 HPD
  const void* const* A;
  const void* const* B;
  void* const* Xr;
  void* const* Xi;
  int* info;            // per matrix: 0, or stage * 1000000 + column (1-based); -1 bad order or kind
  int nmax;             // workspace slots are sized for this order
  const int* order;     // processing order (largest first)
  int* counter;         // queue head
  void* ws;             // per-workgroup slots
  long long slot_elems; // elements (T) per slot
  int nb_table[2][4];   // [kind][size class] panel width
};

BB_IN int size_class(int n) { return n <= 64 ? 0 : n <= 128 ? 1 : n <= 256 ? 2 : 3; }

// Status word of one member: 0, or 1000000 * stage + column.
BB_IN int status_word(int stage, int col) { return col ? 1000000 * stage + col : 0; }

// The persistent worker of workgroup `block`: takes matrices from the queue
// until it is empty.  Every branch that guards a barrier depends only on
// values read through the first lane (uniform to the compiler, not only in
// value), and a failed factorization does not change the control flow: the
// remaining steps run on the (non-finite) values, and the status word records
// the first failing stage and column.  The order and kind are validated
// before they index anything (a kind outside {0, 1} once indexed the
// panel-width table out of bounds).
template <typename T>
BB_IN void batched_worker(const BatchArgs& g, Smem<T>& sm, int block) {
  const int tid = bb_tid();
  T* slot = reinterpret_cast<T*>(g.ws) + (long long)block * g.slot_elems;
  for (;;) {
    if (tid == 0) sm.bcast[0] = bb_atomic_add(g.counter, 1);
    bb_sync();
    const int q = bb_first(sm.bcast[0]);
    bb_sync();
    if (q >= g.count) break;                          // every wave leaves
    const int mi = bb_first(g.order[q]);
    const int n = bb_first(g.n[mi]);
    const int kind = bb_first(g.kind[mi]);
    if (n < 1 || n > g.nmax || (kind != 0 && kind != 1)) {
      if (tid == 0) g.info[mi] = -1;
      continue;
    }
    const int nb = imin(imax(g.nb_table[kind][size_class(n)], 1), PNB);
    const T* A = reinterpret_cast<const T*>(g.A[mi]);
    const T* B = reinterpret_cast<const T*>(g.B[mi]);
    T* Xr = reinterpret_cast<T*>(g.Xr[mi]);
    T* Xi = reinterpret_cast<T*>(g.Xi[mi]);
    const long long nn = (long long)n * n;
    T* F = slot;            // factors of A
    T* Y = slot + nn;       // A^{-1} B
    T* Cm = slot + 2 * nn;  // C and its factors
    int* perm = reinterpret_cast<int*>(slot + 3 * nn);
    int info = 0;
    if (kind == 0) {
      // Algorithm 5
      wg_copy<T>(n, A, F);
      const int i1 = bb_first(wg_getrf<T>(sm, n, F, n, perm, nb));
      info = status_word(1, i1);
      wg_gather_rows<T>(n, n, B, n, perm, Y, n);                        // Y = A^{-1} B = U^{-1} L^{-1} P B
      wg_trsm<T>(sm, 0, n, n, F, n, true, Y, n, nb);
      wg_trsm<T>(sm, 2, n, n, F, n, false, Y, n, nb);
      wg_copy<T>(n, A, Cm);                                             // C = A + B Y
      wg_gemm<T>(sm, n, n, n, T(1), B, n, false, Y, n, false, T(1), Cm, n);
      const int i2 = bb_first(wg_getrf<T>(sm, n, Cm, n, perm, nb));
      if (!info) info = status_word(2, i2);
      // Re X = C^{-1} = U^{-1} L^{-1} P: L^{-1} by a solve against I (lower
      // triangular, n^3 / 3), then U^{-1} (n^3), then the column permutation;
      // the factors of A in F are no longer needed
      wg_identity<T>(n, F);
      wg_trsm<T>(sm, 0, n, n, Cm, n, true, F, n, nb, true);
      wg_trsm<T>(sm, 2, n, n, Cm, n, false, F, n, nb);
      wg_scatter_cols<T>(n, F, perm, Xr);
      wg_gemm<T>(sm, n, n, n, T(-1), Y, n, false, Xr, n, false, T(0), Xi, n);   // Im X = -Y C^{-1}
    } else {
      // Algorithm 7
      wg_copy<T>(n, A, F);
      const int i1 = bb_first(wg_potrf<T>(sm, n, F, n, nb));
      info = status_word(1, i1);
      wg_copy<T>(n, B, Cm);                                             // X1 = R1^{-T} B (Cm as scratch)
      wg_trsm<T>(sm, 0, n, n, F, n, false, Cm, n, nb);
      wg_copy<T>(n, Cm, Y);                                             // Y = R1^{-1} X1
      wg_trsm<T>(sm, 1, n, n, F, n, false, Y, n, nb);
      // C = A - X1^T X1 into F's place (F is no longer needed)
      wg_copy<T>(n, A, F);
      wg_gemm<T>(sm, n, n, n, T(-1), Cm, n, true, Cm, n, false, T(1), F, n, true);   // lower triangle only
      const int i2 = bb_first(wg_potrf<T>(sm, n, F, n, nb));
      if (!info) info = status_word(2, i2);
      // Re X = C^{-1} = R2^{-1} R2^{-T} = W^T W with W = R2^{-T} (lower
      // triangular, a solve against the identity into Cm, whose X1 is no
      // longer needed): one product for the lower triangle, mirrored
      wg_identity<T>(n, Cm);
      wg_trsm<T>(sm, 0, n, n, F, n, false, Cm, n, nb, true);
      wg_gemm<T>(sm, n, n, n, T(1), Cm, n, true, Cm, n, false, T(0), Xr, n, true);
      wg_mirror<T>(n, Xr, T(1));
      // Im X = -Y C^{-1} is skew (X is Hermitian): the lower triangle, mirrored
      wg_gemm<T>(sm, n, n, n, T(-1), Y, n, false, Xr, n, false, T(0), Xi, n, true);
      wg_mirror<T>(n, Xi, T(-1));
    }
    if (tid == 0) g.info[mi] = info;
    bb_sync();
  }
}

// Processing order, largest order first (counting sort on n by one workgroup
// of `nt` threads; hist holds BNMAX + 2 ints of workgroup memory), and reset
// of the queue head (a kernel, not a memset, so the pair can be captured in
// a graph).
BB_IN void batched_order_body(int nt, int count, const int* n, int* order, int* counter, int* hist) {
  const int tid = bb_tid();
  for (int i = tid; i < BNMAX + 2; i += nt) hist[i] = 0;
  bb_sync();
  for (int i = tid; i < count; i += nt) bb_atomic_add(&hist[BNMAX - imin(imax(n[i], 0), BNMAX)], 1);
  bb_sync();
  if (tid == 0) {
    int run = 0;
    for (int b = 0; b <= BNMAX; ++b) { const int c = hist[b]; hist[b] = run; run += c; }
    *counter = 0;
  }
  bb_sync();
  for (int i = tid; i < count; i += nt) {
    const int pos = bb_atomic_add(&hist[BNMAX - imin(imax(n[i], 0), BNMAX)], 1);
    order[pos] = i;
  }
}

}  // namespace bat
}  // namespace frob
