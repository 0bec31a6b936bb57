// gemm_f64.hip -- FP64 matrix-core GEMM for gfx950.
//
//   C = alpha * op(A) * op(B) + beta * C       (row-major, op = N or T)
//
// with optional row indirection on A, B and C, an optional column scatter on
// C, triangular interpretation of op(A)/op(B) (entries outside the triangle are
// read as zero and skipped along k, a unit diagonal reads as one), a
// lower-triangle-only output mode, and a batch index on blockIdx.z.  This one
// kernel serves the trailing updates of the factorizations (row-indirect NN),
// the triangular solves and inverses (trmm-like products), the symmetric
// rank-k updates (lower-only), and the plain products B*Y and -Y*C^{-1}.
//
// Tiling: 256 threads = 4 wave64s, block tile BM x BN, k-step 16.  Each wave
// owns a (BM/WM) x (BN/WN) sub-tile built from 16x16 v_mfma_f64_16x16x4f64
// tiles.  Operand tiles are staged through LDS in the same orientation as in
// HBM (no transposition on the way in; the fragment read indexing handles op),
// with padding chosen so the 16-lane fragment reads hit distinct banks.  The
// next k-tile is fetched into registers while the current one is multiplied.
// Linear block ids are remapped so that each of the 8 XCDs (hardware assigns
// block b to XCD b % 8) works on a contiguous band of tiles, which keeps the
// shared A rows in that XCD's L2.
#include "common.hpp"
#include "internal.hpp"

namespace frob {

struct GemmF64Params {
  int M, N, K;
  double alpha, beta;
  DOp A, B;
  DOut C;
  int triA, triB;
  int lowerOnly;
  long long sA, sB, sC;
  int tilesM, tilesN;
};

__device__ __forceinline__ double tri_mask(double v, int tri, int r, int c) {
  // (r, c) are logical coordinates of the operand element
  switch (tri) {
    case TRI_LOWER: return c > r ? 0.0 : v;
    case TRI_LOWER_UNIT: return c > r ? 0.0 : (c == r ? 1.0 : v);
    case TRI_UPPER: return c < r ? 0.0 : v;
    case TRI_UPPER_UNIT: return c < r ? 0.0 : (c == r ? 1.0 : v);
    default: return v;
  }
}

template <int BM, int BN, int WM, int WN, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmF64Params g) {
  constexpr int BK = 16;
  constexpr int FM = BM / WM / 16;
  constexpr int FN = BN / WN / 16;
  static_assert(WM * WN == 4, "four waves");
  static_assert(FM >= 1 && FN >= 1, "tile too small");
  constexpr int A_LD = TA ? (BM + 16) : (BK + 1);
  constexpr int A_SZ = TA ? BK * A_LD : BM * A_LD;
  constexpr int B_LD = TB ? (BK + 1) : (BN + 16);
  constexpr int B_SZ = TB ? BN * B_LD : BK * B_LD;
  constexpr int A_PER = BM * BK / 256;
  constexpr int B_PER = BN * BK / 256;
  __shared__ double As[A_SZ];
  __shared__ double Bs[B_SZ];

  const int tiles = g.tilesM * g.tilesN;
  const int per = (tiles + 7) / 8;
  const int bid = blockIdx.x;
  const int t = (bid & 7) * per + (bid >> 3);
  if (t >= tiles) return;
  const int bm0 = (t / g.tilesN) * BM;
  const int bn0 = (t % g.tilesN) * BN;
  if (g.lowerOnly && bn0 > bm0 + BM - 1) return;

  const long long z = blockIdx.z;
  const double* __restrict__ Ap = g.A.p + z * g.sA;
  const double* __restrict__ Bp = g.B.p + z * g.sB;
  double* __restrict__ Cp = g.C.p + z * g.sC;
  const int M = g.M, N = g.N;

  // k range that can hold non-zero products for this tile
  int kbeg = 0, kend = g.K;
  if (g.triA == TRI_UPPER || g.triA == TRI_UPPER_UNIT) kbeg = max(kbeg, bm0);
  if (g.triA == TRI_LOWER || g.triA == TRI_LOWER_UNIT) kend = min(kend, bm0 + BM);
  if (g.triB == TRI_LOWER || g.triB == TRI_LOWER_UNIT) kbeg = max(kbeg, bn0);
  if (g.triB == TRI_UPPER || g.triB == TRI_UPPER_UNIT) kend = min(kend, bn0 + BN);
  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wm0 = (w / WN) * (BM / WM);
  const int wn0 = (w % WN) * (BN / WN);

  double ra[A_PER], rb[B_PER];

  auto load_tiles = [&](int kt) {
#pragma unroll
    for (int r = 0; r < A_PER; ++r) {
      const int e = tid + r * 256;
      int i, k;
      if (!TA) { i = e / BK; k = e % BK; } else { k = e / BM; i = e % BM; }
      const int gi = bm0 + i, gk = kt + k;
      double v = 0.0;
      if (gi < M && gk < kend) {
        if (!TA) {
          const int pr = g.A.rows ? g.A.rows[gi] : gi;
          v = Ap[(long long)pr * g.A.ld + gk];
        } else {
          const int pr = g.A.rows ? g.A.rows[gk] : gk;
          v = Ap[(long long)pr * g.A.ld + gi];
        }
        v = tri_mask(v, g.triA, gi, gk);
      }
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < B_PER; ++r) {
      const int e = tid + r * 256;
      int k, j;
      if (!TB) { k = e / BN; j = e % BN; } else { j = e / BK; k = e % BK; }
      const int gk = kt + k, gj = bn0 + j;
      double v = 0.0;
      if (gj < N && gk < kend) {
        if (!TB) {
          const int pr = g.B.rows ? g.B.rows[gk] : gk;
          v = Bp[(long long)pr * g.B.ld + gj];
        } else {
          const int pr = g.B.rows ? g.B.rows[gj] : gj;
          v = Bp[(long long)pr * g.B.ld + gk];
        }
        v = tri_mask(v, g.triB, gk, gj);
      }
      rb[r] = v;
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int r = 0; r < A_PER; ++r) {
      const int e = tid + r * 256;
      if (!TA) { As[(e / BK) * A_LD + (e % BK)] = ra[r]; }
      else { As[(e / BM) * A_LD + (e % BM)] = ra[r]; }
    }
#pragma unroll
    for (int r = 0; r < B_PER; ++r) {
      const int e = tid + r * 256;
      if (!TB) { Bs[(e / BN) * B_LD + (e % BN)] = rb[r]; }
      else { Bs[(e / BK) * B_LD + (e % BK)] = rb[r]; }
    }
  };

  d4 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  if (nk > 0) load_tiles(kbeg);
  for (int it = 0; it < nk; ++it) {
    store_tiles();
    __syncthreads();
    if (it + 1 < nk) load_tiles(kbeg + (it + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int k = kk * 4 + (lane >> 4);
      double af[FM], bf[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) {
        const int i = wm0 + a * 16 + (lane & 15);
        af[a] = TA ? As[k * A_LD + i] : As[i * A_LD + k];
      }
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int j = wn0 + b * 16 + (lane & 15);
        bf[b] = TB ? Bs[j * B_LD + k] : Bs[k * B_LD + j];
      }
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }

  // epilogue: lane holds D[l/16 + 4v][l%16] of each 16x16 tile
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = bm0 + wm0 + a * 16 + (lane >> 4) + 4 * v;
        const int j = bn0 + wn0 + b * 16 + (lane & 15);
        if (i < M && j < N && (!g.lowerOnly || i >= j)) {
          const int pr = g.C.rows ? g.C.rows[i] : i;
          const int pc = g.C.cols ? g.C.cols[j] : j;
          double* cp = Cp + (long long)pr * g.C.ld + pc;
          double val = g.alpha * acc[a][b][v];
          if (g.beta != 0.0) val += g.beta * *cp;
          *cp = val;
        }
      }
}

template <int BM, int BN, int WM, int WN, bool TA, bool TB>
static void launch_cfg(const GemmF64Params& p0, int batch, hipStream_t s) {
  GemmF64Params p = p0;
  p.tilesM = ceil_div(p.M, BM);
  p.tilesN = ceil_div(p.N, BN);
  const int tiles = p.tilesM * p.tilesN;
  const int grid = 8 * ((tiles + 7) / 8);
  hipLaunchKernelGGL((k_gemm_f64<BM, BN, WM, WN, TA, TB>), dim3(grid, 1, batch), dim3(256), 0, s, p);
  FROB_LAUNCH_CHECK();
}

template <bool TA, bool TB>
static void launch_pick(const GemmF64Params& p, int batch, int cfg, hipStream_t s) {
  switch (cfg) {
    case GEMM_CFG_128x128: launch_cfg<128, 128, 2, 2, TA, TB>(p, batch, s); break;
    case GEMM_CFG_64x64: launch_cfg<64, 64, 2, 2, TA, TB>(p, batch, s); break;
    case GEMM_CFG_128x32: launch_cfg<128, 32, 4, 1, TA, TB>(p, batch, s); break;
    case GEMM_CFG_32x128: launch_cfg<32, 128, 1, 4, TA, TB>(p, batch, s); break;
    default: throw std::runtime_error("gemm_f64: bad tile config");
  }
}

int gemm_pick_cfg(int M, int N, int need) {
  if (need == GEMM_NEED_FULL_M) return M <= 64 ? GEMM_CFG_64x64 : GEMM_CFG_128x128;
  if (need == GEMM_NEED_FULL_N) return N <= 64 ? GEMM_CFG_64x64 : GEMM_CFG_128x128;
  if (N <= 32) return GEMM_CFG_128x32;
  if (M <= 32) return GEMM_CFG_32x128;
  const long long big_tiles = (long long)ceil_div(M, 128) * ceil_div(N, 128);
  if (big_tiles >= 192) return GEMM_CFG_128x128;
  return GEMM_CFG_64x64;
}

void gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, DOp A, int triA, DOp B,
              int triB, double beta, DOut C, bool lowerOnly, int batch, long long sA, long long sB,
              long long sC, int need) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0 && beta == 1.0) return;
  GemmF64Params p;
  p.M = M; p.N = N; p.K = K < 0 ? 0 : K;
  p.alpha = alpha; p.beta = beta;
  p.A = A; p.B = B; p.C = C;
  p.triA = triA; p.triB = triB;
  p.lowerOnly = lowerOnly ? 1 : 0;
  p.sA = sA; p.sB = sB; p.sC = sC;
  const int cfg = gemm_pick_cfg(M, N, need);
  if (!ta && !tb) launch_pick<false, false>(p, batch, cfg, s);
  else if (!ta && tb) launch_pick<false, true>(p, batch, cfg, s);
  else if (ta && !tb) launch_pick<true, false>(p, batch, cfg, s);
  else launch_pick<true, true>(p, batch, cfg, s);
}

}  // namespace frob
