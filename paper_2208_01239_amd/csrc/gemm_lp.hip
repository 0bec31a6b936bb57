// gemm_lp.hip -- low-precision matrix-core GEMM for gfx950:
//
//   C = alpha * op(A) * op(B) + beta * C       (row-major, op = N or T)
//
// with the operands rounded to FP32 (v_mfma_f32_16x16x4f32) or to BF16
// (v_mfma_f32_16x16x32_bf16) when a tile is staged, and FP32 accumulation.
// Storage is FP64 (the mixed-precision factorization: working matrices stay
// FP64 in HBM, only the MFMA operands are rounded) or FP32 (the batched
// adjoint).  Row indirection on A, B and C, a lower-triangle-only output mode
// and a batch index on blockIdx.z follow the FP64 GEMM's conventions.
//
// Tiling: 256 threads = 4 wave64s in a 2x2 grid, block tile BM x BN, k-step
// 32.  A tile is read from HBM with one batch of unconditional loads at
// clamped addresses (the next k-step's batch is in flight while the current
// one is multiplied; row indices are fetched a k-step earlier still),
// rounded, and written to LDS k-major, which is the
// order the MFMA fragments read (16 consecutive lanes, 16 consecutive
// floats).  Fragment layouts (lane l): A[l % 16][k] / B[k][l % 16] with
// k = l / 16 (FP32, one value) or k = 8 (l / 16) + 0..7 (BF16, eight values);
// the 16x16 result holds D[4 (l / 16) + v][l % 16] in accumulator v.
#include "common.hpp"
#include "internal.hpp"

namespace frob {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename TS>
struct GemmLpParams {
  int M, N, K;
  double alpha, beta;
  const TS* A; int lda; const int* rA;
  const TS* B; int ldb; const int* rB;
  TS* C; int ldc; const int* rC;
  long long sA, sB, sC;   // batch strides of the data pointers
  int lowerOnly;
  int tilesM, tilesN;
};

constexpr int LBK = 32;

template <typename TS, int MODE, int BM, int BN, bool TA, bool TB>
__global__ __launch_bounds__(256, (BM * BN > 64 * 64) ? 1 : 2) void k_gemm_lp(GemmLpParams<TS> g) {
  constexpr int PA = BM + 4, PB = BN + 4;            // LDS row pitch (floats)
  constexpr int EA = BM * LBK / 256, EB = BN * LBK / 256;
  constexpr int FM = BM / 32, FN = BN / 32;          // 16x16 tiles per wave
  __shared__ float As[LBK * PA];
  __shared__ float Bs[LBK * PB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles = g.tilesM * g.tilesN;
  const int per = (tiles + 7) / 8;
  const int bid = blockIdx.x;
  const int t = (bid & 7) * per + (bid >> 3);        // XCD-contiguous ranges of tile indices
  if (t >= tiles) return;
  // tile indices run through groups of eight tile-rows column by column
  const int gsz = 8 * g.tilesN;
  const int grp = t / gsz;
  const int gh = min(8, g.tilesM - grp * 8);
  const int wt = t - grp * gsz;
  const int bm0 = (grp * 8 + wt % gh) * BM;
  const int bn0 = (wt / gh) * BN;
  if (g.lowerOnly && bn0 > bm0 + BM - 1) return;
  const int z = blockIdx.z;
  const TS* Ap = g.A + z * g.sA;
  const TS* Bp = g.B + z * g.sB;
  TS* Cp = g.C + z * g.sC;
  const int M = g.M, N = g.N, K = g.K;

  // Element u of this thread's share of a tile is the logical (row, k) pair
  // below.  The physical rows of the row-band operands (A for N, B for T) do
  // not change with k and are looked up once; the k-band operands' row
  // indices are fetched one k-step ahead of their data, unconditionally (from
  // a readable stand-in when there is no index array; the value is then
  // ignored), so no wait on an index stalls the products.
  constexpr int RA = TA ? 1 : EA, RB = TB ? EB : 1;
  constexpr int XA = TA ? EA : 1, XB = TB ? 1 : EB;
  int rowA[RA], rowB[RB], ixa[XA], ixb[XB];
  if (!TA) {
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      const int gi = min(bm0 + (tid + 256 * u) / LBK, M - 1);
      rowA[u] = g.rA ? g.rA[gi] : gi;
    }
  }
  if (TB) {
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int gj = min(bn0 + (tid + 256 * u) / LBK, N - 1);
      rowB[u] = g.rB ? g.rB[gj] : gj;
    }
  }
  const int* rAs = g.rA ? g.rA : reinterpret_cast<const int*>(Ap);
  const int* rBs = g.rB ? g.rB : reinterpret_cast<const int*>(Bp);
  auto load_index = [&](int k0) {
    if (TA) {
#pragma unroll
      for (int u = 0; u < EA; ++u) ixa[u] = rAs[min(k0 + (tid + 256 * u) / BM, K - 1)];
    }
    if (!TB) {
#pragma unroll
      for (int u = 0; u < EB; ++u) ixb[u] = rBs[min(k0 + (tid + 256 * u) / BN, K - 1)];
    }
  };
  TS ra[EA], rb[EB];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      const int e = tid + 256 * u;
      if (!TA) {
        ra[u] = Ap[(long long)rowA[u] * g.lda + min(k0 + e % LBK, K - 1)];
      } else {
        const int gk = min(k0 + e / BM, K - 1), gi = min(bm0 + e % BM, M - 1);
        ra[u] = Ap[(long long)(g.rA ? ixa[u] : gk) * g.lda + gi];
      }
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int e = tid + 256 * u;
      if (!TB) {
        const int gk = min(k0 + e / BN, K - 1), gj = min(bn0 + e % BN, N - 1);
        rb[u] = Bp[(long long)(g.rB ? ixb[u] : gk) * g.ldb + gj];
      } else {
        rb[u] = Bp[(long long)rowB[u] * g.ldb + min(k0 + e % LBK, K - 1)];
      }
    }
  };
  auto store_tiles = [&](int k0) {
#pragma unroll
    for (int u = 0; u < EA; ++u) {
      const int e = tid + 256 * u;
      int i, k;
      if (!TA) { i = e / LBK; k = e % LBK; } else { k = e / BM; i = e % BM; }
      const bool ok = bm0 + i < M && k0 + k < K;
      As[k * PA + i] = ok ? (float)ra[u] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int e = tid + 256 * u;
      int k, j;
      if (!TB) { k = e / BN; j = e % BN; } else { j = e / LBK; k = e % LBK; }
      const bool ok = bn0 + j < N && k0 + k < K;
      Bs[k * PB + j] = ok ? (float)rb[u] : 0.0f;
    }
  };

  const int wm0 = (wave >> 1) * (BM / 2), wn0 = (wave & 1) * (BN / 2);
  f4 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

  const int nk = (K + LBK - 1) / LBK;
  if (nk > 0) {
    load_index(0);
    load_tiles(0);
    if (nk > 1) load_index(LBK);
  }
  for (int it = 0; it < nk; ++it) {
    store_tiles(it * LBK);
    __syncthreads();
    if (it + 1 < nk) {
      load_tiles((it + 1) * LBK);
      if (it + 2 < nk) load_index((it + 2) * LBK);
    }
    if (MODE == LP_F32) {
#pragma unroll
      for (int kk = 0; kk < LBK; kk += 4) {
        float fa[FM], fb[FN];
#pragma unroll
        for (int a = 0; a < FM; ++a) fa[a] = As[(kk + (lane >> 4)) * PA + wm0 + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < FN; ++b) fb[b] = Bs[(kk + (lane >> 4)) * PB + wn0 + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a], fb[b], acc[a][b], 0, 0, 0);
      }
    } else {
      bf16x8 fa[FM], fb[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int q = 0; q < 8; ++q) fa[a][q] = (__bf16)As[(8 * (lane >> 4) + q) * PA + wm0 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int q = 0; q < 8; ++q) fb[b][q] = (__bf16)Bs[(8 * (lane >> 4) + q) * PB + wn0 + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }

  // epilogue: accumulator v of tile (a, b) is D[4 (l / 16) + v][l % 16]
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    long long ro[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ic = min(bm0 + wm0 + a * 16 + 4 * (lane >> 4) + v, M - 1);
      ro[v] = (long long)(g.rC ? g.rC[ic] : ic) * g.ldc;
    }
    TS cold[4][FN];
    if (g.beta != 0.0) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int b = 0; b < FN; ++b) cold[v][b] = Cp[ro[v] + min(bn0 + wn0 + b * 16 + (lane & 15), N - 1)];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = bm0 + wm0 + a * 16 + 4 * (lane >> 4) + v;
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int j = bn0 + wn0 + b * 16 + (lane & 15);
        if (i < M && j < N && (!g.lowerOnly || i >= j)) {
          double val = g.alpha * (double)acc[a][b][v];
          if (g.beta != 0.0) val += g.beta * (double)cold[v][b];
          Cp[ro[v] + j] = (TS)val;
        }
      }
    }
  }
}

template <typename TS, int MODE, int BM, int BN, bool TA, bool TB>
void launch_lp(GemmLpParams<TS> p, int batch, hipStream_t s) {
  p.tilesM = ceil_div(p.M, BM);
  p.tilesN = ceil_div(p.N, BN);
  const int tiles = p.tilesM * p.tilesN;
  const int grid = 8 * ((tiles + 7) / 8);
  hipLaunchKernelGGL((k_gemm_lp<TS, MODE, BM, BN, TA, TB>), dim3(grid, 1, batch), dim3(256), 0, s, p);
  FROB_LAUNCH_CHECK();
}

template <typename TS, int MODE, bool TA, bool TB>
void pick_lp(const GemmLpParams<TS>& p, int batch, hipStream_t s) {
  const long long big = (long long)ceil_div(p.M, 128) * ceil_div(p.N, 128) * batch;
  if (big >= 160) launch_lp<TS, MODE, 128, 128, TA, TB>(p, batch, s);
  else launch_lp<TS, MODE, 64, 64, TA, TB>(p, batch, s);
}

template <typename TS>
void gemm_lp_t(hipStream_t s, int mode, bool ta, bool tb, int M, int N, int K, double alpha, const TS* A, int lda,
               const int* rA, const TS* B, int ldb, const int* rB, double beta, TS* C, int ldc, const int* rC,
               bool lowerOnly, int batch, long long sA, long long sB, long long sC) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0 && beta == 1.0) return;
  GemmLpParams<TS> p;
  p.M = M; p.N = N; p.K = K < 0 ? 0 : K;
  p.alpha = alpha; p.beta = beta;
  p.A = A; p.lda = lda; p.rA = rA;
  p.B = B; p.ldb = ldb; p.rB = rB;
  p.C = C; p.ldc = ldc; p.rC = rC;
  p.sA = sA; p.sB = sB; p.sC = sC;
  p.lowerOnly = lowerOnly ? 1 : 0;
  p.tilesM = p.tilesN = 0;
  if (mode == LP_F32) {
    if (!ta && !tb) pick_lp<TS, LP_F32, false, false>(p, batch, s);
    else if (!ta && tb) pick_lp<TS, LP_F32, false, true>(p, batch, s);
    else if (ta && !tb) pick_lp<TS, LP_F32, true, false>(p, batch, s);
    else pick_lp<TS, LP_F32, true, true>(p, batch, s);
  } else if (mode == LP_BF16) {
    if (!ta && !tb) pick_lp<TS, LP_BF16, false, false>(p, batch, s);
    else if (!ta && tb) pick_lp<TS, LP_BF16, false, true>(p, batch, s);
    else if (ta && !tb) pick_lp<TS, LP_BF16, true, false>(p, batch, s);
    else pick_lp<TS, LP_BF16, true, true>(p, batch, s);
  } else {
    throw std::runtime_error("gemm_lp: unknown precision mode");
  }
}

}  // namespace

void gemm_lp(hipStream_t s, int mode, bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
             const int* rA, const double* B, int ldb, const int* rB, double beta, double* C, int ldc, const int* rC,
             bool lowerOnly, int batch, long long sA, long long sB, long long sC) {
  gemm_lp_t<double>(s, mode, ta, tb, M, N, K, alpha, A, lda, rA, B, ldb, rB, beta, C, ldc, rC, lowerOnly, batch, sA,
                    sB, sC);
}

void gemm_lp(hipStream_t s, int mode, bool ta, bool tb, int M, int N, int K, double alpha, const float* A, int lda,
             const int* rA, const float* B, int ldb, const int* rB, double beta, float* C, int ldc, const int* rC,
             bool lowerOnly, int batch, long long sA, long long sB, long long sC) {
  gemm_lp_t<float>(s, mode, ta, tb, M, N, K, alpha, A, lda, rA, B, ldb, rB, beta, C, ldc, rC, lowerOnly, batch, sA,
                   sB, sC);
}

}  // namespace frob
