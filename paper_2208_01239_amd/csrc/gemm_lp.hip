// gemm_lp.hip -- low-precision matrix-core GEMM for gfx950:
//
//   C = alpha * op(A) * op(B) + beta * C       (row-major, op = N or T)
//
// with the operands rounded to FP32 (v_mfma_f32_16x16x4f32) or to BF16
// (v_mfma_f32_16x16x32_bf16) when a tile is staged, and FP32 accumulation.
// Storage is FP64 (the mixed-precision factorization: working matrices stay
// FP64 in HBM, only the MFMA operands are rounded) or FP32 (the batched
// adjoint).  Row indirection on A, B and C, a lower-triangle-only output mode
// and the batch index (folded into blockIdx.x except for lower-triangle-only
// products) follow the FP64 GEMM's conventions.
//
// Tiling: 256 threads = 4 wave64s in a 2x2 grid, block tile BM x BN, k-step
// 32.  A tile is read from HBM with one batch of unconditional loads at
// clamped addresses (the next k-step's batch is in flight while the current
// one is multiplied; row indices are fetched a k-step earlier still),
// rounded, and written to LDS: FP32 k-major, the order the MFMA fragments
// read (16 consecutive lanes, 16 consecutive floats); BF16 row by row with k
// contiguous, so that each lane's eight values are one 16-byte read.
// Fragment layouts (lane l): A[l % 16][k] / B[k][l % 16] with
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
  int flat;               // > 0: that many batch entries folded into blockIdx.x (else batch on blockIdx.z)
};

constexpr int LBK = 32;

template <typename TS, int MODE, int BM, int BN, bool TA, bool TB>
__global__ __launch_bounds__(256, (BM * BN > 64 * 64) ? 1 : 2) void k_gemm_lp(GemmLpParams<TS> g) {
  constexpr int PA = BM + 4, PB = BN + 4;            // LDS row pitch (floats)
  constexpr int EA = BM * LBK / 256, EB = BN * LBK / 256;
  constexpr int FM = BM / 32, FN = BN / 32;          // 16x16 tiles per wave
  // FP32 operands are staged k-major as floats; BF16 operands are converted
  // once when staged and kept k-contiguous per row (pitch PH), so that a
  // lane's fragment of eight consecutive k is one aligned 16-byte read
  constexpr bool HB = MODE == LP_BF16;
  constexpr int PH = LBK + 8;
  __shared__ float As[HB ? 1 : LBK * PA];
  __shared__ float Bs[HB ? 1 : LBK * PB];
  __shared__ __attribute__((aligned(16))) __bf16 Ah[HB ? BM * PH : 8];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[HB ? BN * PH : 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles = g.tilesM * g.tilesN;
  const int bid = blockIdx.x;
  // XCD-contiguous ranges of work items (a tile of a batch entry, the entries
  // folded in when g.flat > 0, so that every XCD gets its share of a batch of
  // small products); interleaved tiles for lower-only products (the idle
  // tiles above the diagonal would otherwise leave whole XCDs idle)
  const int items = g.flat > 0 ? tiles * g.flat : tiles;
  const int per = (items + 7) / 8;
  const int wi = g.lowerOnly ? bid : (bid & 7) * per + (bid >> 3);
  if (wi >= items) return;
  const int t = g.flat > 0 ? wi % tiles : wi;
  // tile indices run through groups of eight tile-rows column by column
  const int gsz = 8 * g.tilesN;
  const int grp = t / gsz;
  const int gh = min(8, g.tilesM - grp * 8);
  const int wt = t - grp * gsz;
  const int bm0 = (grp * 8 + wt % gh) * BM;
  const int bn0 = (wt / gh) * BN;
  if (g.lowerOnly && bn0 > bm0 + BM - 1) return;
  const int z = g.flat > 0 ? wi / tiles : (int)blockIdx.z;
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
      if constexpr (HB) Ah[i * PH + k] = (__bf16)(ok ? (float)ra[u] : 0.0f);
      else As[k * PA + i] = ok ? (float)ra[u] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int e = tid + 256 * u;
      int k, j;
      if (!TB) { k = e / BN; j = e % BN; } else { j = e / LBK; k = e % LBK; }
      const bool ok = bn0 + j < N && k0 + k < K;
      if constexpr (HB) Bh[j * PH + k] = (__bf16)(ok ? (float)rb[u] : 0.0f);
      else Bs[k * PB + j] = ok ? (float)rb[u] : 0.0f;
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
      // lane l supplies A(l % 16, 8 (l / 16) + q) and B(8 (l / 16) + q, l % 16), q < 8
      bf16x8 fa[FM], fb[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a)
        fa[a] = *reinterpret_cast<const bf16x8*>(&Ah[(wm0 + a * 16 + (lane & 15)) * PH + 8 * (lane >> 4)]);
#pragma unroll
      for (int b = 0; b < FN; ++b)
        fb[b] = *reinterpret_cast<const bf16x8*>(&Bh[(wn0 + b * 16 + (lane & 15)) * PH + 8 * (lane >> 4)]);
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

// FP32-operand kernel, built like the FP64 GEMM: k-step 32 through a
// double-buffered LDS ring (one barrier per k-step), the next tile's global
// loads (pairs along the contiguous direction, 16 or 8 bytes when aligned)
// in flight while the current tile is multiplied, two workgroups per CU.
// Row-band operands (A for N, B for T) sit in LDS as [rows][32 + 4] and
// k-band operands as [32][cols + 16] floats: the fragment reads (16 rows x 4
// k, or 4 k x 16 columns) then fall on distinct banks.
template <typename TS, int BM, int BN, bool TA, bool TB, bool VEC>
__global__ __launch_bounds__(256, 2) void k_gemm_lp32(GemmLpParams<TS> g) {
  constexpr int KP = LBK / 2;                       // pairs per row of a row-band tile
  constexpr int RP = 256 / KP;                      // rows of a row-band tile per pass
  constexpr int RB_LD = LBK + 4, KB_PAD = 16;
  constexpr int A_LD = TA ? BM + KB_PAD : RB_LD;
  constexpr int A_SZ = TA ? LBK * A_LD : BM * A_LD;
  constexpr int B_LD = TB ? RB_LD : BN + KB_PAD;
  constexpr int B_SZ = TB ? BN * B_LD : LBK * B_LD;
  constexpr int A_P = BM * LBK / 512, B_P = BN * LBK / 512;   // pairs per thread per tile
  constexpr int FM = BM / 32, FN = BN / 32;         // 16x16 tiles per wave (2x2 waves)
  __shared__ __attribute__((aligned(16))) float smem[2 * (A_SZ + B_SZ)];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles = g.tilesM * g.tilesN;
  const int bid = blockIdx.x;
  // XCD-contiguous ranges of work items (a tile of a batch entry, the entries
  // folded in when g.flat > 0, so that every XCD gets its share of a batch of
  // small products); interleaved tiles for lower-only products (the idle
  // tiles above the diagonal would otherwise leave whole XCDs idle)
  const int items = g.flat > 0 ? tiles * g.flat : tiles;
  const int per = (items + 7) / 8;
  const int wi = g.lowerOnly ? bid : (bid & 7) * per + (bid >> 3);
  if (wi >= items) return;
  const int t = g.flat > 0 ? wi % tiles : wi;
  const int gsz = 8 * g.tilesN;
  const int grp = t / gsz;
  const int gh = min(8, g.tilesM - grp * 8);
  const int wt = t - grp * gsz;
  const int bm0 = (grp * 8 + wt % gh) * BM;
  const int bn0 = (wt / gh) * BN;
  if (g.lowerOnly && bn0 > bm0 + BM - 1) return;
  const int z = g.flat > 0 ? wi / tiles : (int)blockIdx.z;
  const TS* Ap = g.A + z * g.sA;
  const TS* Bp = g.B + z * g.sB;
  TS* Cp = g.C + z * g.sC;
  const int M = g.M, N = g.N, K = g.K;

  // row-band rows are fixed across k: pointers looked up once
  const TS* aRow[TA ? 1 : A_P];
  int aOk[TA ? 1 : A_P];
  const TS* bRow[TB ? B_P : 1];
  int bOk[TB ? B_P : 1];
  if (!TA) {
#pragma unroll
    for (int p = 0; p < A_P; ++p) {
      const int gi = bm0 + tid / KP + RP * p;
      aOk[p] = gi < M;
      const int gc = min(gi, M - 1);
      aRow[p] = Ap + (long long)(g.rA ? g.rA[gc] : gc) * g.lda;
    }
  }
  if (TB) {
#pragma unroll
    for (int p = 0; p < B_P; ++p) {
      const int gj = bn0 + tid / KP + RP * p;
      bOk[p] = gj < N;
      const int gc = min(gj, N - 1);
      bRow[p] = Bp + (long long)(g.rB ? g.rB[gc] : gc) * g.ldb;
    }
  }
  // k-band row indices are fetched one k-step ahead of their data, from a
  // readable stand-in when there is no index array (the value is then unused)
  constexpr int KA = TA ? A_P : 1, KB = TB ? 1 : B_P;
  const int* rAs = g.rA ? g.rA : reinterpret_cast<const int*>(Ap);
  const int* rBs = g.rB ? g.rB : reinterpret_cast<const int*>(Bp);
  int ixa[KA], ixb[KB];
  auto load_index = [&](int k0) {
    if (TA) {
      constexpr int TPR = BM / 2, RPP = 256 / TPR;
#pragma unroll
      for (int p = 0; p < KA; ++p) ixa[p] = rAs[min(k0 + tid / TPR + RPP * p, K - 1)];
    }
    if (!TB) {
      constexpr int TPR = BN / 2, RPP = 256 / TPR;
#pragma unroll
      for (int p = 0; p < KB; ++p) ixb[p] = rBs[min(k0 + tid / TPR + RPP * p, K - 1)];
    }
  };
  // a pair at (c, c + 1) of a row whose extent is lim, at a clamped address
  auto ld_pair = [&](const TS* row, int c, int lim, float& x, float& y) {
    if (VEC) {
      if constexpr (sizeof(TS) == 8) {
        const double2 v = *reinterpret_cast<const double2*>(row + min(c, (lim - 1) & ~1));
        x = (float)v.x; y = (float)v.y;
      } else {
        const float2 v = *reinterpret_cast<const float2*>(row + min(c, (lim - 1) & ~1));
        x = v.x; y = v.y;
      }
    } else {
      x = (float)row[min(c, lim - 1)];
      y = (float)row[min(c + 1, lim - 1)];
    }
  };
  float ra[A_P][2], rb[B_P][2];
  auto load_tiles = [&](int k0) {
    if (!TA) {
      const int gk = k0 + (tid % KP) * 2;
#pragma unroll
      for (int p = 0; p < A_P; ++p) ld_pair(aRow[p], gk, K, ra[p][0], ra[p][1]);
    } else {
      constexpr int TPR = BM / 2, RPP = 256 / TPR;
      const int gi = bm0 + (tid % TPR) * 2;
#pragma unroll
      for (int p = 0; p < A_P; ++p) {
        const int gk = min(k0 + tid / TPR + RPP * p, K - 1);
        ld_pair(Ap + (long long)(g.rA ? ixa[p] : gk) * g.lda, gi, M, ra[p][0], ra[p][1]);
      }
    }
    if (!TB) {
      constexpr int TPR = BN / 2, RPP = 256 / TPR;
      const int gj = bn0 + (tid % TPR) * 2;
#pragma unroll
      for (int p = 0; p < B_P; ++p) {
        const int gk = min(k0 + tid / TPR + RPP * p, K - 1);
        ld_pair(Bp + (long long)(g.rB ? ixb[p] : gk) * g.ldb, gj, N, rb[p][0], rb[p][1]);
      }
    } else {
      const int gk = k0 + (tid % KP) * 2;
#pragma unroll
      for (int p = 0; p < B_P; ++p) ld_pair(bRow[p], gk, K, rb[p][0], rb[p][1]);
    }
  };
  // mask the loaded tile of k-step k0 and write it to LDS stage `st`
  auto store_tiles = [&](int st, int k0) {
    float* As = smem + st * (A_SZ + B_SZ);
    float* Bs = As + A_SZ;
#pragma unroll
    for (int p = 0; p < A_P; ++p) {
      if (!TA) {
        const int r = tid / KP + RP * p, gk = k0 + (tid % KP) * 2;
        const bool ok = aOk[p];
        *reinterpret_cast<float2*>(&As[r * A_LD + (tid % KP) * 2]) =
            make_float2((ok && gk < K) ? ra[p][0] : 0.f, (ok && gk + 1 < K) ? ra[p][1] : 0.f);
      } else {
        constexpr int TPR = BM / 2, RPP = 256 / TPR;
        const int kr = tid / TPR + RPP * p, gi = bm0 + (tid % TPR) * 2;
        const bool ok = k0 + kr < K;
        *reinterpret_cast<float2*>(&As[kr * A_LD + (tid % TPR) * 2]) =
            make_float2((ok && gi < M) ? ra[p][0] : 0.f, (ok && gi + 1 < M) ? ra[p][1] : 0.f);
      }
    }
#pragma unroll
    for (int p = 0; p < B_P; ++p) {
      if (TB) {
        const int r = tid / KP + RP * p, gk = k0 + (tid % KP) * 2;
        const bool ok = bOk[p];
        *reinterpret_cast<float2*>(&Bs[r * B_LD + (tid % KP) * 2]) =
            make_float2((ok && gk < K) ? rb[p][0] : 0.f, (ok && gk + 1 < K) ? rb[p][1] : 0.f);
      } else {
        constexpr int TPR = BN / 2, RPP = 256 / TPR;
        const int kr = tid / TPR + RPP * p, gj = bn0 + (tid % TPR) * 2;
        const bool ok = k0 + kr < K;
        *reinterpret_cast<float2*>(&Bs[kr * B_LD + (tid % TPR) * 2]) =
            make_float2((ok && gj < N) ? rb[p][0] : 0.f, (ok && gj + 1 < N) ? rb[p][1] : 0.f);
      }
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
    store_tiles(0, 0);
    __syncthreads();
  }
  for (int it = 0; it < nk; ++it) {
    const int st = it & 1;
    if (it + 1 < nk) {
      load_tiles((it + 1) * LBK);
      if (it + 2 < nk) load_index((it + 2) * LBK);
    }
    const float* As = smem + st * (A_SZ + B_SZ);
    const float* Bs = As + A_SZ;
#pragma unroll
    for (int kk = 0; kk < LBK; kk += 4) {
      const int k = kk + (lane >> 4);
      float fa[FM], fb[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) {
        const int i = wm0 + a * 16 + (lane & 15);
        fa[a] = TA ? As[k * A_LD + i] : As[i * A_LD + k];
      }
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int j = wn0 + b * 16 + (lane & 15);
        fb[b] = TB ? Bs[j * B_LD + k] : Bs[k * B_LD + j];
      }
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    if (it + 1 < nk) store_tiles(st ^ 1, (it + 1) * LBK);
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

// A batch of more than one entry (not lower-only) is folded into blockIdx.x;
// returns the grid's z extent.
template <typename TS>
int flat_batch(GemmLpParams<TS>& p, int batch) {
  p.flat = (batch > 1 && !p.lowerOnly) ? batch : 0;
  return p.flat > 0 ? 1 : batch;
}

template <typename TS, int BM, int BN, bool TA, bool TB>
void launch_lp32(GemmLpParams<TS> p, int batch, hipStream_t s, bool vec) {
  p.tilesM = ceil_div(p.M, BM);
  p.tilesN = ceil_div(p.N, BN);
  const int gz = flat_batch(p, batch);
  const int grid = 8 * ((p.tilesM * p.tilesN * (p.flat > 0 ? p.flat : 1) + 7) / 8);
  if (vec)
    hipLaunchKernelGGL((k_gemm_lp32<TS, BM, BN, TA, TB, true>), dim3(grid, 1, gz), dim3(256), 0, s, p);
  else
    hipLaunchKernelGGL((k_gemm_lp32<TS, BM, BN, TA, TB, false>), dim3(grid, 1, gz), dim3(256), 0, s, p);
  FROB_LAUNCH_CHECK();
}

template <typename TS, int MODE, int BM, int BN, bool TA, bool TB>
void launch_lp(GemmLpParams<TS> p, int batch, hipStream_t s) {
  p.tilesM = ceil_div(p.M, BM);
  p.tilesN = ceil_div(p.N, BN);
  const int gz = flat_batch(p, batch);
  const int grid = 8 * ((p.tilesM * p.tilesN * (p.flat > 0 ? p.flat : 1) + 7) / 8);
  hipLaunchKernelGGL((k_gemm_lp<TS, MODE, BM, BN, TA, TB>), dim3(grid, 1, gz), dim3(256), 0, s, p);
  FROB_LAUNCH_CHECK();
}

template <typename TS>
bool pairs_ok(const TS* p, int ld, long long st, int extent) {
  return (reinterpret_cast<uintptr_t>(p) % (2 * sizeof(TS))) == 0 && ld % 2 == 0 && st % 2 == 0 && extent % 2 == 0;
}

template <typename TS, int MODE, bool TA, bool TB>
void pick_lp(const GemmLpParams<TS>& p, int batch, hipStream_t s) {
  const long long big = (long long)ceil_div(p.M, 128) * ceil_div(p.N, 128) * batch;
  if (MODE == LP_F32) {
    // pairs along each operand's contiguous direction, aligned to their size
    const bool vec = pairs_ok(p.A, p.lda, p.sA, TA ? p.M : p.K) && pairs_ok(p.B, p.ldb, p.sB, TB ? p.K : p.N);
    if (big >= 160) launch_lp32<TS, 128, 128, TA, TB>(p, batch, s, vec);
    else launch_lp32<TS, 64, 64, TA, TB>(p, batch, s, vec);
    return;
  }
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
  p.flat = 0;
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
