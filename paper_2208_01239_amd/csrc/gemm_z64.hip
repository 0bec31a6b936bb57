// gemm_z64.hip -- planar complex FP64 matrix-core GEMM for gfx950 (the
// complex-arithmetic baselines: Algorithms 4 and 8 in complex arithmetic).
//
//   C = alpha * op(A) * op(B) + beta * C,   op in {N, T, C = conjugate transpose},
//
// real alpha, beta; complex matrices stored planar (separate real and
// imaginary arrays with one leading dimension).  Same tiling, staging, row
// indirection, triangular masks, lower-only output and XCD-aware block order
// as the real kernel in gemm_f64.hip; each complex tile product is four real
// v_mfma_f64_16x16x4f64 products on the two planes:
//   Re C += Re A Re B - Im A Im B,   Im C += Re A Im B + Im A Re B,
// with the imaginary fragment of a conjugated operand negated once per k-step.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace frob {

struct GemmZ64Params {
  int M, N, K;
  double alpha, beta;
  ZOp A, B;
  ZOut C;
  int conjA, conjB;
  int triA, triB;
  int lowerOnly;
  int vecA, vecB;
  long long sA, sB, sC;      // batch strides (both planes)
  int rsA, rsB, rsC;         // batch strides of the row-index pointers
  int tilesM, tilesN;
  int flat;                  // > 0: that many batch entries folded into blockIdx.x (else batch on blockIdx.z)
};

__device__ __forceinline__ void ztri_mask(double& re, double& im, int tri, int r, int c) {
  switch (tri) {
    case TRI_LOWER: if (c > r) { re = 0.0; im = 0.0; } break;
    case TRI_LOWER_UNIT: if (c > r) { re = 0.0; im = 0.0; } else if (c == r) { re = 1.0; im = 0.0; } break;
    case TRI_UPPER: if (c < r) { re = 0.0; im = 0.0; } break;
    case TRI_UPPER_UNIT: if (c < r) { re = 0.0; im = 0.0; } else if (c == r) { re = 1.0; im = 0.0; } break;
    default: break;
  }
}

// LDS of the double-buffered planar operand tiles, in doubles
constexpr int zgemm_lds_doubles(int BM, int BN, int BK, bool TA, bool TB) {
  return 2 * 2 * ((TA ? BK * (BM + 16) : BM * (BK + 2)) + (TB ? BN * (BK + 2) : BK * (BN + 16)));
}

// One output tile t (an index in the XCD-contiguous, grouped order).
template <int BM, int BN, int WM, int WN, bool TA, bool TB, bool VEC>
__device__ __forceinline__ void gemm_z64_tile(const GemmZ64Params& g, int t, int zb, double* __restrict__ smem) {
  constexpr int BK = 16;
  constexpr int FM = BM / WM / 16;
  constexpr int FN = BN / WN / 16;
  static_assert(WM * WN == 4, "four waves");
  static_assert(FM >= 1 && FN >= 1, "tile too small");
  static_assert(BM >= 32 && BN >= 32, "tile sides must be >= 32");
  // A tile: !TA row-band [BM][BK+2]; TA k-band [BK][BM+16]
  constexpr int A_LD = TA ? (BM + 16) : (BK + 2);
  constexpr int A_SZ = TA ? BK * A_LD : BM * A_LD;
  // B tile: !TB k-band [BK][BN+16]; TB row-band [BN][BK+2]
  constexpr int B_LD = TB ? (BK + 2) : (BN + 16);
  constexpr int B_SZ = TB ? BN * B_LD : BK * B_LD;
  // pairs per thread per tile
  constexpr int A_P = BM * BK / 512;
  constexpr int B_P = BN * BK / 512;
  // smem: [stage][re A, im A, re B, im B]
  static_assert(2 * 2 * (A_SZ + B_SZ) == zgemm_lds_doubles(BM, BN, BK, TA, TB), "LDS size");

  // tile indices run through groups of eight tile-rows column by column
  const int gsz = 8 * g.tilesN;
  const int grp = t / gsz;
  const int gh = min(8, g.tilesM - grp * 8);
  const int wt = t - grp * gsz;
  const int bm0 = (grp * 8 + wt % gh) * BM;
  const int bn0 = (wt / gh) * BN;
  if (g.lowerOnly && bn0 > bm0 + BM - 1) return;

  const long long z = zb;
  const double* __restrict__ Ar = g.A.re + z * g.sA;
  const double* __restrict__ Ai = g.A.im + z * g.sA;
  const double* __restrict__ Br = g.B.re + z * g.sB;
  const double* __restrict__ Bi = g.B.im + z * g.sB;
  double* __restrict__ Cre = g.C.re + z * g.sC;
  double* __restrict__ Cim = g.C.im + z * g.sC;
  const int* __restrict__ rA = g.A.rows ? g.A.rows + z * g.rsA : nullptr;
  const int* __restrict__ rB = g.B.rows ? g.B.rows + z * g.rsB : nullptr;
  const int* __restrict__ rC = g.C.rows ? g.C.rows + z * g.rsC : nullptr;
  const int M = g.M, N = g.N;

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

  // ---- per-thread load coordinates (fixed across k-steps) ----
  // row-band: 8 pairs per 16-wide row, 32 rows per pass; k-band: C/2 pairs per row
  long long aRow[TA ? 1 : A_P];  // !TA: row offsets of A (rows fixed across k)
  int aRowOk[TA ? 1 : A_P];
  long long bRow[TB ? B_P : 1];  // TB: row offsets of B
  int bRowOk[TB ? B_P : 1];
  if (!TA) {
#pragma unroll
    for (int p = 0; p < A_P; ++p) {
      const int gi = bm0 + tid / 8 + 32 * p;
      aRowOk[p] = gi < M;
      const int pr = gi < M ? (rA ? rA[gi] : gi) : 0;
      aRow[p] = (long long)pr * g.A.ld;
    }
  }
  if (TB) {
#pragma unroll
    for (int p = 0; p < B_P; ++p) {
      const int gj = bn0 + tid / 8 + 32 * p;
      bRowOk[p] = gj < N;
      const int pr = gj < N ? (rB ? rB[gj] : gj) : 0;
      bRow[p] = (long long)pr * g.B.ld;
    }
  }

  double ra[A_P][2], rb[B_P][2], ia[A_P][2], ib[B_P][2];

  // Raw tile loads at clamped in-range addresses, issued unconditionally;
  // nothing reads their registers until the tile is written to LDS after the
  // current tile's products, where values outside the operand or its
  // triangle are zeroed.  Row indices of k-band operands are fetched one
  // k-step ahead (from a readable stand-in when there is no index array).
  auto ld_pair = [&](const double* row, int c, int lim, double& x, double& y) {
    if (VEC) {
      const double2 t2 = *reinterpret_cast<const double2*>(row + min(c, (lim - 1) & ~1));
      x = t2.x;
      y = t2.y;
    } else {
      x = row[min(c, lim - 1)];
      y = row[min(c + 1, lim - 1)];
    }
  };
  constexpr int KA = TA ? A_P : 1, KB = TB ? 1 : B_P;
  const int* rAs = rA ? rA : reinterpret_cast<const int*>(Ar);
  const int* rBs = rB ? rB : reinterpret_cast<const int*>(Br);
  int ixa[KA], ixb[KB];
  auto load_index = [&](int kt) {
    if (TA) {
      constexpr int TPR = BM / 2, RPP = 256 / TPR;
#pragma unroll
      for (int p = 0; p < KA; ++p) ixa[p] = rAs[min(kt + tid / TPR + RPP * p, kend - 1)];
    }
    if (!TB) {
      constexpr int TPR = BN / 2, RPP = 256 / TPR;
#pragma unroll
      for (int p = 0; p < KB; ++p) ixb[p] = rBs[min(kt + tid / TPR + RPP * p, kend - 1)];
    }
  };
  auto load_tiles = [&](int kt) {
    if (!TA) {
      const int gk = kt + (tid & 7) * 2;
#pragma unroll
      for (int p = 0; p < A_P; ++p) {
        ld_pair(Ar + aRow[p], gk, kend, ra[p][0], ra[p][1]);
        ld_pair(Ai + aRow[p], gk, kend, ia[p][0], ia[p][1]);
      }
    } else {
      constexpr int TPR = BM / 2, RPP = 256 / TPR;
      const int gi = bm0 + (tid % TPR) * 2;
#pragma unroll
      for (int p = 0; p < A_P; ++p) {
        const int gk = min(kt + tid / TPR + RPP * p, kend - 1);
        const long long ro = (long long)(rA ? ixa[p] : gk) * g.A.ld;
        ld_pair(Ar + ro, gi, M, ra[p][0], ra[p][1]);
        ld_pair(Ai + ro, gi, M, ia[p][0], ia[p][1]);
      }
    }
    if (!TB) {
      constexpr int TPR = BN / 2, RPP = 256 / TPR;
      const int gj = bn0 + (tid % TPR) * 2;
#pragma unroll
      for (int p = 0; p < B_P; ++p) {
        const int gk = min(kt + tid / TPR + RPP * p, kend - 1);
        const long long ro = (long long)(rB ? ixb[p] : gk) * g.B.ld;
        ld_pair(Br + ro, gj, N, rb[p][0], rb[p][1]);
        ld_pair(Bi + ro, gj, N, ib[p][0], ib[p][1]);
      }
    } else {
      const int gk = kt + (tid & 7) * 2;
#pragma unroll
      for (int p = 0; p < B_P; ++p) {
        ld_pair(Br + bRow[p], gk, kend, rb[p][0], rb[p][1]);
        ld_pair(Bi + bRow[p], gk, kend, ib[p][0], ib[p][1]);
      }
    }
  };

  auto store_tiles = [&](int stage, int kt) {
    double* As = smem + stage * 2 * (A_SZ + B_SZ);
    double* AsI = As + A_SZ;
    double* Bs = AsI + A_SZ;
    double* BsI = Bs + B_SZ;
#pragma unroll
    for (int p = 0; p < A_P; ++p) {
      int off, gi, gk, di, dk;
      bool ok;
      if (!TA) {
        gi = bm0 + tid / 8 + 32 * p;
        gk = kt + (tid & 7) * 2;
        di = 0; dk = 1;
        ok = aRowOk[p];
        off = (tid / 8 + 32 * p) * A_LD + (tid & 7) * 2;
      } else {
        constexpr int TPR = BM / 2, RPP = 256 / TPR;
        gi = bm0 + (tid % TPR) * 2;
        gk = kt + tid / TPR + RPP * p;
        di = 1; dk = 0;
        ok = true;
        off = (tid / TPR + RPP * p) * A_LD + (tid % TPR) * 2;
      }
      const bool ok0 = ok && gi < M && gk < kend, ok1 = ok && gi + di < M && gk + dk < kend;
      double xr = ok0 ? ra[p][0] : 0.0, xi = ok0 ? ia[p][0] : 0.0;
      double yr = ok1 ? ra[p][1] : 0.0, yi = ok1 ? ia[p][1] : 0.0;
      if (g.triA) {
        ztri_mask(xr, xi, g.triA, gi, gk);
        ztri_mask(yr, yi, g.triA, gi + di, gk + dk);
      }
      *reinterpret_cast<double2*>(As + off) = double2{xr, yr};
      *reinterpret_cast<double2*>(AsI + off) = double2{xi, yi};
    }
#pragma unroll
    for (int p = 0; p < B_P; ++p) {
      int off, gj, gk, dj, dk;
      bool ok;
      if (TB) {
        gj = bn0 + tid / 8 + 32 * p;
        gk = kt + (tid & 7) * 2;
        dj = 0; dk = 1;
        ok = bRowOk[p];
        off = (tid / 8 + 32 * p) * B_LD + (tid & 7) * 2;
      } else {
        constexpr int TPR = BN / 2, RPP = 256 / TPR;
        gj = bn0 + (tid % TPR) * 2;
        gk = kt + tid / TPR + RPP * p;
        dj = 1; dk = 0;
        ok = true;
        off = (tid / TPR + RPP * p) * B_LD + (tid % TPR) * 2;
      }
      const bool ok0 = ok && gj < N && gk < kend, ok1 = ok && gj + dj < N && gk + dk < kend;
      double xr = ok0 ? rb[p][0] : 0.0, xi = ok0 ? ib[p][0] : 0.0;
      double yr = ok1 ? rb[p][1] : 0.0, yi = ok1 ? ib[p][1] : 0.0;
      if (g.triB) {
        ztri_mask(xr, xi, g.triB, gk, gj);
        ztri_mask(yr, yi, g.triB, gk + dk, gj + dj);
      }
      *reinterpret_cast<double2*>(Bs + off) = double2{xr, yr};
      *reinterpret_cast<double2*>(BsI + off) = double2{xi, yi};
    }
  };

  d4 acc[FM][FN], acci[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) { acc[a][b] = d4{0.0, 0.0, 0.0, 0.0}; acci[a][b] = d4{0.0, 0.0, 0.0, 0.0}; }
  const double sA = g.conjA ? -1.0 : 1.0, sB = g.conjB ? -1.0 : 1.0;

  if (nk > 0) {
    load_index(kbeg);
    load_tiles(kbeg);
    if (nk > 1) load_index(kbeg + BK);
    store_tiles(0, kbeg);
    __syncthreads();
  }
  for (int it = 0; it < nk; ++it) {
    const int stage = it & 1;
    if (it + 1 < nk) {
      load_tiles(kbeg + (it + 1) * BK);
      if (it + 2 < nk) load_index(kbeg + (it + 2) * BK);
    }
    const double* As = smem + stage * 2 * (A_SZ + B_SZ);
    const double* AsI = As + A_SZ;
    const double* Bs = AsI + A_SZ;
    const double* BsI = Bs + B_SZ;
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int k = kk * 4 + (lane >> 4);
      double af[FM], afi[FM], afn[FM], bf[FN], bfi[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) {
        const int i = wm0 + a * 16 + (lane & 15);
        af[a] = TA ? As[k * A_LD + i] : As[i * A_LD + k];
        afi[a] = sA * (TA ? AsI[k * A_LD + i] : AsI[i * A_LD + k]);
        afn[a] = -afi[a];
      }
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int j = wn0 + b * 16 + (lane & 15);
        bf[b] = TB ? Bs[j * B_LD + k] : Bs[k * B_LD + j];
        bfi[b] = sB * (TB ? BsI[j * B_LD + k] : BsI[k * B_LD + j]);
      }
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(afn[a], bfi[b], acc[a][b], 0, 0, 0);
          acci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bfi[b], acci[a][b], 0, 0, 0);
          acci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(afi[a], bf[b], acci[a][b], 0, 0, 0);
        }
    }
    if (it + 1 < nk) store_tiles(stage ^ 1, kbeg + (it + 1) * BK);
    __syncthreads();
  }

  // epilogue: lane holds D[l/16 + 4v][l%16] of each 16x16 tile; C is read
  // (beta != 0) per 16-row tile in one unconditional batch at clamped
  // addresses so the reads overlap
  int pc[FN];
#pragma unroll
  for (int b = 0; b < FN; ++b) {
    const int jc = min(bn0 + wn0 + b * 16 + (lane & 15), N - 1);
    pc[b] = g.C.cols ? g.C.cols[jc] : jc;
  }
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    long long ro[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ic = min(bm0 + wm0 + a * 16 + (lane >> 4) + 4 * v, M - 1);
      ro[v] = (long long)(rC ? rC[ic] : ic) * g.C.ld;
    }
    double cr[4][FN], ci[4][FN];
    if (g.beta != 0.0) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
          cr[v][b] = Cre[ro[v] + pc[b]];
          ci[v][b] = Cim[ro[v] + pc[b]];
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = bm0 + wm0 + a * 16 + (lane >> 4) + 4 * v;
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int j = bn0 + wn0 + b * 16 + (lane & 15);
        if (i < M && j < N && (!g.lowerOnly || i >= j)) {
          double vr = g.alpha * acc[a][b][v], vi = g.alpha * acci[a][b][v];
          if (g.beta != 0.0) { vr += g.beta * cr[v][b]; vi += g.beta * ci[v][b]; }
          Cre[ro[v] + pc[b]] = vr;
          Cim[ro[v] + pc[b]] = vi;
        }
      }
    }
  }
}

// Block b works on XCD b % 8 in that XCD's contiguous range of tile indices,
// one tile per block (with g.flat > 0, of (batch entry, tile) items, so that
// a batch of small products fills every XCD); PERSIST: a capped grid
// (GridCapScope, as in the real GEMM) whose blocks take several tiles.
template <int BM, int BN, int WM, int WN, bool TA, bool TB, bool VEC, bool PERSIST>
__global__ __launch_bounds__(256, 2) void k_gemm_z64(GemmZ64Params g) {
  __shared__ __attribute__((aligned(16))) double smem[zgemm_lds_doubles(BM, BN, 16, TA, TB)];
  const int tiles = g.tilesM * g.tilesN;
  const int per = (tiles + 7) / 8;
  const int bid = blockIdx.x;
  if (!PERSIST) {
    if (g.flat > 0) {
      const int items = tiles * g.flat;
      const int pi = (items + 7) / 8;
      const int wi = (bid & 7) * pi + (bid >> 3);
      if (wi >= items) return;
      gemm_z64_tile<BM, BN, WM, WN, TA, TB, VEC>(g, wi % tiles, wi / tiles, smem);
      return;
    }
    const int t = (bid & 7) * per + (bid >> 3);
    if (t >= tiles) return;
    gemm_z64_tile<BM, BN, WM, WN, TA, TB, VEC>(g, t, blockIdx.z, smem);
  } else {
    const int step = gridDim.x >> 3;
    for (int li = bid >> 3; li < per; li += step) {
      const int t = (bid & 7) * per + li;
      if (t >= tiles) break;
      gemm_z64_tile<BM, BN, WM, WN, TA, TB, VEC>(g, t, blockIdx.z, smem);
      // the tile's last k-step ended with a barrier; the epilogue reads no LDS
    }
  }
}

template <int BM, int BN, int WM, int WN, bool TA, bool TB>
static void launch_cfg_z(const GemmZ64Params& p0, int batch, hipStream_t s) {
  GemmZ64Params p = p0;
  p.tilesM = ceil_div(p.M, BM);
  p.tilesN = ceil_div(p.N, BN);
  p.flat = 0;
  const int tiles = p.tilesM * p.tilesN;
  const int grid = 8 * ((tiles + 7) / 8);
  const bool vec = p.vecA && p.vecB;
  if constexpr (!TA && !TB) {
    const int cap = grid_cap() > 0 ? std::max(8, grid_cap() & ~7) : 0;
    if (cap > 0 && cap < grid) {
      if (vec)
        hipLaunchKernelGGL((k_gemm_z64<BM, BN, WM, WN, TA, TB, true, true>), dim3(cap, 1, batch), dim3(256), 0, s, p);
      else
        hipLaunchKernelGGL((k_gemm_z64<BM, BN, WM, WN, TA, TB, false, true>), dim3(cap, 1, batch), dim3(256), 0, s,
                           p);
      FROB_LAUNCH_CHECK();
      return;
    }
  }
  // a batch of more than one entry (not lower-only) is folded into blockIdx.x
  if (batch > 1 && !p.lowerOnly) p.flat = batch;
  const dim3 gd = p.flat > 0 ? dim3(8 * ((tiles * batch + 7) / 8), 1, 1) : dim3(grid, 1, batch);
  if (vec)
    hipLaunchKernelGGL((k_gemm_z64<BM, BN, WM, WN, TA, TB, true, false>), gd, dim3(256), 0, s, p);
  else
    hipLaunchKernelGGL((k_gemm_z64<BM, BN, WM, WN, TA, TB, false, false>), gd, dim3(256), 0, s, p);
  FROB_LAUNCH_CHECK();
}

enum { ZCFG_64x64 = 0, ZCFG_128x32 = 1, ZCFG_32x128 = 2, ZCFG_128x64 = 3 };

template <bool TA, bool TB>
static void launch_pick_z(const GemmZ64Params& p, int batch, int cfg, hipStream_t s) {
  switch (cfg) {
    case ZCFG_64x64: launch_cfg_z<64, 64, 2, 2, TA, TB>(p, batch, s); break;
    case ZCFG_128x32: launch_cfg_z<128, 32, 4, 1, TA, TB>(p, batch, s); break;
    case ZCFG_32x128: launch_cfg_z<32, 128, 1, 4, TA, TB>(p, batch, s); break;
    default: throw std::runtime_error("gemm_z64: bad tile config");
  }
}

static int zpick(int M, int N, int need) {
  if (need == GEMM_NEED_FULL_M) {
    if (M > 128) throw std::runtime_error("gemm_z64: in-place product taller than 128");
    return M <= 64 ? ZCFG_64x64 : ZCFG_128x32;
  }
  if (need == GEMM_NEED_FULL_N) {
    if (N > 128) throw std::runtime_error("gemm_z64: in-place product wider than 128");
    return N <= 64 ? ZCFG_64x64 : ZCFG_32x128;
  }
  if (N <= 32) return ZCFG_128x32;
  if (M <= 32) return ZCFG_32x128;
  return ZCFG_64x64;
}

static bool zaligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

void gemm_z64_batched(hipStream_t s, int opA, int opB, int M, int N, int K, double alpha, ZOp A, int triA, ZOp B,
                      int triB, double beta, ZOut C, bool lowerOnly, int batch, long long sA, long long sB,
                      long long sC, int rsA, int rsB, int rsC, int need) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0 && beta == 1.0) return;
  GemmZ64Params p;
  p.M = M; p.N = N; p.K = K < 0 ? 0 : K;
  p.alpha = alpha; p.beta = beta;
  p.A = A; p.B = B; p.C = C;
  p.conjA = opA == OP_C; p.conjB = opB == OP_C;
  p.triA = triA; p.triB = triB;
  p.lowerOnly = lowerOnly ? 1 : 0;
  const bool ta = opA != OP_N, tb = opB != OP_N;
  // 16-byte loads: aligned rows and an even extent along the rows
  p.vecA = zaligned16(A.re) && zaligned16(A.im) && (A.ld % 2 == 0) && (sA % 2 == 0) && ((ta ? M : K) % 2 == 0);
  p.vecB = zaligned16(B.re) && zaligned16(B.im) && (B.ld % 2 == 0) && (sB % 2 == 0) && ((tb ? K : N) % 2 == 0);
  p.sA = sA; p.sB = sB; p.sC = sC;
  p.rsA = rsA; p.rsB = rsB; p.rsC = rsC;
  const int cfg = zpick(M, N, need);
  if (!ta && !tb) launch_pick_z<false, false>(p, batch, cfg, s);
  else if (!ta && tb) launch_pick_z<false, true>(p, batch, cfg, s);
  else if (ta && !tb) launch_pick_z<true, false>(p, batch, cfg, s);
  else launch_pick_z<true, true>(p, batch, cfg, s);
}

void gemm_z64(hipStream_t s, int opA, int opB, int M, int N, int K, double alpha, ZOp A, int triA, ZOp B, int triB,
              double beta, ZOut C, bool lowerOnly, int need) {
  gemm_z64_batched(s, opA, opB, M, N, K, alpha, A, triA, B, triB, beta, C, lowerOnly, 1, 0, 0, 0, 0, 0, 0, need);
}

}  // namespace frob
