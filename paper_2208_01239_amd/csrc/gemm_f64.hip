// gemm_f64.hip -- FP64 matrix-core GEMM for gfx950.
//
//   C = alpha * op(A) * op(B) + beta * C       (row-major, op = N or T)
//
// with optional row indirection on A, B and C, an optional column scatter on
// C, triangular interpretation of op(A)/op(B) (entries outside the triangle
// read as zero and the k range is clipped to the triangle, a unit diagonal
// reads as one), a lower-triangle-only output mode, and a batch index
// (folded into blockIdx.x with the tile index; on blockIdx.z for
// lower-triangle-only and capped launches).  This one kernel serves the trailing updates of the
// factorizations (row-indirect NN), the triangular solves and inverses
// (trmm-like products), the symmetric rank-k updates (lower-only), and the
// plain products B*Y and -Y*C^{-1}.
//
// Tiling: 256 threads = 4 wave64s, block tile BM x BN, k-step 16 (128 x 128)
// or 32 (smaller tiles).  Each wave
// owns a (BM/WM) x (BN/WN) sub-tile built from 16x16 v_mfma_f64_16x16x4f64
// tiles.  Operand tiles are staged through a double-buffered LDS ring in the
// same orientation as in HBM (the fragment read indexing applies op), so a
// k-step costs one workgroup barrier; the next tile's global loads (16-byte
// when the operand is 16-byte aligned with an even leading dimension) are in
// flight while the current tile is multiplied.  Padding keeps the 16-lane
// fragment reads on distinct banks.  Linear block ids are remapped so that
// each of the 8 XCDs (hardware assigns block b to XCD b % 8) works on a
// contiguous range of tile indices, and tile indices run through groups of
// eight tile-rows column by column, so the tiles one XCD runs at the same
// time form a square block whose A rows and B columns stay in its L2.
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
  int vecA, vecB;
  long long sA, sB, sC;      // batch strides of the data pointers
  int rsA, rsB, rsC;         // batch strides of the row-index pointers
  int tilesM, tilesN;
  int flat;                  // > 0: that many batch entries folded into blockIdx.x (else batch on blockIdx.z)
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

constexpr int TILE_GROUP = 8;

// LDS of the double-buffered operand tiles; two workgroups per CU when they fit
constexpr int gemm_lds_bytes(int BM, int BN, int BK, bool TA, bool TB) {
  return 2 * 8 * ((TA ? BK * (BM + 16) : BM * (BK + 2)) + (TB ? BN * (BK + 2) : BK * (BN + 16)));
}
constexpr int gemm_min_blocks(int BM, int BN, int BK, bool TA, bool TB) {
  return 2 * gemm_lds_bytes(BM, BN, BK, TA, TB) <= 160 * 1024 ? 2 : 1;
}

// One output tile t (an index in the XCD-contiguous, grouped order) of the
// product; smem holds gemm_lds_bytes(BM, BN, BK, TA, TB) bytes.  PLAIN: no
// triangular operand, no output indirection and no row indices on a k-band
// operand (known at compile time, so the k-loop carries none of their masking
// and index loads); row indices of a row-band operand (A untransposed, B
// transposed) are looked up once per tile and stay allowed.
template <int BM, int BN, int WM, int WN, bool TA, bool TB, bool VEC, int BK, bool PLAIN = false>
__device__ __forceinline__ void gemm_f64_tile(const GemmF64Params& g, int t, int zb, double* __restrict__ smem) {
  constexpr int KP = BK / 2;       // 16-byte pairs per row of a row-band tile
  constexpr int RP = 256 / KP;     // rows of a row-band tile per pass
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
  static_assert(BK == 16 || BK == 32, "k-step");
  static_assert(2 * (A_SZ + B_SZ) * 8 == gemm_lds_bytes(BM, BN, BK, TA, TB), "LDS size");

  // grouped order: TILE_GROUP tile-rows at a time, column-major inside the
  // group, so that the tiles an XCD runs at once form a square block
  const int gsz = TILE_GROUP * g.tilesN;
  const int grp = t / gsz;
  const int gh = min(TILE_GROUP, g.tilesM - grp * TILE_GROUP);
  const int wt = t - grp * gsz;
  const int bm0 = (grp * TILE_GROUP + wt % gh) * BM;
  const int bn0 = (wt / gh) * BN;
  if (g.lowerOnly && bn0 > bm0 + BM - 1) return;

  const long long z = zb;
  const double* __restrict__ Ap = g.A.p + z * g.sA;
  const double* __restrict__ Bp = g.B.p + z * g.sB;
  double* __restrict__ Cp = g.C.p + z * g.sC;
  const int* __restrict__ rA = (!PLAIN || !TA) && g.A.rows ? g.A.rows + z * g.rsA : nullptr;
  const int* __restrict__ rB = (!PLAIN || TB) && g.B.rows ? g.B.rows + z * g.rsB : nullptr;
  const int* __restrict__ rC = !PLAIN && g.C.rows ? g.C.rows + z * g.rsC : nullptr;
  const int triA = PLAIN ? TRI_NONE : g.triA, triB = PLAIN ? TRI_NONE : g.triB;
  const int M = g.M, N = g.N;

  int kbeg = 0, kend = g.K;
  if (triA == TRI_UPPER || triA == TRI_UPPER_UNIT) kbeg = max(kbeg, bm0);
  if (triA == TRI_LOWER || triA == TRI_LOWER_UNIT) kend = min(kend, bm0 + BM);
  if (triB == TRI_LOWER || triB == TRI_LOWER_UNIT) kbeg = max(kbeg, bn0);
  if (triB == TRI_UPPER || triB == TRI_UPPER_UNIT) kend = min(kend, bn0 + BN);
  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wm0 = (w / WN) * (BM / WM);
  const int wn0 = (w % WN) * (BN / WN);

  // ---- per-thread load coordinates (fixed across k-steps) ----
  // row-band: 8 pairs per 16-wide row, 32 rows per pass; k-band: C/2 pairs per row
  const double* aRow[TA ? 1 : A_P];  // !TA: row pointers of A (rows fixed across k)
  int aRowOk[TA ? 1 : A_P];
  const double* bRow[TB ? B_P : 1];  // TB: row pointers of B
  int bRowOk[TB ? B_P : 1];
  if (!TA) {
#pragma unroll
    for (int p = 0; p < A_P; ++p) {
      const int gi = bm0 + tid / KP + RP * p;
      aRowOk[p] = gi < M;
      const int pr = gi < M ? (rA ? rA[gi] : gi) : 0;
      aRow[p] = Ap + (long long)pr * g.A.ld;
    }
  }
  if (TB) {
#pragma unroll
    for (int p = 0; p < B_P; ++p) {
      const int gj = bn0 + tid / KP + RP * p;
      bRowOk[p] = gj < N;
      const int pr = gj < N ? (rB ? rB[gj] : gj) : 0;
      bRow[p] = Bp + (long long)pr * g.B.ld;
    }
  }

  double ra[A_P][2], rb[B_P][2];

  // Raw tile loads: every address is clamped into the operand, so the loads
  // are issued unconditionally and nothing consumes their registers until the
  // tile is written to LDS (after the current tile's products).  Elements
  // outside the operand (ragged edges, the k tail) and outside a triangle are
  // zeroed at that point.  With VEC (16-byte aligned rows, even row extents)
  // pairs are read with one 16-byte load and never straddle the extent.
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
  // k-band operands (TA for A, !TB for B) address their rows through a row
  // index that changes with k: the indices of a tile are fetched one k-step
  // before its data, unconditionally (from a readable stand-in when there is
  // no index array; the value is then ignored), so no wait on them stalls
  // the products in between.
  constexpr int KA = TA ? A_P : 1, KB = TB ? 1 : B_P;
  const int* rAs = rA ? rA : reinterpret_cast<const int*>(Ap);
  const int* rBs = rB ? rB : reinterpret_cast<const int*>(Bp);
  int ixa[KA], ixb[KB];
  auto load_index = [&](int kt) {
    if constexpr (PLAIN) return;
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
      const int gk = kt + (tid % KP) * 2;
#pragma unroll
      for (int p = 0; p < A_P; ++p) ld_pair(aRow[p], gk, kend, ra[p][0], ra[p][1]);
    } else {
      constexpr int TPR = BM / 2, RPP = 256 / TPR;
      const int gi = bm0 + (tid % TPR) * 2;
#pragma unroll
      for (int p = 0; p < A_P; ++p) {
        const int gk = min(kt + tid / TPR + RPP * p, kend - 1);
        ld_pair(Ap + (long long)(rA ? ixa[p] : gk) * g.A.ld, gi, M, ra[p][0], ra[p][1]);
      }
    }
    if (!TB) {
      constexpr int TPR = BN / 2, RPP = 256 / TPR;
      const int gj = bn0 + (tid % TPR) * 2;
#pragma unroll
      for (int p = 0; p < B_P; ++p) {
        const int gk = min(kt + tid / TPR + RPP * p, kend - 1);
        ld_pair(Bp + (long long)(rB ? ixb[p] : gk) * g.B.ld, gj, N, rb[p][0], rb[p][1]);
      }
    } else {
      const int gk = kt + (tid % KP) * 2;
#pragma unroll
      for (int p = 0; p < B_P; ++p) ld_pair(bRow[p], gk, kend, rb[p][0], rb[p][1]);
    }
  };

  // mask and write the loaded tile of k-step kt into LDS stage `stage`
  auto store_tiles = [&](int stage, int kt) {
    double* As = smem + stage * (A_SZ + B_SZ);
    double* Bs = As + A_SZ;
#pragma unroll
    for (int p = 0; p < A_P; ++p) {
      int off, gi, gk, di, dk;
      bool ok;
      if (!TA) {
        gi = bm0 + tid / KP + RP * p;
        gk = kt + (tid % KP) * 2;
        di = 0; dk = 1;
        ok = aRowOk[p];
        off = (tid / KP + RP * p) * A_LD + (tid % KP) * 2;
      } else {
        constexpr int TPR = BM / 2, RPP = 256 / TPR;
        gi = bm0 + (tid % TPR) * 2;
        gk = kt + tid / TPR + RPP * p;
        di = 1; dk = 0;
        ok = true;
        off = (tid / TPR + RPP * p) * A_LD + (tid % TPR) * 2;
      }
      double x = (ok && gi < M && gk < kend) ? ra[p][0] : 0.0;
      double y = (ok && gi + di < M && gk + dk < kend) ? ra[p][1] : 0.0;
      if (triA) {
        x = tri_mask(x, triA, gi, gk);
        y = tri_mask(y, triA, gi + di, gk + dk);
      }
      *reinterpret_cast<double2*>(As + off) = double2{x, y};
    }
#pragma unroll
    for (int p = 0; p < B_P; ++p) {
      int off, gj, gk, dj, dk;
      bool ok;
      if (TB) {
        gj = bn0 + tid / KP + RP * p;
        gk = kt + (tid % KP) * 2;
        dj = 0; dk = 1;
        ok = bRowOk[p];
        off = (tid / KP + RP * p) * B_LD + (tid % KP) * 2;
      } else {
        constexpr int TPR = BN / 2, RPP = 256 / TPR;
        gj = bn0 + (tid % TPR) * 2;
        gk = kt + tid / TPR + RPP * p;
        dj = 1; dk = 0;
        ok = true;
        off = (tid / TPR + RPP * p) * B_LD + (tid % TPR) * 2;
      }
      double x = (ok && gj < N && gk < kend) ? rb[p][0] : 0.0;
      double y = (ok && gj + dj < N && gk + dk < kend) ? rb[p][1] : 0.0;
      if (triB) {
        x = tri_mask(x, triB, gk, gj);
        y = tri_mask(y, triB, gk + dk, gj + dj);
      }
      *reinterpret_cast<double2*>(Bs + off) = double2{x, y};
    }
  };

  d4 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

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
    const double* As = smem + stage * (A_SZ + B_SZ);
    const double* Bs = As + A_SZ;
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
    if (it + 1 < nk) store_tiles(stage ^ 1, kbeg + (it + 1) * BK);
    __syncthreads();
  }

  // epilogue: lane holds D[l/16 + 4v][l%16] of each 16x16 tile.  The reads
  // of C (beta != 0) are issued per 16-row tile as one unconditional batch
  // at clamped addresses, so they overlap instead of costing one memory
  // latency each.
  int pc[FN];
#pragma unroll
  for (int b = 0; b < FN; ++b) {
    const int jc = min(bn0 + wn0 + b * 16 + (lane & 15), N - 1);
    pc[b] = !PLAIN && g.C.cols ? g.C.cols[jc] : jc;
  }
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    double* crow[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ic = min(bm0 + wm0 + a * 16 + (lane >> 4) + 4 * v, M - 1);
      crow[v] = Cp + (long long)(rC ? rC[ic] : ic) * g.C.ld;
    }
    double cold[4][FN];
    if (g.beta != 0.0) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int b = 0; b < FN; ++b) cold[v][b] = crow[v][pc[b]];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = bm0 + wm0 + a * 16 + (lane >> 4) + 4 * v;
#pragma unroll
      for (int b = 0; b < FN; ++b) {
        const int j = bn0 + wn0 + b * 16 + (lane & 15);
        if (i < M && j < N && (!g.lowerOnly || i >= j)) {
          double val = g.alpha * acc[a][b][v];
          if (g.beta != 0.0) val += g.beta * cold[v][b];
          crow[v][pc[b]] = val;
        }
      }
    }
  }
}

// Block b works on XCD b % 8 (hardware round-robin), in that XCD's
// contiguous range of tile indices.  The usual grid gives every block one
// tile.  PERSIST: a capped grid (GridCapScope) whose blocks take several
// tiles, in steps of the number of blocks per XCD, and leave compute units
// free for concurrent work.
template <int BM, int BN, int WM, int WN, bool TA, bool TB, bool VEC, int BK, bool PERSIST, bool PLAIN = false>
__global__ __launch_bounds__(256, gemm_min_blocks(BM, BN, BK, TA, TB)) void k_gemm_f64(GemmF64Params g) {
  __shared__ __attribute__((aligned(16))) double smem[gemm_lds_bytes(BM, BN, BK, TA, TB) / 8];
  const int tiles = g.tilesM * g.tilesN;
  const int per = (tiles + 7) / 8;
  const int bid = blockIdx.x;
  // A lower-triangle-only product leaves the tiles above the diagonal idle.
  // Contiguous per-XCD ranges of the grouped order would then give the XCDs
  // of the first tile-rows almost nothing to do; interleaving hands XCD x
  // tile-row x of every group instead (all its columns, so its A rows stay
  // in its L2), and the live tiles spread evenly.
  if (!PERSIST) {
    if (g.flat > 0) {
      // a batch folded into blockIdx.x: XCD-contiguous ranges of (batch
      // entry, tile) items, so a batch of small products fills every XCD
      const int items = tiles * g.flat;
      const int pi = (items + 7) / 8;
      const int wi = (bid & 7) * pi + (bid >> 3);
      if (wi >= items) return;
      gemm_f64_tile<BM, BN, WM, WN, TA, TB, VEC, BK, PLAIN>(g, wi % tiles, wi / tiles, smem);
      return;
    }
    const int t = g.lowerOnly ? bid : (bid & 7) * per + (bid >> 3);
    if (t >= tiles) return;
    gemm_f64_tile<BM, BN, WM, WN, TA, TB, VEC, BK, PLAIN>(g, t, blockIdx.z, smem);
  } else {
    const int step = gridDim.x >> 3;
    for (int li = bid >> 3; li < per; li += step) {
      const int t = g.lowerOnly ? 8 * li + (bid & 7) : (bid & 7) * per + li;
      if (t >= tiles) break;
      gemm_f64_tile<BM, BN, WM, WN, TA, TB, VEC, BK, PLAIN>(g, t, blockIdx.z, smem);
      // a next tile reuses the LDS ring: the tile's last k-step ended with a
      // barrier after its last LDS read, and the epilogue reads no LDS
    }
  }
}

template <int BM, int BN, int WM, int WN, bool TA, bool TB>
static void launch_cfg(const GemmF64Params& p0, int batch, hipStream_t s) {
  GemmF64Params p = p0;
  p.tilesM = ceil_div(p.M, BM);
  p.tilesN = ceil_div(p.N, BN);
  p.flat = 0;
  const int tiles = p.tilesM * p.tilesN;
  const int grid = 8 * ((tiles + 7) / 8);
  // capped grids for the untransposed products (the factorizations' updates)
  const int cap = (!TA && !TB && grid_cap() > 0) ? std::max(8, grid_cap() & ~7) : 0;
  // the big tile keeps a 16-deep k-step (two workgroups per CU fit in LDS);
  // the smaller tiles, used for latency-bound products, take 32 (half as
  // many dependent k-steps)
  constexpr int BK = (BM * BN >= 128 * 128) ? 16 : 32;
  const bool vec = p.vecA && p.vecB;
  if constexpr (!TA && !TB) {
    if (cap > 0 && cap < grid) {
      if (vec)
        hipLaunchKernelGGL((k_gemm_f64<BM, BN, WM, WN, TA, TB, true, BK, true>), dim3(cap, 1, batch), dim3(256), 0, s,
                           p);
      else
        hipLaunchKernelGGL((k_gemm_f64<BM, BN, WM, WN, TA, TB, false, BK, true>), dim3(cap, 1, batch), dim3(256), 0,
                           s, p);
      FROB_LAUNCH_CHECK();
      return;
    }
  }
  // a batch of more than one entry (not lower-only) is folded into blockIdx.x
  if (batch > 1 && !p.lowerOnly) p.flat = batch;
  const dim3 gd = p.flat > 0 ? dim3(8 * ((tiles * batch + 7) / 8), 1, 1) : dim3(grid, 1, batch);
  const bool plain =
      !p.triA && !p.triB && !p.C.rows && !p.C.cols && (TA ? !p.A.rows : true) && (TB ? true : !p.B.rows);
  if constexpr (BM == 128 && BN == 128) {
    if (vec && plain) {
      hipLaunchKernelGGL((k_gemm_f64<BM, BN, WM, WN, TA, TB, true, BK, false, true>), gd, dim3(256), 0, s, p);
      FROB_LAUNCH_CHECK();
      return;
    }
  }
  if (vec)
    hipLaunchKernelGGL((k_gemm_f64<BM, BN, WM, WN, TA, TB, true, BK, false>), gd, dim3(256), 0, s, p);
  else
    hipLaunchKernelGGL((k_gemm_f64<BM, BN, WM, WN, TA, TB, false, BK, false>), gd, dim3(256), 0, s, p);
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
  if (need == GEMM_NEED_FULL_M) {
    if (M > 128) throw std::runtime_error("gemm_f64: in-place product taller than 128");
    return M <= 64 ? GEMM_CFG_64x64 : GEMM_CFG_128x32;
  }
  if (need == GEMM_NEED_FULL_N) {
    if (N > 128) throw std::runtime_error("gemm_f64: in-place product wider than 128");
    return N <= 64 ? GEMM_CFG_64x64 : GEMM_CFG_32x128;
  }
  if (N <= 32) return GEMM_CFG_128x32;
  if (M <= 32) return GEMM_CFG_32x128;
  const long long big_tiles = (long long)ceil_div(M, 128) * ceil_div(N, 128);
  if (big_tiles >= 160) return GEMM_CFG_128x128;
  return GEMM_CFG_64x64;
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

namespace {
thread_local int t_lp_mode = LP_NONE;
thread_local int t_grid_cap = 0;
}
int lp_mode() { return t_lp_mode; }
LowPrecScope::LowPrecScope(int mode) : prev(t_lp_mode) { t_lp_mode = mode; }
LowPrecScope::~LowPrecScope() { t_lp_mode = prev; }
int grid_cap() { return t_grid_cap; }
GridCapScope::GridCapScope(int blocks) : prev(t_grid_cap) { t_grid_cap = blocks; }
GridCapScope::~GridCapScope() { t_grid_cap = prev; }

void gemm_f64_batched(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, DOp A, int triA, DOp B,
                      int triB, double beta, DOut C, bool lowerOnly, int batch, long long sA, long long sB,
                      long long sC, int rsA, int rsB, int rsC, int need) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0 && beta == 1.0) return;
  if (t_lp_mode != LP_NONE && triA == TRI_NONE && triB == TRI_NONE && need == GEMM_NEED_ANY && !C.cols &&
      K >= 32 && (batch == 1 || (rsA == 0 && rsB == 0 && rsC == 0))) {
    gemm_lp(s, t_lp_mode, ta, tb, M, N, K, alpha, A.p, A.ld, A.rows, B.p, B.ld, B.rows, beta, C.p, C.ld, C.rows,
            lowerOnly, batch, sA, sB, sC);
    return;
  }
  GemmF64Params p;
  p.M = M; p.N = N; p.K = K < 0 ? 0 : K;
  p.alpha = alpha; p.beta = beta;
  p.A = A; p.B = B; p.C = C;
  p.triA = triA; p.triB = triB;
  p.lowerOnly = lowerOnly ? 1 : 0;
  // 16-byte loads need 16-byte aligned rows in every batch entry and an even
  // extent along the rows (the pairs then never cross it)
  p.vecA = aligned16(A.p) && (A.ld % 2 == 0) && (sA % 2 == 0) && ((ta ? M : K) % 2 == 0);
  p.vecB = aligned16(B.p) && (B.ld % 2 == 0) && (sB % 2 == 0) && ((tb ? K : N) % 2 == 0);
  p.sA = sA; p.sB = sB; p.sC = sC;
  p.rsA = rsA; p.rsB = rsB; p.rsC = rsC;
  int cfg = gemm_pick_cfg(M, N, need);
  // a large batch of small products takes the big tile (its k-loop runs at
  // the better matrix-core rate) once the batch gives it 1024 tiles
  if (batch > 1 && !lowerOnly && need == GEMM_NEED_ANY && cfg == GEMM_CFG_64x64 && M >= 128 && N >= 128 &&
      (long long)ceil_div(M, 128) * ceil_div(N, 128) * batch >= 1024)
    cfg = GEMM_CFG_128x128;
  if (!ta && !tb) launch_pick<false, false>(p, batch, cfg, s);
  else if (!ta && tb) launch_pick<false, true>(p, batch, cfg, s);
  else if (ta && !tb) launch_pick<true, false>(p, batch, cfg, s);
  else launch_pick<true, true>(p, batch, cfg, s);
}

void gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, DOp A, int triA, DOp B,
              int triB, double beta, DOut C, bool lowerOnly, int batch, long long sA, long long sB,
              long long sC, int need) {
  gemm_f64_batched(s, ta, tb, M, N, K, alpha, A, triA, B, triB, beta, C, lowerOnly, batch, sA, sB, sC, 0, 0, 0,
                   need);
}

}  // namespace frob
