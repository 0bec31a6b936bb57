// batched.hip -- many Frobenius inversions of uneven order in one persistent
// launch (the batching line of growth).
//
// One workgroup (256 threads) inverts one matrix at a time, start to finish:
// it takes the next matrix index from an atomic queue whose order (largest
// order first, the longest-processing-time rule) is prepared on the device,
// and runs Algorithm 5 (general) or Algorithm 7 (Hermitian positive definite)
// with blocked in-workgroup building blocks:
//   - GEMM: 64x64 output tiles, k-step 32, operands staged in LDS, 16x16x4
//     matrix-core products (FP64, or FP32 with FP32 accumulation), next
//     k-step's global loads in flight during the current products;
//   - LU with partial pivoting: right-looking, panels of NB columns factored in
//     LDS (pivot search by wave reductions plus an LDS reduction), physical row
//     interchanges, triangular solve of the block row, GEMM trailing update;
//   - Cholesky: NB x NB diagonal blocks in LDS, row-wise substitution for the
//     block column, GEMM trailing update;
//   - triangular solves: NB x NB diagonal blocks by substitution (one thread
//     per right-hand side), GEMM updates in between.
// The matrices stay in global memory (L2-resident at these orders); each
// workgroup owns a private slot of workspace (three n_max x n_max matrices and
// the pivot indices).  Panel width NB per size class comes from the caller's
// table (autotuned by frob_batched_tune).
#include <climits>

#include "common.hpp"
#include "handle.hpp"
#include "internal.hpp"

namespace frob {

namespace {

constexpr int BT = 256;          // threads per workgroup
constexpr int BNMAX = 512;       // largest order handled in-workgroup
constexpr int PNB = 32;          // largest LU panel width
constexpr int XNB = 16;          // diagonal blocks solved by register substitution (triangular solves, Cholesky)
constexpr int GT = 64;           // GEMM output tile
constexpr int GP = GT + 4;       // LDS pitch of a GEMM tile row
// GEMM k-step: 32 in FP32, 16 in FP64 (keeps the FP64 panel plus tiles under 160 KiB of LDS)
template <typename T>
struct GKof { static constexpr int v = sizeof(T) == 8 ? 16 : 32; };

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef d4 acc;
  __device__ static acc op(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef f4 acc;
  __device__ static acc op(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <typename T>
struct Smem {
  T ga[GKof<T>::v * GP];     // GEMM A tile, k-major
  T gb[GKof<T>::v * GP];     // GEMM B tile, k-major
  T panel[BNMAX * PNB];      // LU panel / Cholesky diagonal block / triangular diagonal block
  T red_v[BT / 64];
  int red_i[BT / 64];
  int bcast[4];
};

// Scalar arguments of the non-inlined building blocks arrive in vector
// registers; re-reading them through readfirstlane makes every loop bound and
// branch condition derived from them uniform to the compiler (they are
// uniform in value), so barrier-containing regions are never entered with a
// partial or empty exec mask.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ bool uni(bool v) { return __builtin_amdgcn_readfirstlane((int)v) != 0; }

// ---------------------------------------------------------------- GEMM
// C (M x N) = alpha op(A) op(B) + beta C; op(A) is M x K (A stored K x M if ta)
template <typename T>
__device__ __noinline__ void wg_gemm(Smem<T>& sm, int M, int N, int K, T alpha, const T* A, int lda, bool ta, const T* B, int ldb,
                        bool tb, T beta, T* C, int ldc) {
  M = uni(M); N = uni(N); K = uni(K); lda = uni(lda); ldb = uni(ldb); ldc = uni(ldc); ta = uni(ta); tb = uni(tb);
  typedef typename Mfma<T>::acc acc_t;
  constexpr int GK = GKof<T>::v;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int tilesN = (N + GT - 1) / GT;
  const int tiles = ((M + GT - 1) / GT) * tilesN;
  constexpr int E = GT * GK / BT;   // elements per thread per operand tile
  for (int t = 0; t < tiles; ++t) {
    const int tm = (t / tilesN) * GT, tn = (t % tilesN) * GT;
    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
    T ra[E], rb[E];
    auto load = [&](int k0) {
#pragma unroll
      for (int u = 0; u < E; ++u) {
        const int e = tid + BT * u;
        int i, k;
        if (!ta) { i = e / GK; k = e % GK; } else { k = e / GT; i = e % GT; }
        const int gi = min(tm + i, M - 1), gk = min(k0 + k, K - 1);
        ra[u] = ta ? A[(long long)gk * lda + gi] : A[(long long)gi * lda + gk];
      }
#pragma unroll
      for (int u = 0; u < E; ++u) {
        const int e = tid + BT * u;
        int k, j;
        if (!tb) { k = e / GT; j = e % GT; } else { j = e / GK; k = e % GK; }
        const int gk = min(k0 + k, K - 1), gj = min(tn + j, N - 1);
        rb[u] = tb ? B[(long long)gj * ldb + gk] : B[(long long)gk * ldb + gj];
      }
    };
    auto store = [&](int k0) {
#pragma unroll
      for (int u = 0; u < E; ++u) {
        const int e = tid + BT * u;
        int i, k;
        if (!ta) { i = e / GK; k = e % GK; } else { k = e / GT; i = e % GT; }
        sm.ga[k * GP + i] = (tm + i < M && k0 + k < K) ? ra[u] : T(0);
      }
#pragma unroll
      for (int u = 0; u < E; ++u) {
        const int e = tid + BT * u;
        int k, j;
        if (!tb) { k = e / GT; j = e % GT; } else { j = e / GK; k = e % GK; }
        sm.gb[k * GP + j] = (tn + j < N && k0 + k < K) ? rb[u] : T(0);
      }
    };
    const int nk = (K + GK - 1) / GK;
    if (nk > 0) load(0);
    for (int it = 0; it < nk; ++it) {
      store(it * GK);
      __syncthreads();
      if (it + 1 < nk) load((it + 1) * GK);
#pragma unroll
      for (int kk = 0; kk < GK; kk += 4) {
        T fa[2], fb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) fa[a] = sm.ga[(kk + (lane >> 4)) * GP + wm + 16 * a + (lane & 15)];
#pragma unroll
        for (int b = 0; b < 2; ++b) fb[b] = sm.gb[(kk + (lane >> 4)) * GP + wn + 16 * b + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::op(fa[a], fb[b], acc[a][b]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = tm + wm + 16 * a + Mfma<T>::row(lane, v);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int j = tn + wn + 16 * b + (lane & 15);
          if (i < M && j < N) {
            T* cp = C + (long long)i * ldc + j;
            T val = alpha * acc[a][b][v];
            if (beta != T(0)) val += beta * *cp;
            *cp = val;
          }
        }
      }
  }
  __syncthreads();
}

// ------------------------------------------------------- triangular solves
// op(L) X = B in place (B is n x nrhs).  L is lower triangular (unit or not);
// op(L) = L (forward) or L^T (backward).
template <typename T>
__device__ __noinline__ void wg_trsm_left(Smem<T>& sm, int n, int nrhs, const T* L, int ldl, bool unit, bool trans, T* B,
                             int ldb, int nb) {
  n = uni(n); nrhs = uni(nrhs); ldl = uni(ldl); ldb = uni(ldb); unit = uni(unit); trans = uni(trans);
  const int tid = threadIdx.x;
  nb = min(uni(nb), XNB);
  const int nblk = (n + nb - 1) / nb;
  for (int s = 0; s < nblk; ++s) {
    const int blk = trans ? nblk - 1 - s : s;
    const int k0 = blk * nb, kb = min(nb, n - k0);
    // diagonal block of op(L) into LDS: D(i, k) = op(L)(k0 + i, k0 + k)
    T* D = sm.panel;
    for (int e = tid; e < kb * kb; e += BT) {
      const int i = e / kb, k = e % kb;
      const int r = trans ? k : i, c = trans ? i : k;      // stored coordinates within the block
      D[i * PNB + k] = (c <= r) ? L[(long long)(k0 + r) * ldl + k0 + c] : T(0);
    }
    __syncthreads();
    // substitution: one thread per right-hand side column (register indices
    // are compile-time; rows at and beyond kb are masked)
    for (int j = tid; j < nrhs; j += BT) {
      T x[XNB];
#pragma unroll
      for (int i = 0; i < XNB; ++i) x[i] = B[(long long)(k0 + min(i, kb - 1)) * ldb + j];
      if (!trans) {
#pragma unroll
        for (int i = 0; i < XNB; ++i)
          if (i < kb) {
            T v = x[i];
#pragma unroll
            for (int k = 0; k < i; ++k) v -= D[i * PNB + k] * x[k];
            x[i] = unit ? v : v / D[i * PNB + i];
          }
      } else {
#pragma unroll
        for (int i = XNB - 1; i >= 0; --i)
          if (i < kb) {
            T v = x[i];
#pragma unroll
            for (int k = i + 1; k < XNB; ++k)
              if (k < kb) v -= D[i * PNB + k] * x[k];
            x[i] = unit ? v : v / D[i * PNB + i];
          }
      }
#pragma unroll
      for (int i = 0; i < XNB; ++i)
        if (i < kb) B[(long long)(k0 + i) * ldb + j] = x[i];
    }
    __syncthreads();
    // update the rest: forward B[k0+kb:] -= L[k0+kb:, blk] X_blk;  backward B[:k0] -= L[blk, :k0]^T X_blk
    if (!trans) {
      const int m = n - k0 - kb;
      if (m > 0)
        wg_gemm<T>(sm, m, nrhs, kb, T(-1), L + (long long)(k0 + kb) * ldl + k0, ldl, false,
                   B + (long long)k0 * ldb, ldb, false, T(1), B + (long long)(k0 + kb) * ldb, ldb);
    } else {
      if (k0 > 0)
        wg_gemm<T>(sm, k0, nrhs, kb, T(-1), L + (long long)k0 * ldl, ldl, true, B + (long long)k0 * ldb, ldb,
                   false, T(1), B, ldb);
    }
  }
}

// U X = B in place with U upper triangular (non-unit), backward blocks
template <typename T>
__device__ __noinline__ void wg_trsm_upper(Smem<T>& sm, int n, int nrhs, const T* U, int ldu, T* B, int ldb, int nb) {
  n = uni(n); nrhs = uni(nrhs); ldu = uni(ldu); ldb = uni(ldb);
  const int tid = threadIdx.x;
  nb = min(uni(nb), XNB);
  const int nblk = (n + nb - 1) / nb;
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int k0 = blk * nb, kb = min(nb, n - k0);
    T* D = sm.panel;
    for (int e = tid; e < kb * kb; e += BT) {
      const int i = e / kb, k = e % kb;
      D[i * PNB + k] = (k >= i) ? U[(long long)(k0 + i) * ldu + k0 + k] : T(0);
    }
    __syncthreads();
    for (int j = tid; j < nrhs; j += BT) {
      T x[XNB];
#pragma unroll
      for (int i = 0; i < XNB; ++i) x[i] = B[(long long)(k0 + min(i, kb - 1)) * ldb + j];
#pragma unroll
      for (int i = XNB - 1; i >= 0; --i)
        if (i < kb) {
          T v = x[i];
#pragma unroll
          for (int k = i + 1; k < XNB; ++k)
            if (k < kb) v -= D[i * PNB + k] * x[k];
          x[i] = v / D[i * PNB + i];
        }
#pragma unroll
      for (int i = 0; i < XNB; ++i)
        if (i < kb) B[(long long)(k0 + i) * ldb + j] = x[i];
    }
    __syncthreads();
    if (k0 > 0)
      wg_gemm<T>(sm, k0, nrhs, kb, T(-1), U + k0, ldu, false, B + (long long)k0 * ldb, ldb, false, T(1), B, ldb);
  }
}

// ------------------------------------------------------------ reductions
// (value, index) with the largest value; lowest index on ties; returns to all threads
template <typename T>
__device__ int wg_argmax(Smem<T>& sm, T v, int idx) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const T ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
  if (lane == 0) { sm.red_v[wave] = v; sm.red_i[wave] = idx; }
  __syncthreads();
  T bv = sm.red_v[0];
  int bi = sm.red_i[0];
#pragma unroll
  for (int w = 1; w < BT / 64; ++w) {
    const T ov = sm.red_v[w];
    const int oi = sm.red_i[w];
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  __syncthreads();
  return bi;
}

// ------------------------------------------------------------- LU (GEPP)
// P A = L U in place, piv[k] = row exchanged with k (LAPACK ipiv, 0-based).
// Returns the first zero pivot column + 1, or 0.
template <typename T>
__device__ __noinline__ int wg_getrf(Smem<T>& sm, int n, T* A, int lda, int* piv, int nb) {
  n = uni(n); lda = uni(lda); nb = uni(nb);
  const int tid = threadIdx.x;
  int info = 0;
  for (int k0 = 0; k0 < n; k0 += nb) {
    const int kb = min(nb, n - k0), m = n - k0;
    // panel (rows k0.., columns k0..k0+kb) into LDS: P[r][c]
    T* P = sm.panel;
    for (int e = tid; e < m * kb; e += BT) {
      const int r = e / kb, c = e % kb;
      P[r * PNB + c] = A[(long long)(k0 + r) * lda + k0 + c];
    }
    __syncthreads();
    for (int j = 0; j < kb; ++j) {
      T best = T(-1);
      int bi = INT_MAX;
      for (int r = j + tid; r < m; r += BT) {
        const T a = fabs(P[r * PNB + j]);
        if (a > best) { best = a; bi = r; }
      }
      const int p = wg_argmax<T>(sm, best, bi);
      const int pr = (p == INT_MAX) ? j : p;      // an all-NaN column keeps row j
      if (tid == 0) piv[k0 + j] = k0 + pr;
      if (pr != j)
        for (int c = tid; c < kb; c += BT) {
          const T t = P[j * PNB + c];
          P[j * PNB + c] = P[pr * PNB + c];
          P[pr * PNB + c] = t;
        }
      __syncthreads();
      const T d = P[j * PNB + j];
      if (d == T(0)) {
        if (!info) info = k0 + j + 1;
      } else {
        const T rd = T(1) / d;
        for (int r = j + 1 + tid; r < m; r += BT) {
          const T l = P[r * PNB + j] * rd;
          P[r * PNB + j] = l;
          for (int c = j + 1; c < kb; ++c) P[r * PNB + c] -= l * P[j * PNB + c];
        }
      }
      __syncthreads();
    }
    for (int e = tid; e < m * kb; e += BT) {
      const int r = e / kb, c = e % kb;
      A[(long long)(k0 + r) * lda + k0 + c] = P[r * PNB + c];
    }
    // the panel's interchanges on the columns left and right of it
    for (int c = tid; c < n; c += BT) {
      if (c >= k0 && c < k0 + kb) continue;
      for (int j = 0; j < kb; ++j) {
        const int r2 = piv[k0 + j];
        if (r2 != k0 + j) {
          T* a1 = A + (long long)(k0 + j) * lda + c;
          T* a2 = A + (long long)r2 * lda + c;
          const T t = *a1;
          *a1 = *a2;
          *a2 = t;
        }
      }
    }
    __syncthreads();
    const int rest = n - k0 - kb;
    if (rest > 0) {
      // U12 = L11^{-1} A12, then A22 -= L21 U12
      wg_trsm_left<T>(sm, kb, rest, A + (long long)k0 * lda + k0, lda, true, false, A + (long long)k0 * lda + k0 + kb,
                      lda, nb);
      wg_gemm<T>(sm, rest, rest, kb, T(-1), A + (long long)(k0 + kb) * lda + k0, lda, false,
                 A + (long long)k0 * lda + k0 + kb, lda, false, T(1), A + (long long)(k0 + kb) * lda + k0 + kb, lda);
    }
  }
  return info;
}

// apply the interchanges piv[0..n) to the rows of B (n x nrhs), in order
template <typename T>
__device__ void wg_laswp(int n, int nrhs, T* B, int ldb, const int* piv) {
  n = uni(n); nrhs = uni(nrhs);
  for (int c = threadIdx.x; c < nrhs; c += BT)
    for (int k = 0; k < n; ++k) {
      const int r2 = piv[k];
      if (r2 != k) {
        const T t = B[(long long)k * ldb + c];
        B[(long long)k * ldb + c] = B[(long long)r2 * ldb + c];
        B[(long long)r2 * ldb + c] = t;
      }
    }
  __syncthreads();
}

// ------------------------------------------------------------ Cholesky
// A = L L^T in place (lower triangle).  Returns the first non-positive pivot's
// column (1-based), or 0.
template <typename T>
__device__ __noinline__ int wg_potrf(Smem<T>& sm, int n, T* A, int lda, int nb) {
  n = uni(n); lda = uni(lda);
  const int tid = threadIdx.x;
  nb = min(uni(nb), XNB);
  int bad = 0;
  for (int k0 = 0; k0 < n; k0 += nb) {
    const int kb = min(nb, n - k0);
    T* D = sm.panel;
    for (int e = tid; e < kb * kb; e += BT) {
      const int i = e / kb, k = e % kb;
      D[i * PNB + k] = (k <= i) ? A[(long long)(k0 + i) * lda + k0 + k] : T(0);
    }
    __syncthreads();
    for (int j = 0; j < kb; ++j) {
      const T d = D[j * PNB + j];
      // a non-positive pivot is recorded and the factorization runs on (its
      // square root is NaN): the control flow never depends on the data
      if (!bad && !(d > T(0))) bad = k0 + j + 1;
      const T ljj = sqrt(d);
      __syncthreads();
      if (tid == 0) D[j * PNB + j] = ljj;
      for (int i = j + 1 + tid; i < kb; i += BT) D[i * PNB + j] /= ljj;
      __syncthreads();
      for (int e = tid; e < kb * kb; e += BT) {
        const int i = e / kb, c = e % kb;
        if (i > j && c > j && c <= i) D[i * PNB + c] -= D[i * PNB + j] * D[c * PNB + j];
      }
      __syncthreads();
    }
    for (int e = tid; e < kb * kb; e += BT) {
      const int i = e / kb, k = e % kb;
      if (k <= i) A[(long long)(k0 + i) * lda + k0 + k] = D[i * PNB + k];
    }
    __syncthreads();
    const int rest = n - k0 - kb;
    if (rest > 0) {
      // L21 = A21 L11^{-T}: row r solves L11 x = a_r
      for (int r = tid; r < rest; r += BT) {
        T* row = A + (long long)(k0 + kb + r) * lda + k0;
        T x[XNB];
#pragma unroll
        for (int i = 0; i < XNB; ++i) x[i] = row[min(i, kb - 1)];
#pragma unroll
        for (int i = 0; i < XNB; ++i)
          if (i < kb) {
            T v = x[i];
#pragma unroll
            for (int k = 0; k < i; ++k) v -= D[i * PNB + k] * x[k];
            x[i] = v / D[i * PNB + i];
          }
#pragma unroll
        for (int i = 0; i < XNB; ++i)
          if (i < kb) row[i] = x[i];
      }
      __syncthreads();
      // A22 -= L21 L21^T (full block; the upper part is never read)
      wg_gemm<T>(sm, rest, rest, kb, T(-1), A + (long long)(k0 + kb) * lda + k0, lda, false,
                 A + (long long)(k0 + kb) * lda + k0, lda, true, T(1), A + (long long)(k0 + kb) * lda + k0 + kb, lda);
    }
  }
  return bad;
}

template <typename T>
__device__ void wg_copy(int n, const T* src, T* dst) {
  n = uni(n);
  for (int e = threadIdx.x; e < n * n; e += BT) dst[e] = src[e];
  __syncthreads();
}
template <typename T>
__device__ void wg_identity(int n, T* dst) {
  n = uni(n);
  for (int e = threadIdx.x; e < n * n; e += BT) dst[e] = (e / n == e % n) ? T(1) : T(0);
  __syncthreads();
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

__device__ __forceinline__ int size_class(int n) { return n <= 64 ? 0 : n <= 128 ? 1 : n <= 256 ? 2 : 3; }

template <typename T>
__global__ __launch_bounds__(BT, 1) void k_batched_inv(BatchArgs g) {
  __shared__ Smem<T> sm;
  const int tid = threadIdx.x;
  T* slot = reinterpret_cast<T*>(g.ws) + (long long)blockIdx.x * g.slot_elems;
  for (;;) {
    if (tid == 0) sm.bcast[0] = atomicAdd(g.counter, 1);
    __syncthreads();
    // Branches that guard barriers must be uniform in the compiler's view, not
    // only in value: a branch it takes for divergent runs the skipped side with
    // an empty exec mask, barriers included, on loop bounds it never loaded.
    const int q = __builtin_amdgcn_readfirstlane(sm.bcast[0]);
    __syncthreads();
    if (q >= g.count) break;                          // every wave leaves
    const int mi = __builtin_amdgcn_readfirstlane(g.order[q]);
    const int n = __builtin_amdgcn_readfirstlane(g.n[mi]);
    const int kind = __builtin_amdgcn_readfirstlane(g.kind[mi]);
    if (n < 1 || n > g.nmax || (kind != 0 && kind != 1)) {
      if (tid == 0) g.info[mi] = -1;
      continue;
    }
    const int nb = min(max(g.nb_table[kind][size_class(n)], 1), PNB);
    const T* A = reinterpret_cast<const T*>(g.A[mi]);
    const T* B = reinterpret_cast<const T*>(g.B[mi]);
    T* Xr = reinterpret_cast<T*>(g.Xr[mi]);
    T* Xi = reinterpret_cast<T*>(g.Xi[mi]);
    const long long nn = (long long)n * n;
    T* F = slot;            // factors of A
    T* Y = slot + nn;       // A^{-1} B
    T* Cm = slot + 2 * nn;  // C and its factors
    int* piv = reinterpret_cast<int*>(slot + 3 * nn);
    // A failed factorization does not change the control flow: the remaining
    // steps run on the (non-finite) values, and the status word records the
    // first failing stage and column.
    int info = 0;
    if (kind == 0) {
      // Algorithm 5
      wg_copy<T>(n, A, F);
      const int i1 = __builtin_amdgcn_readfirstlane(wg_getrf<T>(sm, n, F, n, piv, nb));
      if (i1) info = 1000000 + i1;
      wg_copy<T>(n, B, Y);                                              // Y = A^{-1} B
      wg_laswp<T>(n, n, Y, n, piv);
      wg_trsm_left<T>(sm, n, n, F, n, true, false, Y, n, nb);
      wg_trsm_upper<T>(sm, n, n, F, n, Y, n, nb);
      wg_copy<T>(n, A, Cm);                                             // C = A + B Y
      wg_gemm<T>(sm, n, n, n, T(1), B, n, false, Y, n, false, T(1), Cm, n);
      const int i2 = __builtin_amdgcn_readfirstlane(wg_getrf<T>(sm, n, Cm, n, piv, nb));
      if (i2 && !info) info = 2000000 + i2;
      wg_identity<T>(n, Xr);                                            // Re X = C^{-1}
      wg_laswp<T>(n, n, Xr, n, piv);
      wg_trsm_left<T>(sm, n, n, Cm, n, true, false, Xr, n, nb);
      wg_trsm_upper<T>(sm, n, n, Cm, n, Xr, n, nb);
      wg_gemm<T>(sm, n, n, n, T(-1), Y, n, false, Xr, n, false, T(0), Xi, n);   // Im X = -Y C^{-1}
    } else {
      // Algorithm 7
      wg_copy<T>(n, A, F);
      const int i1 = __builtin_amdgcn_readfirstlane(wg_potrf<T>(sm, n, F, n, nb));
      if (i1) info = 1000000 + i1;
      wg_copy<T>(n, B, Cm);                                             // X1 = R1^{-T} B (Cm as scratch)
      wg_trsm_left<T>(sm, n, n, F, n, false, false, Cm, n, nb);
      wg_copy<T>(n, Cm, Y);                                             // Y = R1^{-1} X1
      wg_trsm_left<T>(sm, n, n, F, n, false, true, Y, n, nb);
      // C = A - X1^T X1 into F's place (F is no longer needed)
      wg_copy<T>(n, A, F);
      wg_gemm<T>(sm, n, n, n, T(-1), Cm, n, true, Cm, n, false, T(1), F, n);
      const int i2 = __builtin_amdgcn_readfirstlane(wg_potrf<T>(sm, n, F, n, nb));
      if (i2 && !info) info = 2000000 + i2;
      wg_identity<T>(n, Xr);                                            // Re X = R2^{-1} R2^{-T}
      wg_trsm_left<T>(sm, n, n, F, n, false, false, Xr, n, nb);
      wg_trsm_left<T>(sm, n, n, F, n, false, true, Xr, n, nb);
      wg_gemm<T>(sm, n, n, n, T(-1), Y, n, false, Xr, n, false, T(0), Xi, n);   // Im X = -Y C^{-1}
    }
    if (tid == 0) g.info[mi] = info;
    __syncthreads();
  }
}

// Processing order, largest order first (counting sort on n, one workgroup),
// and reset of the queue head (a kernel, not a memset, so the pair can be
// captured in a graph).
__global__ __launch_bounds__(1024) void k_batched_order(int count, const int* n, int* order, int* counter) {
  __shared__ int hist[BNMAX + 2];
  const int tid = threadIdx.x;
  for (int i = tid; i < BNMAX + 2; i += 1024) hist[i] = 0;
  __syncthreads();
  for (int i = tid; i < count; i += 1024) atomicAdd(&hist[BNMAX - min(max(n[i], 0), BNMAX)], 1);
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int b = 0; b <= BNMAX; ++b) { const int c = hist[b]; hist[b] = run; run += c; }
    *counter = 0;
  }
  __syncthreads();
  for (int i = tid; i < count; i += 1024) {
    const int pos = atomicAdd(&hist[BNMAX - min(max(n[i], 0), BNMAX)], 1);
    order[pos] = i;
  }
}

}  // namespace

size_t batched_ws_bytes(int grid, int nmax, int count, int storage) {
  const size_t el = storage == FROB_PREC_F32 ? sizeof(float) : sizeof(double);
  const size_t slot = 3 * (size_t)nmax * nmax + ((size_t)nmax * sizeof(int) + el - 1) / el + 64;
  return 256 + (((size_t)count * sizeof(int) + 255) & ~size_t(255)) + (size_t)grid * slot * el;
}

int batched_grid(frob_handle* h) {
  int cus = 0;
  FROB_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
  return cus > 0 ? cus : 256;
}

// counter | order[count] | per-workgroup slots
void batched_launch(frob_handle* h, int count, int nmax, const int* n_dev, const int* kind_dev, const void* const* A,
                    const void* const* B, void* const* Xr, void* const* Xi, int* info_dev, int storage) {
  hipStream_t s = h->stream;
  const int grid = batched_grid(h);
  char* ws = (char*)ws_reserve(h, batched_ws_bytes(grid, nmax, count, storage));
  int* counter = reinterpret_cast<int*>(ws);
  int* order = reinterpret_cast<int*>(ws + 256);
  void* slots = ws + 256 + (((size_t)count * sizeof(int) + 255) & ~size_t(255));
  hipLaunchKernelGGL(k_batched_order, dim3(1), dim3(1024), 0, s, count, n_dev, order, counter);
  FROB_LAUNCH_CHECK();
  BatchArgs g;
  g.count = count; g.n = n_dev; g.kind = kind_dev;
  g.A = A; g.B = B; g.Xr = Xr; g.Xi = Xi; g.info = info_dev;
  g.order = order; g.counter = counter; g.ws = slots;
  g.nmax = nmax;
  const size_t el = storage == FROB_PREC_F32 ? sizeof(float) : sizeof(double);
  g.slot_elems = 3 * (long long)nmax * nmax + ((long long)nmax * sizeof(int) + el - 1) / el + 64;
  const int si = storage == FROB_PREC_F32 ? 1 : 0;
  for (int k = 0; k < 2; ++k)
    for (int c = 0; c < 4; ++c) g.nb_table[k][c] = h->batch_nb[si][k][c];
  ProfScope ps(h, PROF_BATCHED, 0.0);
  if (storage == FROB_PREC_F32) hipLaunchKernelGGL(k_batched_inv<float>, dim3(grid), dim3(BT), 0, s, g);
  else hipLaunchKernelGGL(k_batched_inv<double>, dim3(grid), dim3(BT), 0, s, g);
  FROB_LAUNCH_CHECK();
}

namespace {

// Synthetic, strongly diagonally dominant test matrices for the autotuner:
// kind 0: A = R + 2n I, B = S;  kind 1: A = (R + R^T)/2 + 2n I, B = (S - S^T)/2
// (Hermitian, and positive definite by Gershgorin).  R, S entries in [-1, 1)
// from a counter-based hash of (matrix, i, j).
__device__ __forceinline__ double hash_unit(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}
template <typename T>
__global__ void k_tune_fill(int n, int kind, T* A, T* B) {
  const int m = blockIdx.y, i = blockIdx.x, j = threadIdx.x;
  if (j >= n) return;
  const unsigned long long base = ((unsigned long long)m << 40);
  auto r = [&](int s, int a, int b) { return hash_unit(base ^ ((unsigned long long)s << 36) ^ ((unsigned long long)a << 18) ^ b); };
  double a, b;
  if (kind == 0) { a = r(0, i, j); b = r(1, i, j); }
  else { a = 0.5 * (r(0, i, j) + r(0, j, i)); b = 0.5 * (r(1, i, j) - r(1, j, i)); }
  if (i == j) a += 2.0 * n;
  A[(long long)m * n * n + (long long)i * n + j] = (T)a;
  B[(long long)m * n * n + (long long)i * n + j] = (T)b;
}
__global__ void k_tune_ptrs(int count, int n, int kind, char* A, char* B, char* Xr, char* Xi, size_t el,
                            const void** pA, const void** pB, void** pXr, void** pXi, int* pn, int* pk) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= count) return;
  const size_t off = (size_t)m * n * n * el;
  pA[m] = A + off; pB[m] = B + off; pXr[m] = Xr + off; pXi[m] = Xi + off;
  pn[m] = n; pk[m] = kind;
}

}  // namespace

}  // namespace frob

// =========================================================================== C ABI
using namespace frob;

extern "C" frob_status_t frob_inv_batched(frob_handle_t h, int count, int nmax, const int* n_dev, const int* kind_dev,
                                          const void* const* A_dev, const void* const* B_dev, void* const* Xr_dev,
                                          void* const* Xi_dev, int* info_dev, int storage) {
  if (!h || count < 1 || nmax < 1 || nmax > BNMAX || !n_dev || !kind_dev || !A_dev || !B_dev || !Xr_dev || !Xi_dev ||
      !info_dev || (storage != FROB_PREC_F64 && storage != FROB_PREC_F32))
    return FROB_E_ARG;
  try {
    FROB_HIP(hipSetDevice(h->device));
    batched_launch(h, count, nmax, n_dev, kind_dev, A_dev, B_dev, Xr_dev, Xi_dev, info_dev, storage);
    return FROB_OK;
  } catch (const std::bad_alloc&) {
    return FROB_E_ALLOC;
  } catch (const HipError&) {
    return FROB_E_HIP;
  } catch (...) {
    return FROB_E_INTERNAL;
  }
}

extern "C" frob_status_t frob_batched_tune(frob_handle_t h, int storage, int table_out[8]) {
  if (!h || (storage != FROB_PREC_F64 && storage != FROB_PREC_F32)) return FROB_E_ARG;
  const int si = storage == FROB_PREC_F32 ? 1 : 0;
  const size_t el = storage == FROB_PREC_F32 ? sizeof(float) : sizeof(double);
  static const int class_n[4] = {64, 128, 256, 512};
  static const int cands[3] = {8, 16, 32};
  char *A = nullptr, *B = nullptr, *Xr = nullptr, *Xi = nullptr, *meta = nullptr;
  frob_status_t st = FROB_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int saved_prof = h->prof;
  h->prof = 0;   // tuning launches stay out of the kernel-class timings
  try {
    FROB_HIP(hipSetDevice(h->device));
    hipStream_t s = h->stream;
    const int count = 2 * batched_grid(h);   // two matrices per workgroup
    const size_t bytes = (size_t)count * BNMAX * BNMAX * el;
    FROB_HIP(hipMalloc((void**)&A, bytes));
    FROB_HIP(hipMalloc((void**)&B, bytes));
    FROB_HIP(hipMalloc((void**)&Xr, bytes));
    FROB_HIP(hipMalloc((void**)&Xi, bytes));
    FROB_HIP(hipMalloc((void**)&meta, (size_t)count * (4 * sizeof(void*) + 3 * sizeof(int)) + 256));
    const void** pA = (const void**)meta;
    const void** pB = pA + count;
    void** pXr = (void**)(pB + count);
    void** pXi = pXr + count;
    int* pn = (int*)(pXi + count);
    int* pk = pn + count;
    int* pinfo = pk + count;
    FROB_HIP(hipEventCreate(&e0));
    FROB_HIP(hipEventCreate(&e1));
    for (int kind = 0; kind < 2; ++kind)
      for (int c = 0; c < 4; ++c) {
        const int n = class_n[c];
        if (storage == FROB_PREC_F32)
          hipLaunchKernelGGL(k_tune_fill<float>, dim3(n, count), dim3(n), 0, s, n, kind, (float*)A, (float*)B);
        else
          hipLaunchKernelGGL(k_tune_fill<double>, dim3(n, count), dim3(n), 0, s, n, kind, (double*)A, (double*)B);
        FROB_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_tune_ptrs, dim3((count + 255) / 256), dim3(256), 0, s, count, n, kind, A, B, Xr, Xi, el,
                           pA, pB, pXr, pXi, pn, pk);
        FROB_LAUNCH_CHECK();
        float best = 1e30f;
        int bestnb = h->batch_nb[si][kind][c];
        for (int nb : cands) {
          h->batch_nb[si][kind][c] = nb;
          batched_launch(h, count, n, pn, pk, pA, pB, pXr, pXi, pinfo, storage);   // warm
          FROB_HIP(hipEventRecord(e0, s));
          batched_launch(h, count, n, pn, pk, pA, pB, pXr, pXi, pinfo, storage);
          FROB_HIP(hipEventRecord(e1, s));
          FROB_HIP(hipEventSynchronize(e1));
          float ms = 0.f;
          FROB_HIP(hipEventElapsedTime(&ms, e0, e1));
          if (ms < best) { best = ms; bestnb = nb; }
        }
        h->batch_nb[si][kind][c] = bestnb;
      }
    FROB_HIP(hipStreamSynchronize(s));
  } catch (const std::bad_alloc&) {
    st = FROB_E_ALLOC;
  } catch (const HipError&) {
    st = FROB_E_HIP;
  } catch (...) {
    st = FROB_E_INTERNAL;
  }
  h->prof = saved_prof;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (char* p : {A, B, Xr, Xi, meta})
    if (p) (void)hipFree(p);
  if (table_out)
    for (int k = 0; k < 2; ++k)
      for (int c = 0; c < 4; ++c) table_out[4 * k + c] = h->batch_nb[si][k][c];
  return st;
}
