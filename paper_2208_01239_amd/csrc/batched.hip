// batched.hip -- many Frobenius inversions of uneven order in one persistent
// launch (the batching line of growth).
//
// One workgroup (256 threads) inverts one matrix at a time, start to finish,
// two workgroups per compute unit: it takes the next matrix index from an
// atomic queue whose order (largest order first, the longest-processing-time
// rule) is prepared on the device, and runs Algorithm 5 (general) or
// Algorithm 7 (Hermitian positive definite) with the in-workgroup building
// blocks of batched_dev.hpp:
//   - GEMM: tile shape chosen per product (128x128 down to 16x256 / 256x16),
//     16x16x4 matrix-core products (FP64, or FP32 with FP32 accumulation),
//     operand tiles double-buffered in LDS;
//   - LU with partial pivoting: panels of NB columns factored in LDS (pivot
//     search by wave reductions), interchanges applied as one composite row
//     map, updates in the order of the recursive algorithm;
//   - Cholesky and triangular solves: NB x NB diagonal blocks by substitution,
//     updates in the same recursive order.
// The matrices stay in global memory; each workgroup owns a private slot of
// workspace (three n_max x n_max matrices and the row map).  Panel width NB
// per size class comes from the caller's table (autotuned by
// frob_batched_tune).
#include <algorithm>
#include <climits>
#include <mutex>

#include "common.hpp"
#include "handle.hpp"
#include "internal.hpp"

namespace frob {

// Primitives of the building blocks in batched_dev.hpp, on gfx950.
namespace bat {
#define BB_FN __device__ __noinline__
#define BB_IN __device__ __forceinline__
#define BB_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ int bb_tid() { return threadIdx.x; }
__device__ __forceinline__ void bb_sync() { __syncthreads(); }
template <class V>
__device__ __forceinline__ V bb_shfl_xor(V v, int mask) { return __shfl_xor(v, mask); }
__device__ __forceinline__ int bb_first(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ d4 bb_mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 bb_mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int bb_atomic_add(int* p, int v) { return atomicAdd(p, v); }
}  // namespace bat
}  // namespace frob

#include "batched_dev.hpp"

namespace frob {

namespace {

using bat::BatchArgs;
using bat::BNMAX;
using bat::BT;
using bat::Smem;

template <typename T>
// Two workgroups per compute unit (LDS and registers are sized for it): while
// one waits on memory or a barrier, the other computes.
__global__ __launch_bounds__(BT, 2) void k_batched_inv(BatchArgs g) {
  __shared__ Smem<T> sm;
  bat::batched_worker<T>(g, sm, blockIdx.x);
}

__global__ __launch_bounds__(1024) void k_batched_order(int count, const int* n, int* order, int* counter) {
  __shared__ int hist[BNMAX + 2];
  bat::batched_order_body(1024, count, n, order, counter, hist);
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
  return 2 * (cus > 0 ? cus : 256);   // two workgroups per compute unit
}

size_t batched_slot_elems(int nmax, int storage) {
  const size_t el = storage == FROB_PREC_F32 ? sizeof(float) : sizeof(double);
  return 3 * (size_t)nmax * nmax + ((size_t)nmax * sizeof(int) + el - 1) / el + 64;
}

// The two launches of a batched inversion on memory the caller provides:
// the queue head, the order array (count ints) and `grid` slots.
static void batched_enqueue(frob_handle* h, int grid, int* counter, int* order, void* slots, int count, int nmax,
                            const int* n_dev, const int* kind_dev, const void* const* A, const void* const* B,
                            void* const* Xr, void* const* Xi, int* info_dev, int storage) {
  hipStream_t s = h->stream;
  hipLaunchKernelGGL(k_batched_order, dim3(1), dim3(1024), 0, s, count, n_dev, order, counter);
  FROB_LAUNCH_CHECK();
  BatchArgs g;
  g.count = count; g.n = n_dev; g.kind = kind_dev;
  g.A = A; g.B = B; g.Xr = Xr; g.Xi = Xi; g.info = info_dev;
  g.order = order; g.counter = counter; g.ws = slots;
  g.nmax = nmax;
  g.slot_elems = (long long)batched_slot_elems(nmax, storage);
  const int si = storage == FROB_PREC_F32 ? 1 : 0;
  for (int k = 0; k < 2; ++k)
    for (int c = 0; c < 4; ++c) g.nb_table[k][c] = h->batch_nb[si][k][c];
  if (storage == FROB_PREC_F32) hipLaunchKernelGGL(k_batched_inv<float>, dim3(grid), dim3(BT), 0, s, g);
  else hipLaunchKernelGGL(k_batched_inv<double>, dim3(grid), dim3(BT), 0, s, g);
  FROB_LAUNCH_CHECK();
}

// counter | order[count] | per-workgroup slots, in the handle's workspace
void batched_launch(frob_handle* h, int count, int nmax, const int* n_dev, const int* kind_dev, const void* const* A,
                    const void* const* B, void* const* Xr, void* const* Xi, int* info_dev, int storage) {
  const int grid = std::min(batched_grid(h), std::max(count, 1));   // no idle workgroups sharing a CU
  char* ws = (char*)ws_reserve(h, batched_ws_bytes(grid, nmax, count, storage));
  mark_ws_captured(h);   // a captured launch keeps this workspace alive
  int* counter = reinterpret_cast<int*>(ws);
  int* order = reinterpret_cast<int*>(ws + 256);
  void* slots = ws + 256 + (((size_t)count * sizeof(int) + 255) & ~size_t(255));
  ProfScope ps(h, PROF_BATCHED, 0.0);
  batched_enqueue(h, grid, counter, order, slots, count, nmax, n_dev, kind_dev, A, B, Xr, Xi, info_dev, storage);
}

// ----------------------------------------------------- no-allocation variant
namespace {

// Scratch of frob_inv_batched_noalloc (queue head, order array, workgroup
// slots) as a file-scope device array: each GPU the library runs on holds
// its own copy until the process ends.  Host code must use the per-device
// address resolved in batched_scratch_init, never the array's name.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(128) << 20;
constexpr int NOALLOC_MAX_COUNT = 1 << 20;
__device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

char* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < NOALLOC_MAX_DEVICES) ? g_scratch_ptr[device] : nullptr;
}

}  // namespace

void batched_scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= NOALLOC_MAX_DEVICES || g_scratch_ptr[device]) return;
  void* p = nullptr;
  FROB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));   // `device` is current
  g_scratch_ptr[device] = static_cast<char*>(p);
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
  } catch (const CaptureGrowth&) {
    return FROB_E_CAPTURE;
  } catch (const HipError&) {
    return FROB_E_HIP;
  } catch (...) {
    return FROB_E_INTERNAL;
  }
}

extern "C" frob_status_t frob_inv_batched_noalloc(frob_handle_t h, int count, int nmax, const int* n_dev,
                                                  const int* kind_dev, const void* const* A_dev,
                                                  const void* const* B_dev, void* const* Xr_dev, void* const* Xi_dev,
                                                  int* info_dev, int storage) {
  if (!h || count < 1 || count > NOALLOC_MAX_COUNT || nmax < 1 || nmax > BNMAX || !n_dev || !kind_dev || !A_dev ||
      !B_dev || !Xr_dev || !Xi_dev || !info_dev || (storage != FROB_PREC_F64 && storage != FROB_PREC_F32))
    return FROB_E_ARG;
  try {
    FROB_HIP(hipSetDevice(h->device));
    char* base = scratch_ptr(h->device);
    if (!base) return FROB_E_INTERNAL;
    const size_t head = 256 + (((size_t)count * sizeof(int) + 255) & ~size_t(255));
    const size_t el = storage == FROB_PREC_F32 ? sizeof(float) : sizeof(double);
    const size_t slot_bytes = batched_slot_elems(nmax, storage) * el;
    const size_t fit = (NOALLOC_SCRATCH_BYTES - head) / slot_bytes;   // >= 20 for every accepted shape
    const int grid = (int)std::min<size_t>(std::min<size_t>((size_t)batched_grid(h), fit), (size_t)std::max(count, 1));
    if (grid < 1) return FROB_E_ARG;
    batched_enqueue(h, grid, reinterpret_cast<int*>(base), reinterpret_cast<int*>(base + 256), base + head, count,
                    nmax, n_dev, kind_dev, A_dev, B_dev, Xr_dev, Xi_dev, info_dev, storage);
    return FROB_OK;
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
  static const int cands[3] = {4, 8, 16};
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
