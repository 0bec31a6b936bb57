// adjoint.hip -- reverse-mode derivative of the inversion, for a batch of
// matrices:  dM = -X^H G X^H,  X = M^{-1},  G = dL/dX (G = dL/dRe X + i dL/dIm X,
// the convention under which dL = Re tr(G^H dX)).  It follows from
// dX = -X dM X: Re tr(G^H dX) = Re tr((-X^H G X^H)^H dM).
//
// The two complex products T = G X^H and dM = -X^H T are each formed with
// Gauss's three-real-multiplication scheme (Proposition 2.2 with tau = 1):
//   (P + iQ)(R + iS):  M1 = (P - Q)(R + S), M2 = P S, M3 = Q R,
//                      real = M1 - M2 + M3,  imag = M2 + M3,
// i.e. three batched real GEMMs plus elementwise combinations instead of four
// GEMMs.  Storage FP64 (FP64 matrix-core GEMMs) or FP32 (FP32 matrix-core
// GEMMs with FP32 accumulation).  Arrays are batch x n x n, contiguous.
#include "common.hpp"
#include "handle.hpp"
#include "internal.hpp"

namespace frob {

namespace {

constexpr int AB = 256;

// out = x + s y over `count` elements
template <typename T>
__global__ void k_axpy_flat(long long count, const T* __restrict__ x, double s, const T* __restrict__ y,
                            T* __restrict__ out) {
  const long long i = (long long)blockIdx.x * AB + threadIdx.x;
  if (i < count) out[i] = (T)((double)x[i] + s * (double)y[i]);
}

// (a, b, w) = (M1, M2, M3)  ->  a = re = sg (M1 - M2 + M3), im = sg (M2 + M3)
// written to `im` (b or w: each element is read before it is written).  With
// d1, d2: also the factors of the next product's M1, d1 = xr + xi and
// d2 = re + im (from the stored, rounded re and im).
template <typename T>
__global__ void k_combine3m(long long count, T* a, T* b, const T* w, T* im, double sg, const T* xr, const T* xi,
                            T* d1, T* d2) {
  const long long i = (long long)blockIdx.x * AB + threadIdx.x;
  if (i >= count) return;
  const double m1 = a[i], m2 = b[i], m3 = w[i];
  const T re = (T)(sg * (m1 - m2 + m3));
  const T ie = (T)(sg * (m2 + m3));
  a[i] = re;
  im[i] = ie;
  if (d1) {
    d1[i] = (T)((double)xr[i] + (double)xi[i]);
    d2[i] = (T)((double)re + (double)ie);
  }
}

template <typename T>
void axpy_flat(hipStream_t s, long long count, const T* x, double sc, const T* y, T* out) {
  hipLaunchKernelGGL(k_axpy_flat<T>, dim3((unsigned)((count + AB - 1) / AB)), dim3(AB), 0, s, count, x, sc, y, out);
  FROB_LAUNCH_CHECK();
}
template <typename T>
void combine3m(hipStream_t s, long long count, T* a, T* b, const T* w, T* im, double sg, const T* xr = nullptr,
               const T* xi = nullptr, T* d1 = nullptr, T* d2 = nullptr) {
  hipLaunchKernelGGL(k_combine3m<T>, dim3((unsigned)((count + AB - 1) / AB)), dim3(AB), 0, s, count, a, b, w, im, sg,
                     xr, xi, d1, d2);
  FROB_LAUNCH_CHECK();
}

// batched C = alpha op(A) op(B), all n x n with stride n^2
void bgemm(hipStream_t s, bool ta, bool tb, int n, int batch, double alpha, const double* A, const double* B,
           double* C) {
  const long long st = (long long)n * n;
  gemm_f64_batched(s, ta, tb, n, n, n, alpha, DOp{A, n, nullptr}, TRI_NONE, DOp{B, n, nullptr}, TRI_NONE, 0.0,
                   DOut{C, n, nullptr, nullptr}, false, batch, st, st, st, 0, 0, 0);
}
void bgemm(hipStream_t s, bool ta, bool tb, int n, int batch, double alpha, const float* A, const float* B,
           float* C) {
  const long long st = (long long)n * n;
  gemm_lp(s, LP_F32, ta, tb, n, n, n, alpha, A, n, nullptr, B, n, nullptr, 0.0, C, n, nullptr, false, batch, st,
          st, st);
}

template <typename T>
void adjoint_t(hipStream_t s, int batch, int n, const T* Xr, const T* Xi, const T* Gr, const T* Gi, T* dMr, T* dMi,
               T* D1, T* D2, T* W) {
  const long long cnt = (long long)batch * n * n;
  // T = G X^H:  P = Gr, Q = Gi, R = Xr^T, S = -Xi^T
  //   M1 = (Gr - Gi)(Xr - Xi)^T,  M2 = -Gr Xi^T,  M3 = Gi Xr^T   (T kept in dMr, dMi)
  axpy_flat(s, cnt, Gr, -1.0, Gi, D1);
  axpy_flat(s, cnt, Xr, -1.0, Xi, D2);
  bgemm(s, false, true, n, batch, 1.0, D1, D2, dMr);
  bgemm(s, false, true, n, batch, -1.0, Gr, Xi, dMi);
  bgemm(s, false, true, n, batch, 1.0, Gi, Xr, W);
  // dM = -X^H T:  P = Xr^T, Q = -Xi^T, R = Tr, S = Ti
  //   M1 = (Xr + Xi)^T (Tr + Ti),  M2 = Xr^T Ti,  M3 = -Xi^T Tr
  // (T into dMr, dMi and the factors of M1 into D1, D2 in one pass)
  combine3m(s, cnt, dMr, dMi, W, dMi, 1.0, Xr, Xi, D1, D2);
  bgemm(s, true, false, n, batch, 1.0, Xr, dMi, W);          // M2 (reads Ti before it is overwritten)
  bgemm(s, true, false, n, batch, -1.0, Xi, dMr, dMi);       // M3 -> dMi (Tr still intact)
  bgemm(s, true, false, n, batch, 1.0, D1, D2, dMr);         // M1 -> dMr
  // (dMr, W, dMi) = (M1, M2, M3): re = -(M1 - M2 + M3) -> dMr, im = -(M2 + M3) -> dMi
  combine3m(s, cnt, dMr, W, (const T*)dMi, dMi, -1.0);
}

}  // namespace

size_t adjoint_ws_bytes(int batch, int n, int storage) {
  const size_t el = storage == FROB_PREC_F32 ? sizeof(float) : sizeof(double);
  Carve c(nullptr);
  for (int k = 0; k < 3; ++k) c.take<char>((size_t)batch * n * n * el);
  return c.off;
}

void adjoint_run(frob_handle* h, int batch, int n, int storage, const void* Xr, const void* Xi, const void* Gr,
                 const void* Gi, void* dMr, void* dMi) {
  hipStream_t s = h->stream;
  Carve c((char*)ws_reserve(h, adjoint_ws_bytes(batch, n, storage)));
  const size_t cnt = (size_t)batch * n * n;
  ProfScope ps(h, PROF_ADJOINT, 12.0 * batch * (double)n * n * n);
  if (storage == FROB_PREC_F32) {
    float* D1 = c.take<float>(cnt);
    float* D2 = c.take<float>(cnt);
    float* W = c.take<float>(cnt);
    adjoint_t<float>(s, batch, n, (const float*)Xr, (const float*)Xi, (const float*)Gr, (const float*)Gi,
                     (float*)dMr, (float*)dMi, D1, D2, W);
  } else {
    double* D1 = c.take<double>(cnt);
    double* D2 = c.take<double>(cnt);
    double* W = c.take<double>(cnt);
    adjoint_t<double>(s, batch, n, (const double*)Xr, (const double*)Xi, (const double*)Gr, (const double*)Gi,
                      (double*)dMr, (double*)dMi, D1, D2, W);
  }
}

}  // namespace frob

// =========================================================================== C ABI
extern "C" frob_status_t frob_inv_adjoint(frob_handle_t h, int batch, int n, int storage, const void* Xr,
                                          const void* Xi, const void* Gr, const void* Gi, void* dMr, void* dMi) {
  using namespace frob;
  if (!h || !Xr || !Xi || !Gr || !Gi || !dMr || !dMi || batch < 1 || n < 1 || n > FROB_MAX_N) return FROB_E_ARG;
  if (storage != FROB_PREC_F64 && storage != FROB_PREC_F32) return FROB_E_ARG;
  if ((long long)batch * n * n > (1LL << 31)) return FROB_E_ARG;
  const void* ins[4] = {Xr, Xi, Gr, Gi};
  for (const void* p : ins)
    if (p == dMr || p == dMi) return FROB_E_ARG;
  if (dMr == dMi) return FROB_E_ARG;
  try {
    FROB_HIP(hipSetDevice(h->device));
    adjoint_run(h, batch, n, storage, Xr, Xi, Gr, Gi, dMr, dMi);
    FROB_HIP(hipStreamSynchronize(h->stream));
    prof_resolve(h);
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
