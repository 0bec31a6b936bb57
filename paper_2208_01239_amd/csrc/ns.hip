// ns.hip -- Newton-Schulz refinement of a computed inverse.
//
//   R = I - M X,   X <- X + X R,     so that I - M X_new = (I - M X)^2.
//
// The residual and its norm are formed in FP64; the correction X R may use a
// lower operand precision (its error is relative to the already small R):
// that of the factorizations, or FP32 after FP64 factorizations when asked.
//
// Convergence control.  R_k = R_0^(2^k), so the iteration converges when the
// spectral radius of R_0 is below one; ||R_0||_2 < 1 suffices, and then
// ||R_{k+1}||_F <= ||R_k||_2 ||R_k||_F decreases every step.
//  - ||R_0||_F < 1: start (it bounds ||R_0||_2).
//  - otherwise ||R_0||_2 is estimated by power iteration on R_0^H R_0 (a lower
//    bound); an estimate >= 1 refuses (FROB_NO_CONVERGENCE, X unrefined).
//    Below one the start is tentative: X_0 is kept, and if ||R||_F grows
//    before it drops below one, X_0 is restored and FROB_NO_CONVERGENCE
//    returned.
//  - Stop with success when ||R||_F / sqrt(n) <= tol, at the step limit
//    (optionally without forming the residual of the last iterate), or at the
//    rounding floor: the norm no longer halves although exact squaring would
//    have made it at least four times smaller (||R_{k+1}||_F > 4 ||R_k||_F^2).
//    A slow start (||R_k||_2 near one) fails the second test and continues.
//
// Both complex products are formed from three real matrix-core GEMMs with
// Gauss's scheme (Proposition 2.2 with tau = 1):
//   (P + iQ)(S + iT):  M1 = (P - Q)(S + T), M2 = P T, M3 = Q S,
//                      real = M1 - M2 + M3, imag = M2 + M3.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "handle.hpp"
#include "internal.hpp"

namespace frob {

size_t ns_ws_bytes(int n, int steps) {
  if (steps <= 0) return 0;
  Carve c(nullptr);
  for (int k = 0; k < 8; ++k) c.take<double>((size_t)n * n);
  c.take<double>(6 * (size_t)n + 64);
  return c.off;
}

namespace {

constexpr int PW_ITERS = 8;     // power iterations of the 2-norm estimate
constexpr int GV = 256;         // threads per block of the matrix-vector kernels
constexpr int GV_ROWS = 64;     // rows per block of the conjugate-transposed product

// y = s R x for planar complex R (n x n, ld), s = *scale; one wave per row.
__global__ void k_zgemv_n(int n, const double* __restrict__ Rr, const double* __restrict__ Ri, int ld,
                          const double* __restrict__ xr, const double* __restrict__ xi,
                          const double* __restrict__ scale, double* __restrict__ yr, double* __restrict__ yi) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (GV / 64) + (threadIdx.x >> 6);
  if (i >= n) return;
  const double* pr = Rr + (long long)i * ld;
  const double* pi = Ri + (long long)i * ld;
  double ar = 0.0, ai = 0.0;
  for (int j = lane; j < n; j += 64) {
    const double a = pr[j], b = pi[j], c = xr[j], d = xi[j];
    ar += a * c - b * d;
    ai += a * d + b * c;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    ar += __shfl_xor(ar, off);
    ai += __shfl_xor(ai, off);
  }
  if (lane == 0) {
    const double s = *scale;
    yr[i] = s * ar;
    yi[i] = s * ai;
  }
}

// y += s R^H x over the rows of this block (y zeroed beforehand); threads run
// over columns, so each row is read contiguously.
__global__ void k_zgemv_h(int n, const double* __restrict__ Rr, const double* __restrict__ Ri, int ld,
                          const double* __restrict__ xr, const double* __restrict__ xi,
                          const double* __restrict__ scale, double* yr, double* yi) {
  const int j = blockIdx.x * GV + threadIdx.x;
  if (j >= n) return;
  const int i0 = blockIdx.y * GV_ROWS, i1 = min(n, i0 + GV_ROWS);
  double ar = 0.0, ai = 0.0;
  for (int i = i0; i < i1; ++i) {
    const double a = Rr[(long long)i * ld + j], b = Ri[(long long)i * ld + j], c = xr[i], d = xi[i];
    ar += a * c + b * d;     // conj(a + ib) (c + id)
    ai += a * d - b * c;
  }
  const double s = *scale;
  atomicAdd(yr + j, s * ar);
  atomicAdd(yi + j, s * ai);
}

// norm = ||x||_2, *scale = 1 / norm (one block)
__global__ void k_znorm(int n, const double* __restrict__ xr, const double* __restrict__ xi, double* norm,
                        double* scale) {
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += GV) acc += xr[j] * xr[j] + xi[j] * xi[j];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  __shared__ double part[GV / 64];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < GV / 64; ++w) t += part[w];
    const double nr = sqrt(t);
    *norm = nr;
    *scale = nr > 0.0 ? 1.0 / nr : 0.0;
  }
}

// start vector: entries in [-1, 1) from a counter-based hash of the index
__global__ void k_zstart(int n, double* xr, double* xi) {
  const int j = blockIdx.x * GV + threadIdx.x;
  if (j >= n) return;
  auto h = [](unsigned long long x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  };
  xr[j] = h(2ull * j);
  xi[j] = h(2ull * j + 1);
}

// Lower bound of ||R||_2 for planar complex R: PW_ITERS power iterations on
// R^H R, returning ||R v|| for the last unit vector v.  `vec` holds 6n + 64
// doubles.
double norm2_estimate(hipStream_t s, int n, const double* Rr, const double* Ri, int ld, double* vec) {
  double *vr = vec, *vi = vec + n, *ur = vec + 2 * n, *ui = vec + 3 * n, *wr = vec + 4 * n, *wi = vec + 5 * n;
  double* sc = vec + 6 * n;            // sc[0]: scale of v, sc[1 + t]: ||R v_t||, sc[32]: scale of u
  const int gb = ceil_div(n, GV);
  hipLaunchKernelGGL(k_zstart, dim3(gb), dim3(GV), 0, s, n, vr, vi);
  FROB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_znorm, dim3(1), dim3(GV), 0, s, n, vr, vi, sc + 40, sc);
  FROB_LAUNCH_CHECK();
  for (int t = 0; t < PW_ITERS; ++t) {
    // u = R v / ||v||;  ||u|| = ||R v_hat||
    hipLaunchKernelGGL(k_zgemv_n, dim3(ceil_div(n, GV / 64)), dim3(GV), 0, s, n, Rr, Ri, ld, vr, vi, sc, ur, ui);
    FROB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_znorm, dim3(1), dim3(GV), 0, s, n, ur, ui, sc + 1 + t, sc + 32);
    FROB_LAUNCH_CHECK();
    // v = R^H u / ||u||
    fill_f64(s, 1, 2 * n, 0.0, wr, 2 * n);
    hipLaunchKernelGGL(k_zgemv_h, dim3(gb, ceil_div(n, GV_ROWS)), dim3(GV), 0, s, n, Rr, Ri, ld, ur, ui, sc + 32,
                       wr, wi);
    FROB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_znorm, dim3(1), dim3(GV), 0, s, n, wr, wi, sc + 40, sc);
    FROB_LAUNCH_CHECK();
    std::swap(vr, wr);
    std::swap(vi, wi);
  }
  double est[PW_ITERS];
  FROB_HIP(hipMemcpyAsync(est, sc + 1, sizeof(est), hipMemcpyDeviceToHost, s));
  FROB_HIP(hipStreamSynchronize(s));
  double e = 0.0;
  for (double v : est) e = std::max(e, v);
  return e;
}

}  // namespace

// (Zr, Zi) = (Pr + i Pi)(Sr + i Si) via three GEMMs; T1, T2 scratch n x n.
static void gauss3m(hipStream_t s, int n, const double* Pr, int ldp, const double* Pi, const double* Sr, int lds,
                    const double* Si, double* Zr, double* Zi, int ldz, double* T1, double* T2) {
  const int ld = n;
  // T1 = P_r - P_i, T2 = S_r + S_i
  lincomb_f64(s, n, n, 1.0, Pr, ldp, -1.0, Pi, ldp, T1, ld);
  lincomb_f64(s, n, n, 1.0, Sr, lds, 1.0, Si, lds, T2, ld);
  // Zi = M2 = P_r S_i ; Zr = M3 = P_i S_r
  gemm_f64(s, false, false, n, n, n, 1.0, DOp{Pr, ldp, nullptr}, TRI_NONE, DOp{Si, lds, nullptr}, TRI_NONE, 0.0,
           DOut{Zi, ldz, nullptr, nullptr});
  gemm_f64(s, false, false, n, n, n, 1.0, DOp{Pi, ldp, nullptr}, TRI_NONE, DOp{Sr, lds, nullptr}, TRI_NONE, 0.0,
           DOut{Zr, ldz, nullptr, nullptr});
  // (Zr, Zi) <- (M3 - M2, M3 + M2), elementwise from the old values
  rotate_f64(s, n, n, 1.0, Zr, ldz, Zi, ldz, Zr, ldz, Zi, ldz);
  gemm_f64(s, false, false, n, n, n, 1.0, DOp{T1, ld, nullptr}, TRI_NONE, DOp{T2, ld, nullptr}, TRI_NONE, 1.0,
           DOut{Zr, ldz, nullptr, nullptr});                        // Zr += M1
}

frob_status_t ns_refine(frob_handle* h, int n, const double* A, int lda, const double* B, int ldb, double* Xr,
                        double* Xi, int ldx, int max_steps, double tol, int prec, int flags, Carve& c,
                        frob_result_t* r) {
  hipStream_t s = h->stream;
  const size_t nn = (size_t)n * n;
  double* Rr = c.take<double>(nn);
  double* Ri = c.take<double>(nn);
  double* Ur = c.take<double>(nn);
  double* Ui = c.take<double>(nn);
  double* T1 = c.take<double>(nn);
  double* T2 = c.take<double>(nn);
  double* X0r = c.take<double>(nn);   // the start, kept while it is tentative
  double* X0i = c.take<double>(nn);
  double* vec = c.take<double>(6 * (size_t)n + 64);
  if (!(tol > 0.0)) tol = 1e-14;
  const double rn = std::sqrt((double)n);
  const int cprec = (prec == LP_NONE && (flags & FROB_REFINE_F32_CORRECTION)) ? LP_F32 : prec;
  double prev = 0.0;
  int steps = 0;
  bool tentative = false;
  frob_status_t st = FROB_OK;
  r->norm2_est = 0.0;
  for (int k = 0;; ++k) {
    if (k > 0 && k == max_steps && (flags & FROB_REFINE_SKIP_FINAL_RESID)) {
      r->resid = std::nan("");   // step limit reached; the closing residual is not formed
      break;
    }
    // R = I - M X in FP64, and its Frobenius norm
    gauss3m(s, n, A, lda, B, Xr, ldx, Xi, Rr, Ri, n, T1, T2);
    resid_form_f64(s, n, Rr, Ri, n, h->dnorm);
    FROB_HIP(hipMemcpyAsync(h->hnorm, h->dnorm, sizeof(double), hipMemcpyDeviceToHost, s));
    FROB_HIP(hipStreamSynchronize(s));
    const double fro = std::sqrt(*h->hnorm);
    const double rho = fro / rn;
    if (k == 0) {
      r->resid0 = rho;
      if (!(fro < 1.0)) {
        // ||R_0||_F does not bound the spectral norm below one: estimate it
        const double e2 = std::isfinite(fro) ? norm2_estimate(s, n, Rr, Ri, n, vec) : INFINITY;
        r->norm2_est = e2;
        if (!(e2 < 1.0)) { st = FROB_NO_CONVERGENCE; r->resid = rho; break; }
        tentative = true;
        copy_f64(s, n, n, Xr, ldx, nullptr, X0r, n);
        copy_f64(s, n, n, Xi, ldx, nullptr, X0i, n);
      }
    } else {
      if (tentative && !(fro < prev)) {
        // the estimate missed: ||R||_F grew before falling below one
        copy_f64(s, n, n, X0r, n, nullptr, Xr, ldx);
        copy_f64(s, n, n, X0i, n, nullptr, Xi, ldx);
        FROB_HIP(hipStreamSynchronize(s));
        st = FROB_NO_CONVERGENCE;
        r->resid = r->resid0;
        steps = 0;
        break;
      }
      if (fro < 1.0) tentative = false;
    }
    r->resid = rho;
    if (rho <= tol) break;                                               // converged
    if (k > 0 && fro > 0.5 * prev && fro > 4.0 * prev * prev) break;     // rounding floor
    if (k == max_steps) break;
    // X <- X + X R, the three products of Gauss's scheme accumulated into X:
    // M2 = Xr Ri, M3 = Xi Rr, then X += (M3 - M2, M3 + M2), then
    // Re X += M1 = (Xr - Xi)(Rr + Ri) (its factors taken before X changes)
    {
      LowPrecScope lp(cprec);
      lincomb_f64(s, n, n, 1.0, Xr, ldx, -1.0, Xi, ldx, T1, n);
      lincomb_f64(s, n, n, 1.0, Rr, n, 1.0, Ri, n, T2, n);
      gemm_f64(s, false, false, n, n, n, 1.0, DOp{Xr, ldx, nullptr}, TRI_NONE, DOp{Ri, n, nullptr}, TRI_NONE, 0.0,
               DOut{Ui, n, nullptr, nullptr});
      gemm_f64(s, false, false, n, n, n, 1.0, DOp{Xi, ldx, nullptr}, TRI_NONE, DOp{Rr, n, nullptr}, TRI_NONE, 0.0,
               DOut{Ur, n, nullptr, nullptr});
      acc_rot_f64(s, n, n, Ur, n, Ui, n, Xr, Xi, ldx);
      gemm_f64(s, false, false, n, n, n, 1.0, DOp{T1, n, nullptr}, TRI_NONE, DOp{T2, n, nullptr}, TRI_NONE, 1.0,
               DOut{Xr, ldx, nullptr, nullptr});
    }
    prev = fro;
    ++steps;
  }
  r->refine_steps = steps;
  return st;
}

}  // namespace frob
