// ns.hip -- Newton-Schulz refinement of a computed inverse.
//
//   R = I - M X,   X <- X + X R,     so that I - M X_new = (I - M X)^2.
//
// The residual and its norm are formed in FP64; the correction X R may use a
// lower operand precision (its error is relative to the already small R):
// that of the factorizations, or FP32 after FP64 factorizations when asked.
// Refinement stops when ||R||_F / sqrt(n) reaches the tolerance, when it no
// longer halves (the FP64 rounding floor, about u kappa(M)), or after the
// step limit (optionally without forming the residual of the last iterate);
// it does not start when ||R||_F >= 1.
//
// Both complex products are formed from three real matrix-core GEMMs with
// Gauss's scheme (Proposition 2.2 with tau = 1):
//   (P + iQ)(S + iT):  M1 = (P - Q)(S + T), M2 = P T, M3 = Q S,
//                      real = M1 - M2 + M3, imag = M2 + M3.
#include <cmath>

#include "common.hpp"
#include "handle.hpp"
#include "internal.hpp"

namespace frob {

size_t ns_ws_bytes(int n, int steps) {
  if (steps <= 0) return 0;
  Carve c(nullptr);
  for (int k = 0; k < 6; ++k) c.take<double>((size_t)n * n);
  return c.off;
}

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
  if (!(tol > 0.0)) tol = 1e-14;
  const double rn = std::sqrt((double)n);
  const int cprec = (prec == LP_NONE && (flags & FROB_REFINE_F32_CORRECTION)) ? LP_F32 : prec;
  double prev = 0.0;
  int steps = 0;
  frob_status_t st = FROB_OK;
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
      // I - M X_{k+1} = (I - M X_k)^2: a Frobenius norm >= 1 gives no guarantee of convergence
      if (!(fro < 1.0)) { st = FROB_NO_CONVERGENCE; r->resid = rho; break; }
    }
    r->resid = rho;
    if (rho <= tol) break;                              // converged
    if (k > 0 && rho > 0.5 * prev) break;               // no longer contracting: rounding floor reached
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
    prev = rho;
    ++steps;
  }
  r->refine_steps = steps;
  return st;
}

}  // namespace frob
