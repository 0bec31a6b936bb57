// cbase.hip -- the complex-arithmetic baselines beside Frobenius inversion.
//
// frob_cinv_lu:   Algorithm 4 (inversion with LU decomposition) in complex
//                 arithmetic on planar storage;
// frob_cinv_chol: Algorithm 8 (inversion with Cholesky decomposition).
// Both run on the same kind of kernels as the Frobenius paths (register-leaf
// LU / LDS-base Cholesky, diagonal-inverse triangular solves, matrix-core
// GEMMs), here with four real MFMA products per complex tile product.
#include <algorithm>
#include <cstring>

#include "../../include/frobinv.h"
#include "common.hpp"
#include "handle.hpp"
#include "internal.hpp"

using namespace frob;

namespace {

size_t zsolver_work_elems(int n) {
  size_t w = trsm_z_work_elems(n);
  w = std::max(w, getrf_z_work_elems(n));
  w = std::max(w, potrf_z_work_elems(n));
  w = std::max(w, trtri_z_tmp_elems(n));
  return w;
}

template <class F>
frob_status_t zguarded(frob_handle_t h, F&& f) {
  if (!h) return FROB_E_ARG;
  try {
    FROB_HIP(hipSetDevice(h->device));
    return f();
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

}  // namespace

size_t frob::cinv_lu_ws(int n) {
  const size_t nn = (size_t)n * n;
  Carve sz(nullptr);
  for (int k = 0; k < 4; ++k) sz.take<double>(nn);
  sz.take<int>(n);
  sz.take<double>(zsolver_work_elems(n));
  return sz.off + 256;
}

extern "C" {

frob_status_t frob_cinv_lu(frob_handle_t h, int n, const double* Mr, const double* Mi, int ldm, double* Xr,
                           double* Xi, int ldx, int form, frob_result_t* res) {
  if (!h || !Mr || !Mi || !Xr || !Xi || n < 1 || n > FROB_MAX_N || ldm < n || ldx < n || (form != 0 && form != 1))
    return FROB_E_ARG;
  return zguarded(h, [&]() -> frob_status_t {
    hipStream_t s = h->stream;
    const size_t nn = (size_t)n * n;
    // behind whatever an enclosing call (a Newton driver) keeps at the front
    const size_t lead = ws_lead();
    Carve c((char*)ws_reserve(h, lead + cinv_lu_ws(n)));
    c.off = lead;
    double* Fr = c.take<double>(nn);
    double* Fi = c.take<double>(nn);
    double* Wr = c.take<double>(nn);
    double* Wi = c.take<double>(nn);
    int* perm = c.take<int>(n);
    double* work = c.take<double>(zsolver_work_elems(n));
    fill_i32(s, INFO_SLOTS, 0, h->dinfo);
    // step 1: X = P^T L U
    copy_f64(s, n, n, Mr, ldm, nullptr, Fr, n);
    copy_f64(s, n, n, Mi, ldm, nullptr, Fi, n);
    getrf_z64(s, n, Fr, Fi, n, perm, h->dinfo, work, lookahead(h));
    ZOp LU{Fr, Fi, n, perm};
    ZOut W{Wr, Wi, n, nullptr, nullptr};
    if (form == 0) {
      // step 2: U X1 = I (substitution against the full identity)
      identity_f64(s, n, Wr, n);
      fill_f64(s, n, n, 0.0, Wi, n);
      trsm_z64(s, false, TRI_UPPER, OP_N, n, n, LU, W, work);
    } else {
      // U^{-1} by a triangular inverse (LAPACK getri style)
      trtri_z64(s, TRI_UPPER, OP_N, n, LU, Wr, Wi, n, work);
    }
    // step 3: X2 L = X1
    trsm_z64(s, true, TRI_LOWER_UNIT, OP_N, n, n, LU, W, work);
    // step 4: X^{-1} = X2 P
    permute_cols_f64(s, n, n, Wr, n, perm, Xr, ldx);
    permute_cols_f64(s, n, n, Wi, n, perm, Xi, ldx);
    read_info(h);
    frob_result_t r;
    std::memset(&r, 0, sizeof(r));
    frob_status_t st = FROB_OK;
    if (h->hinfo[0]) { st = FROB_SINGULAR; r.info = h->hinfo[0]; r.stage = 1; }
    if (res) *res = r;
    return st;
  });
}

frob_status_t frob_cinv_chol(frob_handle_t h, int n, const double* Mr, const double* Mi, int ldm, double* Xr,
                             double* Xi, int ldx, int form, frob_result_t* res) {
  if (!h || !Mr || !Mi || !Xr || !Xi || n < 1 || n > FROB_MAX_N || ldm < n || ldx < n || (form != 0 && form != 1))
    return FROB_E_ARG;
  return zguarded(h, [&]() -> frob_status_t {
    hipStream_t s = h->stream;
    const size_t nn = (size_t)n * n;
    Carve sz(nullptr);
    for (int k = 0; k < 4; ++k) sz.take<double>(nn);
    sz.take<double>(zsolver_work_elems(n));
    Carve c((char*)ws_reserve(h, sz.off));
    double* Fr = c.take<double>(nn);
    double* Fi = c.take<double>(nn);
    double* Wr = c.take<double>(nn);
    double* Wi = c.take<double>(nn);
    double* work = c.take<double>(zsolver_work_elems(n));
    fill_i32(s, INFO_SLOTS, 0, h->dinfo);
    // step 1: M = R^H R, stored as the lower factor L = R^H
    copy_f64(s, n, n, Mr, ldm, nullptr, Fr, n);
    copy_f64(s, n, n, Mi, ldm, nullptr, Fi, n);
    potrf_z64(s, n, Fr, Fi, n, h->dinfo, work);
    ZOp L{Fr, Fi, n, nullptr};
    if (form == 0) {
      // step 2: R^H X1 = I (L X1 = I);  step 3: R X2 = X1 (L^H X2 = X1)
      ZOut X{Xr, Xi, ldx, nullptr, nullptr};
      identity_f64(s, n, Xr, ldx);
      fill_f64(s, n, n, 0.0, Xi, ldx);
      trsm_z64(s, false, TRI_LOWER, OP_N, n, n, L, X, work);
      trsm_z64(s, false, TRI_UPPER, OP_C, n, n, L, X, work);
    } else {
      // LAPACK potri style: W = L^{-1}, X = W^H W (lower half, then mirrored)
      trtri_z64(s, TRI_LOWER, OP_N, n, L, Wr, Wi, n, work);
      gemm_z64(s, OP_C, OP_N, n, n, n, 1.0, ZOp{Wr, Wi, n, nullptr}, TRI_UPPER, ZOp{Wr, Wi, n, nullptr}, TRI_LOWER,
               0.0, ZOut{Xr, Xi, ldx, nullptr, nullptr}, true);
      mirror_lower_f64(s, n, Xr, ldx, 1.0);
      mirror_lower_f64(s, n, Xi, ldx, -1.0);
    }
    read_info(h);
    frob_result_t r;
    std::memset(&r, 0, sizeof(r));
    frob_status_t st = FROB_OK;
    if (h->hinfo[0]) { st = FROB_NOT_HPD; r.info = h->hinfo[0]; r.stage = 1; }
    if (res) *res = r;
    return st;
  });
}

}  // extern "C"
