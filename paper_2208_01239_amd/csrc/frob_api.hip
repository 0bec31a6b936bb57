// frob_api.hip -- the C ABI of libfrobinv and the Frobenius inversion drivers.
//
// frob_inv_general: Algorithm 5 (Frobenius inversion with LU), with the
//   almost-sure shift of Algorithm 6 on demand;
// frob_inv_hpd:     Algorithm 7 (Frobenius inversion with Cholesky);
// frob_solve:       Algorithm 3 (linear systems, sign of step 7 corrected).
// The complex-arithmetic baselines (Algorithms 4 and 8) live in cbase.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>

#include "../../include/frobinv.h"
#include "common.hpp"
#include "handle.hpp"
#include "internal.hpp"

using namespace frob;

namespace frob {

// ------------------------------------------------------------------ handle
uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double draw_mu(frob_handle* h) {
  for (;;) {
    const double u = (double)(splitmix64(h->rng) >> 11) * 0x1.0p-53;
    if (u > 0.0) return u;
  }
}

static bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(s, &cs);
  if (e == hipErrorStreamCaptureImplicit) {   // the null stream while another stream is being captured
    (void)hipGetLastError();
    return true;
  }
  FROB_HIP(e);
  return cs != hipStreamCaptureStatusNone;
}

bool mark_ws_captured(frob_handle* h) {
  if (!stream_capturing(h->stream)) return false;
  h->ws_captured = true;
  return true;
}

void* ws_reserve(frob_handle* h, size_t bytes) {
  bytes += 64 * 256;  // alignment slack: sub-carves may start at unaligned offsets
  if (bytes <= h->ws_cap) return h->ws;
  // a graph being captured would bake in a buffer that the next growth frees:
  // the caller must run the call once eagerly first (documented in the header)
  if (stream_capturing(h->stream)) throw CaptureGrowth();
  FROB_HIP(hipStreamSynchronize(h->stream));
  if (h->ws) {
    if (h->ws_captured) h->ws_retired.push_back(h->ws);   // a graph may still write it
    else FROB_HIP(hipFree(h->ws));
  }
  h->ws = nullptr;
  h->ws_cap = 0;
  h->ws_captured = false;
  const size_t cap = bytes + (bytes >> 3);
  if (hipMalloc(&h->ws, cap) != hipSuccess) {
    h->ws = nullptr;
    throw std::bad_alloc();
  }
  h->ws_cap = cap;
  return h->ws;
}

const LookAhead* lookahead(frob_handle* h) {
  if (!h) return nullptr;
  if (!h->la.s1) {
    // default priority (the same as every other stream the library uses)
    FROB_HIP(hipStreamCreateWithFlags(&h->la.s1, hipStreamNonBlocking));
    for (auto& e : h->la.ev) FROB_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->la.prof = h;
  }
  return &h->la;
}

size_t solver_work_elems(int n) {
  size_t w = trsm_work_elems(n);
  w = std::max(w, getrf_work_elems(n));
  w = std::max(w, potrf_work_elems(n));
  w = std::max(w, trtri_tmp_elems(n));
  return w;
}

void read_info(frob_handle* h) {
  FROB_HIP(hipMemcpyAsync(h->hinfo, h->dinfo, sizeof(int) * INFO_SLOTS, hipMemcpyDeviceToHost, h->stream));
  FROB_HIP(hipStreamSynchronize(h->stream));
  prof_resolve(h);
}

static hipEvent_t prof_event(frob_handle* h) {
  if (!h->pool.empty()) {
    hipEvent_t e = h->pool.back();
    h->pool.pop_back();
    return e;
  }
  hipEvent_t e;
  FROB_HIP(hipEventCreate(&e));
  return e;
}

ProfScope::ProfScope(frob_handle* hh, int c, double fl, hipStream_t s, double by)
    : h(hh), cls(c), flops(fl), bytes(by), st(s) {
  if (!h || !h->prof) return;
  if (!st) st = h->stream;
  e0 = prof_event(h);
  FROB_HIP(hipEventRecord(e0, st));
}

ProfScope::~ProfScope() {
  if (!h || !h->prof || !e0) return;
  try {
    hipEvent_t e1 = prof_event(h);
    if (hipEventRecord(e1, st) != hipSuccess) return;
    h->pending.push_back({e0, e1, cls, flops, bytes});
  } catch (...) {
  }
}

void prof_resolve(frob_handle* h) {
  for (auto& p : h->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.e1) == hipSuccess && hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
      h->prof_ms[p.cls] += ms;
      h->prof_flops[p.cls] += p.flops;
      h->prof_bytes[p.cls] += p.bytes;
      h->prof_count[p.cls] += 1;
    }
    h->pool.push_back(p.e0);
    h->pool.push_back(p.e1);
  }
  h->pending.clear();
}

}  // namespace frob

namespace {

// opts.panel: 0 (the default width) or 16, 32, 48, 64
bool panel_ok(int p) { return p == 0 || (p >= 16 && p <= LA_NB && p % 16 == 0); }

// The look-ahead LUs of one call use the caller's panel width; the handle's
// setting is restored when the call returns.
struct PanelScope {
  frob_handle* h;
  int prev;
  PanelScope(frob_handle* hh, int p) : h(hh), prev(hh->la.nb) { h->la.nb = p ? p : LA_NB; }
  ~PanelScope() { h->la.nb = prev; }
};

frob_opts_t opts_or_default(const frob_opts_t* o) {
  frob_opts_t d;
  frob_default_opts(&d);
  return o ? *o : d;
}

struct Status {
  frob_status_t st;
};

template <class F>
frob_status_t guarded(frob_handle_t h, F&& f) {
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

bool bad_dims(int n, int lda) { return n < 1 || n > FROB_MAX_N || lda < n; }

// ---------------------------------------------------------------------------
// One pass of Algorithm 5 on (A, B) -> (Xr, Xi); factorization status in
// dinfo[0] (LU of A) and dinfo[1] (LU of C).
// ---------------------------------------------------------------------------
struct GenWs {
  double *F, *Y, *C, *W, *tmp;
  int *p1, *p2;
  double* cond;   // n column sums, then ||C||_1 and ||C^{-1}||_1
  bool want_cond;
  int ld;    // Y, W
  int ldF;   // F and C: n x 2n, room for the columns carried through their LU
  frob_handle* h;
};

size_t gen_ws_bytes(int n) {
  Carve c(nullptr);
  const size_t nn = (size_t)n * n;
  c.take<double>(2 * nn); c.take<double>(nn); c.take<double>(2 * nn); c.take<double>(nn);
  c.take<double>(solver_work_elems(n));
  c.take<int>(n); c.take<int>(n);
  c.take<double>((size_t)n + 8);
  return c.off;
}

GenWs gen_ws_carve(Carve& c, int n) {
  GenWs w;
  const size_t nn = (size_t)n * n;
  w.F = c.take<double>(2 * nn); w.Y = c.take<double>(nn); w.C = c.take<double>(2 * nn); w.W = c.take<double>(nn);
  w.tmp = c.take<double>(solver_work_elems(n));
  w.p1 = c.take<int>(n); w.p2 = c.take<int>(n);
  w.cond = c.take<double>((size_t)n + 8);
  w.want_cond = false;
  w.ld = n;
  w.ldF = 2 * n;
  w.h = nullptr;
  return w;
}

// Workspace carved ahead of an entry point's own: the FP32-storage twins keep
// their FP64 copies of the operands there while they call the FP64 entry
// point (set only for the duration of that call, on the calling thread).
thread_local size_t t_lead_bytes = 0;

struct LeadScope {
  size_t prev;
  explicit LeadScope(size_t b) : prev(t_lead_bytes) { t_lead_bytes = b; }
  ~LeadScope() { t_lead_bytes = prev; }
};

size_t lead_total(size_t bytes) { return t_lead_bytes + 256 + bytes; }

// bytes of `doubles` FP64 values, rounded up to the carving alignment
size_t lead_of(size_t doubles) { return ((doubles * sizeof(double)) + 255) & ~size_t(255); }

Carve reserve_carve(frob_handle* h, size_t bytes) {
  Carve c((char*)ws_reserve(h, lead_total(bytes)));
  c.off = t_lead_bytes;
  return c;
}

// Bytes of workspace of one call of each FP64 entry point.
size_t general_ws(int n, int refine, bool keep = false) {
  const size_t nn = (size_t)n * n;
  Carve sz(nullptr);
  sz.take<char>(gen_ws_bytes(n));
  sz.take<double>(nn); sz.take<double>(nn);   // shifted A, B
  if (keep) { sz.take<double>(nn); sz.take<double>(nn); }   // best inverse kept by FROB_SHIFT_COND
  sz.take<char>(ns_ws_bytes(n, refine));
  return sz.off;
}

size_t hpd_ws(int n, int refine) {
  const size_t nn = (size_t)n * n;
  Carve sz(nullptr);
  for (int k = 0; k < 5; ++k) sz.take<double>(nn);
  sz.take<double>(solver_work_elems(n));
  sz.take<double>(trsm_work_elems(n));
  sz.take<char>(ns_ws_bytes(n, refine));
  return sz.off;
}

size_t solve_ws(int n, int nrhs) {
  const size_t nn = (size_t)n * n;
  const int q = 2 * nrhs;
  Carve sz(nullptr);
  sz.take<char>(gen_ws_bytes(n));
  sz.take<double>(nn); sz.take<double>(nn);
  sz.take<double>((size_t)n * q); sz.take<double>((size_t)n * q); sz.take<double>((size_t)n * q);
  return sz.off;
}

// Steps 1-4 of Algorithm 5 (shared with Algorithm 3): LU of A, Y = A^{-1} B,
// C = A + B Y, LU of C.
// With the look-ahead LU (orders up to LA_CARRY_MAX), B rides along the LU
// of A as extra columns (they take L1^{-1} P1 on the second stream, off the
// panel chain), and with `cinv` the identity rides along the LU of C, leaving
// L2^{-1} P2 for C^{-1} = U2^{-1} L2^{-1} P2.  Returns whether it did.
bool frob_lu_front(hipStream_t s, int n, const double* A, int lda, const double* B, int ldb, GenWs& w, int* dinfo,
                   bool cinv) {
  const int ld = w.ld, lf = w.ldF;
  const LookAhead* la = lookahead(w.h);
  const bool carry = getrf_lookahead_on(n, la) && n <= LA_CARRY_MAX;
  DOp LU1{w.F, lf, w.p1};
  DOut Yo{w.Y, ld, nullptr, nullptr};
  // step 1: P1 A = L1 U1;  step 2: Y = U1^{-1} L1^{-1} P1 B
  copy_f64(s, n, n, A, lda, nullptr, w.F, lf);
  if (carry) {
    copy_f64(s, n, n, B, ldb, nullptr, w.F + n, lf);
    getrf_f64(s, n, w.F, lf, w.p1, dinfo + 0, w.tmp, la, n);
    copy_f64(s, n, n, w.F + n, lf, w.p1, w.Y, ld);   // L1^{-1} P1 B in logical row order
  } else {
    getrf_f64(s, n, w.F, lf, w.p1, dinfo + 0, w.tmp, la);
    copy_f64(s, n, n, B, ldb, w.p1, w.Y, ld);
    trsm_f64(s, false, TRI_LOWER_UNIT, false, n, n, LU1, Yo, w.tmp);
  }
  trsm_f64(s, false, TRI_UPPER, false, n, n, LU1, Yo, w.tmp);
  // step 3: C = A + B Y
  copy_f64(s, n, n, A, lda, nullptr, w.C, lf);
  {
    ProfScope ps(w.h, PROF_GEMM_NNN, 2.0 * n * (double)n * n, nullptr, 32.0 * n * (double)n);
    gemm_f64(s, false, false, n, n, n, 1.0, DOp{B, ldb, nullptr}, TRI_NONE, DOp{w.Y, ld, nullptr}, TRI_NONE, 1.0,
             DOut{w.C, lf, nullptr, nullptr});
  }
  if (w.want_cond) norm1_f64(s, n, w.C, lf, w.cond, w.cond + n);   // ||C||_1, before C is factored
  // step 4: P2 C = L2 U2   (a zero pivot here means M is singular, Lemma 2.3)
  const bool carry2 = carry && cinv;
  if (carry2) identity_f64(s, n, w.C + n, lf);
  getrf_f64(s, n, w.C, lf, w.p2, dinfo + 1, w.tmp, la, carry2 ? n : 0);
  return carry2;
}

void frob_lu_pass(hipStream_t s, int n, const double* A, int lda, const double* B, int ldb, double* Xr, double* Xi,
                  int ldx, GenWs& w, int* dinfo) {
  const int ld = w.ld;
  const bool carried = frob_lu_front(s, n, A, lda, B, ldb, w, dinfo, true);
  // step 5, first block row: Re X = C^{-1} = U2^{-1} L2^{-1} P2
  DOp LU2{w.C, w.ldF, w.p2};
  if (carried) {
    copy_f64(s, n, n, w.C + n, w.ldF, w.p2, Xr, ldx);   // L2^{-1} P2 in logical row order
    trsm_f64(s, false, TRI_UPPER, false, n, n, LU2, DOut{Xr, ldx, nullptr, nullptr}, w.tmp);
  } else {
    trtri_f64(s, TRI_UPPER, false, n, LU2, w.W, ld, w.tmp);
    trsm_f64(s, true, TRI_LOWER_UNIT, false, n, n, LU2, DOut{w.W, ld, nullptr, nullptr}, w.tmp);
    permute_cols_f64(s, n, n, w.W, ld, w.p2, Xr, ldx);
  }
  if (w.want_cond) norm1_f64(s, n, Xr, ldx, w.cond, w.cond + n + 1);   // ||C^{-1}||_1
  // step 5, second block row: Im X = -Y C^{-1}
  {
    ProfScope ps(w.h, PROF_GEMM_NNN, 2.0 * n * (double)n * n, nullptr, 24.0 * n * (double)n);
    gemm_f64(s, false, false, n, n, n, -1.0, DOp{w.Y, ld, nullptr}, TRI_NONE, DOp{Xr, ldx, nullptr}, TRI_NONE, 0.0,
             DOut{Xi, ldx, nullptr, nullptr});
  }
}

}  // namespace

// =========================================================================== C ABI
extern "C" {

void frob_default_opts(frob_opts_t* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->shift = FROB_SHIFT_AUTO;
  o->mu = 0.0;
  o->seed = 0;
  o->refine = 0;
  o->prec = FROB_PREC_F64;
  o->refine_tol = 0.0;
  o->refine_flags = 0;
}

frob_status_t frob_create(frob_handle_t* out, int device) {
  if (!out) return FROB_E_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return FROB_E_HIP;
  if (device < 0 || device >= count) return FROB_E_ARG;
  frob_handle* h = new (std::nothrow) frob_handle();
  if (!h) return FROB_E_ALLOC;
  h->device = device;
  h->rng = 0x2208012390ull;
  try {
    FROB_HIP(hipSetDevice(device));
    batched_scratch_init(device);
    h->stream = nullptr;   // the device's null stream until frob_set_stream says otherwise
    FROB_HIP(hipMalloc((void**)&h->dinfo, sizeof(int) * INFO_SLOTS));
    FROB_HIP(hipHostMalloc((void**)&h->hinfo, sizeof(int) * INFO_SLOTS, hipHostMallocDefault));
    FROB_HIP(hipMalloc((void**)&h->dnorm, sizeof(double)));
    FROB_HIP(hipHostMalloc((void**)&h->hnorm, sizeof(double), hipHostMallocDefault));
  } catch (...) {
    frob_destroy(h);
    return FROB_E_HIP;
  }
  *out = h;
  return FROB_OK;
}

frob_status_t frob_destroy(frob_handle_t h) {
  if (!h) return FROB_E_ARG;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  if (h->ws) (void)hipFree(h->ws);
  for (void* p : h->ws_retired) (void)hipFree(p);
  if (h->dinfo) (void)hipFree(h->dinfo);
  if (h->hinfo) (void)hipHostFree(h->hinfo);
  if (h->dnorm) (void)hipFree(h->dnorm);
  if (h->hnorm) (void)hipHostFree(h->hnorm);
  for (auto& p : h->pending) { (void)hipEventDestroy(p.e0); (void)hipEventDestroy(p.e1); }
  for (auto e : h->pool) (void)hipEventDestroy(e);
  if (h->la.s1) {
    (void)hipStreamSynchronize(h->la.s1);
    for (auto e : h->la.ev)
      if (e) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(h->la.s1);
  }
  delete h;
  return FROB_OK;
}

frob_status_t frob_set_stream(frob_handle_t h, void* stream) {
  if (!h) return FROB_E_ARG;
  h->stream = (hipStream_t)stream;
  return FROB_OK;
}

size_t frob_workspace_bytes(frob_handle_t h) { return h ? h->ws_cap : 0; }

frob_status_t frob_inv_general(frob_handle_t h, int n, const double* A, int lda, const double* B, int ldb, double* Xr,
                               double* Xi, int ldx, const frob_opts_t* opts, frob_result_t* res) {
  if (!h || !A || !B || !Xr || !Xi || bad_dims(n, lda) || ldb < n || ldx < n) return FROB_E_ARG;
  const frob_opts_t o = opts_or_default(opts);
  if (o.shift < FROB_SHIFT_OFF || o.shift > FROB_SHIFT_COND || o.refine < 0 || o.prec < FROB_PREC_F64 ||
      o.prec > FROB_PREC_BF16 || (o.shift == FROB_SHIFT_PHASE && !std::isfinite(o.theta)) || !panel_ok(o.panel))
    return FROB_E_ARG;
  return guarded(h, [&]() -> frob_status_t {
    PanelScope pw(h, o.panel);
    if (o.seed) h->rng = o.seed;
    hipStream_t s = h->stream;
    const size_t nn = (size_t)n * n;
    const bool keep = o.shift == FROB_SHIFT_COND;
    Carve c = reserve_carve(h, general_ws(n, o.refine, keep));
    GenWs w = gen_ws_carve(c, n);
    w.h = h;
    w.want_cond = keep || (o.refine_flags & FROB_REPORT_COND);
    double* As = c.take<double>(nn);
    double* Bs = c.take<double>(nn);
    double* Kr = keep ? c.take<double>(nn) : nullptr;
    double* Ki = keep ? c.take<double>(nn) : nullptr;
    frob_result_t r;
    std::memset(&r, 0, sizeof(r));
    frob_status_t st = FROB_OK;
    bool done = false;
    LowPrecScope lp(o.prec);   // FP32 / BF16 operands in the products of the factorization passes
    double hc[2] = {0.0, 0.0};
    auto read_cond = [&]() {
      if (!w.want_cond) return 0.0;
      FROB_HIP(hipMemcpyAsync(hc, w.cond + n, sizeof(hc), hipMemcpyDeviceToHost, s));
      FROB_HIP(hipStreamSynchronize(s));
      return hc[0] * hc[1];
    };
    // One pass of Algorithm 5 on e^{i theta} M (theta = 0: M itself), the
    // inverse rotated back; returns false if the real part is singular.
    auto rotated_pass = [&](double theta) {
      const double cs = std::cos(theta), sn = std::sin(theta);
      const bool rot = theta != 0.0;
      if (rot) rot_f64(s, n, n, cs, sn, A, lda, B, ldb, As, n, Bs, n);
      fill_i32(s, INFO_SLOTS, 0, h->dinfo);
      frob_lu_pass(s, n, rot ? As : A, rot ? n : lda, rot ? Bs : B, rot ? n : ldb, Xr, Xi, ldx, w, h->dinfo);
      read_info(h);
      if (h->hinfo[0] != 0) { r.info = h->hinfo[0]; r.stage = 1; return false; }
      if (h->hinfo[1]) { st = FROB_SINGULAR; r.info = h->hinfo[1]; r.stage = 2; return true; }
      if (rot) rot_f64(s, n, n, cs, sn, Xr, ldx, Xi, ldx, Xr, ldx, Xi, ldx);
      r.info = 0; r.stage = 0; r.theta = theta;
      return true;
    };
    if (o.shift == FROB_SHIFT_PHASE) {
      done = rotated_pass(o.theta);
      if (!done) st = FROB_SINGULAR;
      if (st == FROB_OK) r.cond1_C = read_cond();
    } else if (o.shift == FROB_SHIFT_COND) {
      // theta = 0 (eq. (Finv)), -pi/2 (the formula for invertible B), then the diagonals
      const double pi = 3.14159265358979323846;
      const double thetas[4] = {0.0, -0.5 * pi, 0.25 * pi, -0.25 * pi};
      const double tol = o.cond_tol > 0.0 ? o.cond_tol : 1e-10;
      double best = INFINITY, best_theta = 0.0;
      bool have = false, cur_is_best = false;
      for (int t = 0; t < 4; ++t) {
        st = FROB_OK;
        r.shifts_tried++;
        cur_is_best = false;
        if (!rotated_pass(thetas[t]) || st != FROB_OK) { st = FROB_OK; continue; }
        const double k1 = read_cond();
        const bool meets = 0x1p-53 * k1 <= tol;
        if (k1 < best) {
          best = k1; best_theta = thetas[t]; have = true; cur_is_best = true;
          if (!meets && t < 3) {   // kept while the next rotation is tried
            copy_f64(s, n, n, Xr, ldx, nullptr, Kr, n);
            copy_f64(s, n, n, Xi, ldx, nullptr, Ki, n);
          }
        }
        if (meets) break;          // the first rotation that meets the target is also the best so far
      }
      if (have && !cur_is_best) {   // restore the best-conditioned inverse
        copy_f64(s, n, n, Kr, n, nullptr, Xr, ldx);
        copy_f64(s, n, n, Ki, n, nullptr, Xi, ldx);
      }
      done = have;
      st = have ? FROB_OK : FROB_SINGULAR;
      if (have) { r.cond1_C = best; r.theta = best_theta; r.info = 0; r.stage = 0; }
    } else {
      if (o.shift != FROB_SHIFT_ON) {
        fill_i32(s, INFO_SLOTS, 0, h->dinfo);
        frob_lu_pass(s, n, A, lda, B, ldb, Xr, Xi, ldx, w, h->dinfo);
        read_info(h);
        if (h->hinfo[0] == 0) {
          done = true;
          if (h->hinfo[1]) { st = FROB_SINGULAR; r.info = h->hinfo[1]; r.stage = 2; }
        } else if (o.shift == FROB_SHIFT_OFF) {
          done = true;
          st = FROB_SINGULAR; r.info = h->hinfo[0]; r.stage = 1;
        }
      }
      // Algorithm 6: invert (1 + i mu) M, whose real part A - mu B is singular for
      // at most n values of mu (Lemma 4.3), then multiply the inverse by (1 + i mu).
      for (int attempt = 0; !done && attempt < 3; ++attempt) {
        const double mu = (o.mu > 0.0 && attempt == 0) ? o.mu : draw_mu(h);
        r.shifts_tried++;
        rotate_f64(s, n, n, mu, A, lda, B, ldb, As, n, Bs, n);        // X1 = A - mu B, X2 = mu A + B
        fill_i32(s, INFO_SLOTS, 0, h->dinfo);
        frob_lu_pass(s, n, As, n, Bs, n, Xr, Xi, ldx, w, h->dinfo);   // X3 + i X4 = (X1 + i X2)^{-1}
        read_info(h);
        if (h->hinfo[0] != 0) { r.info = h->hinfo[0]; r.stage = 1; continue; }
        done = true;
        r.mu_used = mu;
        if (h->hinfo[1]) { st = FROB_SINGULAR; r.info = h->hinfo[1]; r.stage = 2; break; }
        rotate_f64(s, n, n, mu, Xr, ldx, Xi, ldx, Xr, ldx, Xi, ldx);   // X5 = X3 - mu X4, X6 = mu X3 + X4
        r.info = 0; r.stage = 0;
      }
      if (!done) st = FROB_SINGULAR;
      if (st == FROB_OK) r.cond1_C = read_cond();
    }
    if (st == FROB_OK && o.refine > 0) {
      LowPrecScope fp64(LP_NONE);   // the residual is formed in FP64
      st = ns_refine(h, n, A, lda, B, ldb, Xr, Xi, ldx, o.refine, o.refine_tol, o.prec, o.refine_flags, c, &r);
    } else if (st == FROB_OK) {
      FROB_HIP(hipStreamSynchronize(s));
    }
    if (res) *res = r;
    return st;
  });
}

}  // extern "C"

namespace {

// Algorithm 7.  step5_sign = -1: Hermitian positive definite M (B skew, so
// B A^{-1} B = -X1^T X1 and C = A - X1^T X1); step5_sign = +1: A and B
// symmetric positive definite (B A^{-1} B = X1^T X1, C = A + X1^T X1).
frob_status_t chol_path(frob_handle* h, int n, const double* A, int lda, const double* B, int ldb, double* Xr,
                        double* Xi, int ldx, const frob_opts_t* opts, frob_result_t* res, double step5_sign) {
  if (!h || !A || !B || !Xr || !Xi || bad_dims(n, lda) || ldb < n || ldx < n) return FROB_E_ARG;
  const frob_opts_t o = opts_or_default(opts);
  if (o.refine < 0 || o.prec < FROB_PREC_F64 || o.prec > FROB_PREC_BF16) return FROB_E_ARG;
  return guarded(h, [&]() -> frob_status_t {
    hipStream_t s = h->stream;
    const size_t nn = (size_t)n * n;
    Carve c = reserve_carve(h, hpd_ws(n, o.refine));
    double* F = c.take<double>(nn);   // R1^T (lower)
    double* Wm = c.take<double>(nn);  // W = R2^{-T} (F stays readable for the concurrent solve)
    double* X1 = c.take<double>(nn);
    double* Y = c.take<double>(nn);
    double* Cm = c.take<double>(nn);  // C, then R2^T
    double* tmp = c.take<double>(solver_work_elems(n));
    double* tmp1 = c.take<double>(trsm_work_elems(n));   // the second stream's solve
    const int ld = n;
    fill_i32(s, INFO_SLOTS, 0, h->dinfo);
    std::unique_ptr<LowPrecScope> lp(new LowPrecScope(o.prec));
    // step 1: A = R1^T R1 (stored as the lower factor L1 = R1^T)
    copy_f64(s, n, n, A, lda, nullptr, F, ld);
    potrf_f64(s, n, F, ld, h->dinfo + 0, tmp);
    // step 2: R1^T X1 = B (forward)
    copy_f64(s, n, n, B, ldb, nullptr, X1, ld);
    trsm_f64(s, false, TRI_LOWER, false, n, n, DOp{F, ld, nullptr}, DOut{X1, ld, nullptr, nullptr}, tmp);
    copy_f64(s, n, n, X1, ld, nullptr, Y, ld);
    // step 3: R1 Y = X1 (backward).  Y is needed only by step 9, so from
    // n = LA_MIN this solve runs on the second stream beside steps 4-8 (a
    // latency-bound Cholesky chain), its products on a capped grid.
    const LookAhead* la = n >= LA_MIN ? lookahead(h) : nullptr;
    if (la) {
      FROB_HIP(hipEventRecord(la->ev[0], s));
      FROB_HIP(hipStreamWaitEvent(la->s1, la->ev[0], 0));
      GridCapScope cap(LA_GRID_CAP);
      trsm_f64(la->s1, false, TRI_UPPER, true, n, n, DOp{F, ld, nullptr}, DOut{Y, ld, nullptr, nullptr}, tmp1);
      FROB_HIP(hipEventRecord(la->ev[4], la->s1));
    } else {
      trsm_f64(s, false, TRI_UPPER, true, n, n, DOp{F, ld, nullptr}, DOut{Y, ld, nullptr, nullptr}, tmp);
    }
    // steps 4-5: C = A + step5_sign X1^T X1, lower triangle
    copy_f64(s, n, n, A, lda, nullptr, Cm, ld);
    gemm_f64(s, true, false, n, n, n, step5_sign, DOp{X1, ld, nullptr}, TRI_NONE, DOp{X1, ld, nullptr}, TRI_NONE,
             1.0, DOut{Cm, ld, nullptr, nullptr}, true);
    // step 6: C = R2^T R2
    potrf_f64(s, n, Cm, ld, h->dinfo + 1, tmp);
    // steps 7-8: Re X = C^{-1} = R2^{-1} R2^{-T} = W^T W with W = (R2^T)^{-1} lower
    trtri_f64(s, TRI_LOWER, false, n, DOp{Cm, ld, nullptr}, Wm, ld, tmp);
    gemm_f64(s, true, false, n, n, n, 1.0, DOp{Wm, ld, nullptr}, TRI_UPPER, DOp{Wm, ld, nullptr}, TRI_LOWER, 0.0,
             DOut{Xr, ldx, nullptr, nullptr}, true);
    mirror_lower_f64(s, n, Xr, ldx, 1.0);
    // step 9: Im X = -Y C^{-1}.  The inverse of an HPD M is Hermitian (Im X
    // skew) and that of a complex symmetric M symmetric, so without
    // refinement only the lower triangle is formed and mirrored with the
    // matching sign (half the product).  The mirrored half carries the same
    // forward error, but it no longer matches the factors the way the
    // computed product does: the residual I - M X grows by about kappa(M)
    // times that error, so a refined call (which starts from that residual)
    // forms the whole product.
    if (la) FROB_HIP(hipStreamWaitEvent(s, la->ev[4], 0));
    const bool half = o.refine == 0;
    {
      ProfScope ps(h, PROF_GEMM_NNN, half ? (double)n * (n + 1.0) * n : 2.0 * n * (double)n * n, nullptr,
                   (half ? 20.0 : 24.0) * n * (double)n);
      gemm_f64(s, false, false, n, n, n, -1.0, DOp{Y, ld, nullptr}, TRI_NONE, DOp{Xr, ldx, nullptr}, TRI_NONE, 0.0,
               DOut{Xi, ldx, nullptr, nullptr}, half);
    }
    if (half) mirror_lower_f64(s, n, Xi, ldx, step5_sign < 0.0 ? -1.0 : 1.0);
    lp.reset();
    read_info(h);
    frob_result_t r;
    std::memset(&r, 0, sizeof(r));
    frob_status_t st = FROB_OK;
    if (h->hinfo[0]) { st = FROB_NOT_HPD; r.info = h->hinfo[0]; r.stage = 1; }
    else if (h->hinfo[1]) { st = FROB_NOT_HPD; r.info = h->hinfo[1]; r.stage = 2; }
    if (st == FROB_OK && o.refine > 0)
      st = ns_refine(h, n, A, lda, B, ldb, Xr, Xi, ldx, o.refine, o.refine_tol, o.prec, o.refine_flags, c, &r);
    if (res) *res = r;
    return st;
  });
}

}  // namespace

extern "C" {

frob_status_t frob_inv_hpd(frob_handle_t h, int n, const double* A, int lda, const double* B, int ldb, double* Xr,
                           double* Xi, int ldx, const frob_opts_t* opts, frob_result_t* res) {
  return chol_path(h, n, A, lda, B, ldb, Xr, Xi, ldx, opts, res, -1.0);
}

frob_status_t frob_inv_spd_pair(frob_handle_t h, int n, const double* A, int lda, const double* B, int ldb,
                                double* Xr, double* Xi, int ldx, const frob_opts_t* opts, frob_result_t* res) {
  return chol_path(h, n, A, lda, B, ldb, Xr, Xi, ldx, opts, res, 1.0);
}

frob_status_t frob_solve(frob_handle_t h, int n, int nrhs, const double* A, int lda, const double* B, int ldb,
                         const double* cv, const double* dv, int ldc, double* x, double* y, int ldxy,
                         const frob_opts_t* opts, frob_result_t* res) {
  if (!h || !A || !B || !cv || !dv || !x || !y || bad_dims(n, lda) || ldb < n || nrhs < 1 || ldc < nrhs ||
      ldxy < nrhs)
    return FROB_E_ARG;
  const frob_opts_t o = opts_or_default(opts);
  if (o.shift < FROB_SHIFT_OFF || o.shift > FROB_SHIFT_ON || o.prec != FROB_PREC_F64 || !panel_ok(o.panel))
    return FROB_E_ARG;
  return guarded(h, [&]() -> frob_status_t {
    PanelScope pw(h, o.panel);
    if (o.seed) h->rng = o.seed;
    hipStream_t s = h->stream;
    const size_t nn = (size_t)n * n;
    const int q = 2 * nrhs;
    Carve c = reserve_carve(h, solve_ws(n, nrhs));
    GenWs w = gen_ws_carve(c, n);
    w.h = h;
    double* As = c.take<double>(nn);
    double* Bs = c.take<double>(nn);
    double* Z = c.take<double>((size_t)n * q);   // [x1 y1]
    double* V = c.take<double>((size_t)n * q);   // [y1 x1]
    double* T = c.take<double>((size_t)n * q);   // [x2 y2]
    frob_result_t r;
    std::memset(&r, 0, sizeof(r));

    // (1 + i mu) M (x + iy) = (1 + i mu)(c + id): solve the shifted system with
    // right-hand side c' = c - mu d, d' = mu c + d; the solution is unchanged.
    auto pass = [&](const double* Au, int ldA, const double* Bu, int ldB, double mu) {
      fill_i32(s, INFO_SLOTS, 0, h->dinfo);
      frob_lu_front(s, n, Au, ldA, Bu, ldB, w, h->dinfo, false);
      // step 5: L2 U2 [x1 y1] = P2 [c d]
      copy_f64(s, n, nrhs, cv, ldc, w.p2, Z, q);
      copy_f64(s, n, nrhs, dv, ldc, w.p2, Z + nrhs, q);
      if (mu != 0.0) {
        // rows were gathered by p2 in both halves; rotate them in place
        rotate_f64(s, n, nrhs, mu, Z, q, Z + nrhs, q, Z, q, Z + nrhs, q);
      }
      DOp LU2{w.C, w.ldF, w.p2};
      trsm_f64(s, false, TRI_LOWER_UNIT, false, n, q, LU2, DOut{Z, q, nullptr, nullptr}, w.tmp);
      trsm_f64(s, false, TRI_UPPER, false, n, q, LU2, DOut{Z, q, nullptr, nullptr}, w.tmp);
      // step 6: [x2 y2] = A^{-1} B [y1 x1] = Y [y1 x1]
      copy_f64(s, n, nrhs, Z + nrhs, q, nullptr, V, q);
      copy_f64(s, n, nrhs, Z, q, nullptr, V + nrhs, q);
      gemm_f64(s, false, false, n, q, n, 1.0, DOp{w.Y, w.ld, nullptr}, TRI_NONE, DOp{V, q, nullptr}, TRI_NONE, 0.0,
               DOut{T, q, nullptr, nullptr});
      // step 7: x = x1 + x2, y = y1 - y2
      copy_f64(s, n, nrhs, Z, q, nullptr, x, ldxy);
      axpby_f64(s, n, nrhs, 1.0, T, q, 1.0, x, ldxy);
      copy_f64(s, n, nrhs, Z + nrhs, q, nullptr, y, ldxy);
      axpby_f64(s, n, nrhs, -1.0, T + nrhs, q, 1.0, y, ldxy);
      read_info(h);
    };
    frob_status_t st = FROB_OK;
    bool done = false;
    if (o.shift != FROB_SHIFT_ON) {
      pass(A, lda, B, ldb, 0.0);
      if (h->hinfo[0] == 0) {
        done = true;
        if (h->hinfo[1]) { st = FROB_SINGULAR; r.info = h->hinfo[1]; r.stage = 2; }
      } else if (o.shift == FROB_SHIFT_OFF) {
        done = true;
        st = FROB_SINGULAR; r.info = h->hinfo[0]; r.stage = 1;
      }
    }
    for (int attempt = 0; !done && attempt < 3; ++attempt) {
      const double mu = (o.mu > 0.0 && attempt == 0) ? o.mu : draw_mu(h);
      r.shifts_tried++;
      rotate_f64(s, n, n, mu, A, lda, B, ldb, As, n, Bs, n);
      pass(As, n, Bs, n, mu);
      if (h->hinfo[0] != 0) { r.info = h->hinfo[0]; r.stage = 1; continue; }
      done = true;
      r.mu_used = mu;
      r.info = 0; r.stage = 0;
      if (h->hinfo[1]) { st = FROB_SINGULAR; r.info = h->hinfo[1]; r.stage = 2; }
    }
    if (!done) st = FROB_SINGULAR;
    if (res) *res = r;
    return st;
  });
}

// ------------------------------------------------ FP32-storage twins
// The FP32 operands are widened into FP64 copies at the front of the
// workspace, the FP64 entry point runs on them (its products in opts->prec),
// and the FP64 results are rounded into the caller's FP32 outputs.
frob_status_t frob_inv_general_f32(frob_handle_t h, int n, const float* A, int lda, const float* B, int ldb,
                                   float* Xr, float* Xi, int ldx, const frob_opts_t* opts, frob_result_t* res) {
  if (!h || !A || !B || !Xr || !Xi || bad_dims(n, lda) || ldb < n || ldx < n) return FROB_E_ARG;
  const frob_opts_t o = opts_or_default(opts);
  return guarded(h, [&]() -> frob_status_t {
    hipStream_t s = h->stream;
    const size_t nn = (size_t)n * n;
    const size_t lead = 4 * lead_of(nn);
    double* base = (double*)ws_reserve(h, lead + 256 + general_ws(n, o.refine, o.shift == FROB_SHIFT_COND));
    double *A64 = base, *B64 = base + lead_of(nn) / 8, *Xr64 = base + 2 * lead_of(nn) / 8,
           *Xi64 = base + 3 * lead_of(nn) / 8;
    convert_f32_f64(s, n, n, A, lda, A64, n);
    convert_f32_f64(s, n, n, B, ldb, B64, n);
    frob_status_t st;
    {
      LeadScope ls(lead);
      st = frob_inv_general(h, n, A64, n, B64, n, Xr64, Xi64, n, &o, res);
    }
    if (st == FROB_OK || st == FROB_NO_CONVERGENCE) {
      convert_f64_f32(s, n, n, Xr64, n, Xr, ldx);
      convert_f64_f32(s, n, n, Xi64, n, Xi, ldx);
      FROB_HIP(hipStreamSynchronize(s));
    }
    return st;
  });
}

frob_status_t frob_inv_hpd_f32(frob_handle_t h, int n, const float* A, int lda, const float* B, int ldb, float* Xr,
                               float* Xi, int ldx, const frob_opts_t* opts, frob_result_t* res) {
  if (!h || !A || !B || !Xr || !Xi || bad_dims(n, lda) || ldb < n || ldx < n) return FROB_E_ARG;
  const frob_opts_t o = opts_or_default(opts);
  return guarded(h, [&]() -> frob_status_t {
    hipStream_t s = h->stream;
    const size_t nn = (size_t)n * n;
    const size_t lead = 4 * lead_of(nn);
    double* base = (double*)ws_reserve(h, lead + 256 + hpd_ws(n, o.refine));
    double *A64 = base, *B64 = base + lead_of(nn) / 8, *Xr64 = base + 2 * lead_of(nn) / 8,
           *Xi64 = base + 3 * lead_of(nn) / 8;
    convert_f32_f64(s, n, n, A, lda, A64, n);
    convert_f32_f64(s, n, n, B, ldb, B64, n);
    frob_status_t st;
    {
      LeadScope ls(lead);
      st = frob_inv_hpd(h, n, A64, n, B64, n, Xr64, Xi64, n, &o, res);
    }
    if (st == FROB_OK || st == FROB_NO_CONVERGENCE) {
      convert_f64_f32(s, n, n, Xr64, n, Xr, ldx);
      convert_f64_f32(s, n, n, Xi64, n, Xi, ldx);
      FROB_HIP(hipStreamSynchronize(s));
    }
    return st;
  });
}

frob_status_t frob_solve_f32(frob_handle_t h, int n, int nrhs, const float* A, int lda, const float* B, int ldb,
                             const float* cv, const float* dv, int ldc, float* x, float* y, int ldxy,
                             const frob_opts_t* opts, frob_result_t* res) {
  if (!h || !A || !B || !cv || !dv || !x || !y || bad_dims(n, lda) || ldb < n || nrhs < 1 || ldc < nrhs ||
      ldxy < nrhs)
    return FROB_E_ARG;
  const frob_opts_t o = opts_or_default(opts);
  return guarded(h, [&]() -> frob_status_t {
    hipStream_t s = h->stream;
    const size_t nn = (size_t)n * n, np = (size_t)n * nrhs;
    const size_t lead = 2 * lead_of(nn) + 4 * lead_of(np);
    char* base = (char*)ws_reserve(h, lead + 256 + solve_ws(n, nrhs));
    double* A64 = (double*)base;
    double* B64 = (double*)(base + lead_of(nn));
    double* c64 = (double*)(base + 2 * lead_of(nn));
    double* d64 = (double*)(base + 2 * lead_of(nn) + lead_of(np));
    double* x64 = (double*)(base + 2 * lead_of(nn) + 2 * lead_of(np));
    double* y64 = (double*)(base + 2 * lead_of(nn) + 3 * lead_of(np));
    convert_f32_f64(s, n, n, A, lda, A64, n);
    convert_f32_f64(s, n, n, B, ldb, B64, n);
    convert_f32_f64(s, n, nrhs, cv, ldc, c64, nrhs);
    convert_f32_f64(s, n, nrhs, dv, ldc, d64, nrhs);
    frob_status_t st;
    {
      LeadScope ls(lead);
      st = frob_solve(h, n, nrhs, A64, n, B64, n, c64, d64, nrhs, x64, y64, nrhs, &o, res);
    }
    if (st == FROB_OK) {
      convert_f64_f32(s, n, nrhs, x64, nrhs, x, ldxy);
      convert_f64_f32(s, n, nrhs, y64, nrhs, y, ldxy);
      FROB_HIP(hipStreamSynchronize(s));
    }
    return st;
  });
}

frob_status_t frob_refine(frob_handle_t h, int n, const double* A, int lda, const double* B, int ldb, double* Xr,
                          double* Xi, int ldx, const frob_opts_t* opts, frob_result_t* res) {
  if (!h || !A || !B || !Xr || !Xi || bad_dims(n, lda) || ldb < n || ldx < n) return FROB_E_ARG;
  const frob_opts_t o = opts_or_default(opts);
  if (o.refine < 1 || o.prec < FROB_PREC_F64 || o.prec > FROB_PREC_BF16) return FROB_E_ARG;
  return guarded(h, [&]() -> frob_status_t {
    Carve c((char*)ws_reserve(h, ns_ws_bytes(n, o.refine)));
    frob_result_t r;
    std::memset(&r, 0, sizeof(r));
    LowPrecScope fp64(LP_NONE);   // the residual is formed in FP64; ns_refine scopes the correction
    const frob_status_t st = ns_refine(h, n, A, lda, B, ldb, Xr, Xi, ldx, o.refine, o.refine_tol, o.prec,
                                       o.refine_flags, c, &r);
    if (res) *res = r;
    return st;
  });
}

// ------------------------------------------------ Newton iterations (Section 5)
void frob_default_newton_opts(frob_newton_opts_t* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-3;
  o->max_iter = 100;
  frob_default_opts(&o->inv);
}

namespace {

// workspace of one inversion of the iteration, beyond the iterate's
size_t newton_inv_ws(int n, const frob_newton_opts_t& o) {
  return o.inverse == FROB_NEWTON_COMPLEX_LU ? cinv_lu_ws(n)
                                             : general_ws(n, o.inv.refine, o.inv.shift == FROB_SHIFT_COND);
}

frob_newton_opts_t newton_opts_or_default(const frob_newton_opts_t* o) {
  frob_newton_opts_t d;
  frob_default_newton_opts(&d);
  if (!o) return d;
  frob_newton_opts_t r = *o;
  if (!(r.tol > 0.0)) r.tol = d.tol;
  if (r.max_iter <= 0) r.max_iter = d.max_iter;
  frob_opts_t zero;
  std::memset(&zero, 0, sizeof(zero));
  if (std::memcmp(&r.inv, &zero, sizeof(zero)) == 0) r.inv = d.inv;   // zeroed: the inversion's defaults
  return r;
}

// The iteration X <- (X + op(X^{-1})) / 2 on X (n x n, ld n, at the front of
// the workspace), each inverse by frob_inv_general (or the complex-LU
// baseline) into I (ld n).  `lead` is
// the size of the region holding X, I and the two max-norm words.
frob_status_t newton_iterate(frob_handle* h, int n, double* Xr, double* Xi, double* Ir, double* Ii,
                             unsigned long long* maxes, size_t lead, bool herm, const frob_newton_opts_t& o,
                             frob_newton_result_t* res) {
  frob_newton_result_t r;
  std::memset(&r, 0, sizeof(r));
  frob_status_t st = FROB_OK;
  unsigned long long hm[2];
  for (int k = 0; k < o.max_iter; ++k) {
    {
      LeadScope ls(lead);
      st = o.inverse == FROB_NEWTON_COMPLEX_LU ? frob_cinv_lu(h, n, Xr, Xi, n, Ir, Ii, n, 1, &r.inv)
                                               : frob_inv_general(h, n, Xr, n, Xi, n, Ir, Ii, n, &o.inv, &r.inv);
    }
    if (st != FROB_OK && st != FROB_NO_CONVERGENCE) break;
    st = FROB_OK;
    newton_step(h->stream, n, Xr, Xi, n, Ir, Ii, n, herm, maxes);
    FROB_HIP(hipMemcpyAsync(hm, maxes, sizeof(hm), hipMemcpyDeviceToHost, h->stream));
    FROB_HIP(hipStreamSynchronize(h->stream));
    double d, x;
    std::memcpy(&d, &hm[0], sizeof(d));
    std::memcpy(&x, &hm[1], sizeof(x));
    r.iterations = k + 1;
    r.last_change = x > 0.0 ? d / x : 0.0;
    if (r.last_change <= o.tol) break;
  }
  if (res) *res = r;
  return st;
}

}  // namespace

frob_status_t frob_sign(frob_handle_t h, int n, const double* Xr, const double* Xi, int ldx, double* Sr, double* Si,
                        int lds, const frob_newton_opts_t* opts, frob_newton_result_t* res) {
  if (!h || !Xr || !Xi || !Sr || !Si || bad_dims(n, ldx) || lds < n) return FROB_E_ARG;
  const frob_newton_opts_t o = newton_opts_or_default(opts);
  if (o.inverse != FROB_NEWTON_FROBENIUS && o.inverse != FROB_NEWTON_COMPLEX_LU) return FROB_E_ARG;
  return guarded(h, [&]() -> frob_status_t {
    hipStream_t s = h->stream;
    const size_t nn = (size_t)n * n;
    const size_t lead = 4 * lead_of(nn) + 256;
    char* base = (char*)ws_reserve(h, lead + 256 + newton_inv_ws(n, o));
    double* Wr = (double*)base;
    double* Wi = (double*)(base + lead_of(nn));
    double* Ir = (double*)(base + 2 * lead_of(nn));
    double* Ii = (double*)(base + 3 * lead_of(nn));
    unsigned long long* maxes = (unsigned long long*)(base + 4 * lead_of(nn));
    copy_f64(s, n, n, Xr, ldx, nullptr, Wr, n);
    copy_f64(s, n, n, Xi, ldx, nullptr, Wi, n);
    const frob_status_t st = newton_iterate(h, n, Wr, Wi, Ir, Ii, maxes, lead, false, o, res);
    if (st == FROB_OK) {
      copy_f64(s, n, n, Wr, n, nullptr, Sr, lds);
      copy_f64(s, n, n, Wi, n, nullptr, Si, lds);
      FROB_HIP(hipStreamSynchronize(s));
    }
    return st;
  });
}

frob_status_t frob_polar(frob_handle_t h, int n, const double* Xr, const double* Xi, int ldx, double* Qr, double* Qi,
                         int ldq, double* Pr, double* Pi, int ldp, const frob_newton_opts_t* opts,
                         frob_newton_result_t* res) {
  if (!h || !Xr || !Xi || !Qr || !Qi || !Pr || !Pi || bad_dims(n, ldx) || ldq < n || ldp < n) return FROB_E_ARG;
  const frob_newton_opts_t o = newton_opts_or_default(opts);
  if (o.inverse != FROB_NEWTON_FROBENIUS && o.inverse != FROB_NEWTON_COMPLEX_LU) return FROB_E_ARG;
  return guarded(h, [&]() -> frob_status_t {
    hipStream_t s = h->stream;
    const size_t nn = (size_t)n * n;
    const size_t lead = 4 * lead_of(nn) + 256;
    char* base = (char*)ws_reserve(h, lead + 256 + newton_inv_ws(n, o));
    double* Wr = (double*)base;
    double* Wi = (double*)(base + lead_of(nn));
    double* Ir = (double*)(base + 2 * lead_of(nn));
    double* Ii = (double*)(base + 3 * lead_of(nn));
    unsigned long long* maxes = (unsigned long long*)(base + 4 * lead_of(nn));
    copy_f64(s, n, n, Xr, ldx, nullptr, Wr, n);
    copy_f64(s, n, n, Xi, ldx, nullptr, Wi, n);
    const frob_status_t st = newton_iterate(h, n, Wr, Wi, Ir, Ii, maxes, lead, true, o, res);
    if (st == FROB_OK) {
      copy_f64(s, n, n, Wr, n, nullptr, Qr, ldq);
      copy_f64(s, n, n, Wi, n, nullptr, Qi, ldq);
      // P = Q^H X
      gemm_z64(s, OP_C, OP_N, n, n, n, 1.0, ZOp{Wr, Wi, n, nullptr}, TRI_NONE, ZOp{Xr, Xi, ldx, nullptr}, TRI_NONE,
               0.0, ZOut{Pr, Pi, ldp, nullptr, nullptr});
      FROB_HIP(hipStreamSynchronize(s));
    }
    return st;
  });
}

namespace {

frob_status_t sylvester_impl(frob_handle* h, int p, int q, const double* Ar, const double* Ai, int lda,
                             const double* Br, const double* Bi, int ldb, bool lyap, const double* Cr,
                             const double* Ci, int ldc, double* Yr, double* Yi, int ldy, const frob_newton_opts_t& o,
                             frob_newton_result_t* res) {
  hipStream_t s = h->stream;
  const int N = p + q;
  const size_t nn = (size_t)N * N;
  const size_t lead = 4 * lead_of(nn) + 256;
  char* base = (char*)ws_reserve(h, lead + 256 + newton_inv_ws(N, o));
  double* Wr = (double*)base;
  double* Wi = (double*)(base + lead_of(nn));
  double* Ir = (double*)(base + 2 * lead_of(nn));
  double* Ii = (double*)(base + 3 * lead_of(nn));
  unsigned long long* maxes = (unsigned long long*)(base + 4 * lead_of(nn));
  sylvester_assemble(s, p, q, Ar, Ai, lda, Br, Bi, ldb, lyap, Cr, Ci, ldc, Wr, Wi);
  const frob_status_t st = newton_iterate(h, N, Wr, Wi, Ir, Ii, maxes, lead, false, o, res);
  if (st == FROB_OK) {
    sylvester_extract(s, p, q, Wr, Wi, Yr, Yi, ldy);
    FROB_HIP(hipStreamSynchronize(s));
  }
  return st;
}

}  // namespace

frob_status_t frob_sylvester(frob_handle_t h, int p, int q, const double* Ar, const double* Ai, int lda,
                             const double* Br, const double* Bi, int ldb, const double* Cr, const double* Ci, int ldc,
                             double* Yr, double* Yi, int ldy, const frob_newton_opts_t* opts,
                             frob_newton_result_t* res) {
  if (!h || !Ar || !Ai || !Br || !Bi || !Cr || !Ci || !Yr || !Yi || p < 1 || q < 1 || p + q > FROB_MAX_N ||
      lda < p || ldb < q || ldc < q || ldy < q)
    return FROB_E_ARG;
  const frob_newton_opts_t o = newton_opts_or_default(opts);
  if (o.inverse != FROB_NEWTON_FROBENIUS && o.inverse != FROB_NEWTON_COMPLEX_LU) return FROB_E_ARG;
  return guarded(h, [&]() -> frob_status_t {
    return sylvester_impl(h, p, q, Ar, Ai, lda, Br, Bi, ldb, false, Cr, Ci, ldc, Yr, Yi, ldy, o, res);
  });
}

frob_status_t frob_lyapunov(frob_handle_t h, int p, const double* Ar, const double* Ai, int lda, const double* Cr,
                            const double* Ci, int ldc, double* Yr, double* Yi, int ldy, const frob_newton_opts_t* opts,
                            frob_newton_result_t* res) {
  if (!h || !Ar || !Ai || !Cr || !Ci || !Yr || !Yi || p < 1 || 2 * p > FROB_MAX_N || lda < p || ldc < p || ldy < p)
    return FROB_E_ARG;
  const frob_newton_opts_t o = newton_opts_or_default(opts);
  if (o.inverse != FROB_NEWTON_FROBENIUS && o.inverse != FROB_NEWTON_COMPLEX_LU) return FROB_E_ARG;
  return guarded(h, [&]() -> frob_status_t {
    return sylvester_impl(h, p, p, Ar, Ai, lda, Ar, Ai, lda, true, Cr, Ci, ldc, Yr, Yi, ldy, o, res);
  });
}

// ------------------------------------- iterated quadratic extensions (Section 2.4)
namespace {

// Elements of F_k^{n x n} (xi_j^2 = -tau_j, j < k) are 2^k contiguous real
// planes of n x n (ld n), plane p the coefficient of xi^alpha with
// alpha_j = bit j of p; the top generator xi_k splits an element into its
// low and high halves (eq. (iterquadmat2)).
struct Tower {
  frob_handle* h;
  hipStream_t s;
  int n;
  const double* tau;        // tau[0 .. m)
  frob_opts_t o;
  size_t lead;              // bytes of the region holding every tower buffer
  frob_result_t r;          // result of the last base inversion
  size_t nn() const { return (size_t)n * n; }
};

// temporaries (doubles) of a product / an inversion at level k
size_t tower_mul_tmp(int k, size_t nn) { return k == 0 ? 0 : 3 * ((size_t)1 << (k - 1)) * nn + tower_mul_tmp(k - 1, nn); }
size_t tower_inv_tmp(int k, size_t nn) {
  if (k == 1) return nn;   // the scaled imaginary part
  return 3 * ((size_t)1 << (k - 1)) * nn + std::max(tower_inv_tmp(k - 1, nn), tower_mul_tmp(k - 1, nn));
}

// Z = X Y at level k: Gauss's three products per level (Theorem 2.10 (i))
void tower_mul(Tower& t, int k, const double* X, const double* Y, double* Z, double* tmp) {
  const int n = t.n;
  if (k == 0) {
    gemm_f64(t.s, false, false, n, n, n, 1.0, DOp{X, n, nullptr}, TRI_NONE, DOp{Y, n, nullptr}, TRI_NONE, 0.0,
             DOut{Z, n, nullptr, nullptr});
    return;
  }
  const size_t half = ((size_t)1 << (k - 1)) * t.nn();
  double *S = tmp, *U = tmp + half, *P3 = tmp + 2 * half, *rest = tmp + 3 * half;
  tower_mul(t, k - 1, X, Y, Z, rest);                       // P1 = X0 Y0  (in Z0)
  tower_mul(t, k - 1, X + half, Y + half, Z + half, rest);  // P2 = X1 Y1  (in Z1)
  lincomb_f64(t.s, 1, (int)half, 1.0, X, (int)half, 1.0, X + half, (int)half, S, (int)half);
  lincomb_f64(t.s, 1, (int)half, 1.0, Y, (int)half, 1.0, Y + half, (int)half, U, (int)half);
  tower_mul(t, k - 1, S, U, P3, rest);                      // P3 = (X0 + X1)(Y0 + Y1)
  gauss3_combine_f64(t.s, (long long)half, Z, Z + half, P3, t.tau[k - 1]);
}

// Xi = X^{-1} at level k >= 1: Algorithm 1 over x^2 + tau_k (eq. (lem:inverse)):
//   X1 = A^{-1}, X2 = X1 B, X3 = A + tau B X2, X4 = X3^{-1}, X5 = X2 X4,
//   X^{-1} = X4 - xi_k X5;  at k = 1 the inversion over C with xi = i sqrt(tau).
frob_status_t tower_inv(Tower& t, int k, const double* X, double* Xi, double* tmp) {
  const int n = t.n;
  const size_t nn = t.nn();
  if (k == 1) {
    const double sq = std::sqrt(t.tau[0]);
    const double* B = X + nn;
    if (sq != 1.0) {
      lincomb_f64(t.s, 1, (int)nn, sq, X + nn, (int)nn, 0.0, X + nn, (int)nn, tmp, (int)nn);
      B = tmp;
    }
    frob_status_t st;
    {
      LeadScope ls(t.lead);
      st = frob_inv_general(t.h, n, X, n, B, n, Xi, Xi + nn, n, &t.o, &t.r);
    }
    if (st == FROB_OK && sq != 1.0) axpby_f64(t.s, 1, (int)nn, 1.0 / sq, Xi + nn, (int)nn, 0.0, Xi + nn, (int)nn);
    return st;
  }
  const size_t half = ((size_t)1 << (k - 1)) * nn;
  const double *A = X, *B = X + half;
  double *X1 = tmp, *X2 = tmp + half, *X3 = tmp + 2 * half, *rest = tmp + 3 * half;
  frob_status_t st = tower_inv(t, k - 1, A, X1, rest);
  if (st != FROB_OK) return st;
  tower_mul(t, k - 1, X1, B, X2, rest);
  tower_mul(t, k - 1, B, X2, X3, rest);
  lincomb_f64(t.s, 1, (int)half, 1.0, A, (int)half, t.tau[k - 1], X3, (int)half, X3, (int)half);
  st = tower_inv(t, k - 1, X3, Xi, rest);                  // X4 -> low half
  if (st != FROB_OK) return st;
  tower_mul(t, k - 1, X2, Xi, Xi + half, rest);             // X5 -> high half
  axpby_f64(t.s, 1, (int)half, -1.0, Xi + half, (int)half, 0.0, Xi + half, (int)half);
  return FROB_OK;
}

}  // namespace

frob_status_t frob_inv_tower(frob_handle_t h, int m, int n, const double* tau, const double* const* C, int ldc,
                             double* const* X, int ldx, const frob_opts_t* opts, frob_result_t* res) {
  if (!h || m < 1 || m > 4 || !tau || !C || !X || bad_dims(n, ldc) || ldx < n) return FROB_E_ARG;
  const int P = 1 << m;
  for (int k = 0; k < m; ++k)
    if (!(tau[k] > 0.0) || !std::isfinite(tau[k])) return FROB_E_ARG;
  for (int p = 0; p < P; ++p)
    if (!C[p] || !X[p]) return FROB_E_ARG;
  if ((size_t)P * n * n > ((size_t)1 << 31)) return FROB_E_ARG;   // plane-flat element counts fit in int
  const frob_opts_t o = opts_or_default(opts);
  return guarded(h, [&]() -> frob_status_t {
    Tower t{h, h->stream, n, tau, o, 0, {}};
    const size_t nn = t.nn();
    const size_t doubles = 2 * (size_t)P * nn + tower_inv_tmp(m, nn);
    t.lead = lead_of(doubles);
    double* base = (double*)ws_reserve(h, t.lead + 256 + general_ws(n, o.refine, o.shift == FROB_SHIFT_COND));
    double* Xin = base;
    double* Xout = base + (size_t)P * nn;
    double* tmp = Xout + (size_t)P * nn;
    for (int p = 0; p < P; ++p) copy_f64(t.s, n, n, C[p], ldc, nullptr, Xin + (size_t)p * nn, n);
    const frob_status_t st = tower_inv(t, m, Xin, Xout, tmp);
    if (st == FROB_OK) {
      for (int p = 0; p < P; ++p) copy_f64(t.s, n, n, Xout + (size_t)p * nn, n, nullptr, X[p], ldx);
      FROB_HIP(hipStreamSynchronize(t.s));
    }
    if (res) *res = t.r;
    return st;
  });
}

frob_status_t frob_profile_enable(frob_handle_t h, int on) {
  if (!h) return FROB_E_ARG;
  h->prof = on ? 1 : 0;
  for (int k = 0; k < 16; ++k) { h->prof_ms[k] = 0; h->prof_flops[k] = 0; h->prof_bytes[k] = 0; h->prof_count[k] = 0; }
  return FROB_OK;
}

frob_status_t frob_profile_read(frob_handle_t h, int cls, long long* launches, double* total_ms, double* flops,
                                double* bytes) {
  if (!h || cls < 0 || cls >= 16) return FROB_E_ARG;
  return guarded(h, [&]() -> frob_status_t {
    prof_resolve(h);
    if (launches) *launches = h->prof_count[cls];
    if (total_ms) *total_ms = h->prof_ms[cls];
    if (flops) *flops = h->prof_flops[cls];
    if (bytes) *bytes = h->prof_bytes[cls];
    return FROB_OK;
  });
}

const char* frob_status_string(frob_status_t s) {
  switch (s) {
    case FROB_OK: return "FROB_OK";
    case FROB_SINGULAR: return "FROB_SINGULAR";
    case FROB_NOT_HPD: return "FROB_NOT_HPD";
    case FROB_NO_CONVERGENCE: return "FROB_NO_CONVERGENCE";
    case FROB_E_ARG: return "FROB_E_ARG";
    case FROB_E_ALLOC: return "FROB_E_ALLOC";
    case FROB_E_HIP: return "FROB_E_HIP";
    case FROB_E_INTERNAL: return "FROB_E_INTERNAL";
    case FROB_E_CAPTURE: return "FROB_E_CAPTURE";
  }
  return "FROB_UNKNOWN";
}

}  // extern "C"

// Bytes an enclosing call keeps ahead of the workspace on this thread (used
// by the complex baselines when a Newton driver calls them).
size_t frob::ws_lead() { return t_lead_bytes; }
