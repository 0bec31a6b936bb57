// handle.hpp -- the library handle and workspace carving (host side).
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/frobinv.h"
#include "common.hpp"
#include "internal.hpp"

// Optional per-kernel-class timing: HIP events recorded on the handle's stream
// around selected launches, resolved after the call's final synchronization.
struct frob_prof_pending {
  hipEvent_t e0, e1;
  int cls;
  double flops, bytes;
};

struct frob_handle {
  int device = 0;
  hipStream_t stream = nullptr;  // stream all work is enqueued on (null stream by default)
  void* ws = nullptr;            // grow-only device workspace
  size_t ws_cap = 0;
  bool ws_captured = false;      // a captured launch references ws: never free it, retire it on growth
  std::vector<void*> ws_retired; // retired workspaces, freed by frob_destroy
  int* dinfo = nullptr;          // device status words (factorization info)
  int* hinfo = nullptr;          // pinned host copy
  double* dnorm = nullptr;       // device scalar for residual norms
  double* hnorm = nullptr;       // pinned host copy
  uint64_t rng = 0;              // splitmix64 state for the shift mu
  int prof = 0;                  // profiling enabled
  std::vector<frob_prof_pending> pending;
  std::vector<hipEvent_t> pool;
  int batch_nb[2][2][4] = {{{16, 16, 16, 16}, {16, 16, 16, 16}}, {{16, 16, 16, 16}, {16, 16, 16, 16}}};
                                 // batched panel width [FP64/FP32][general/HPD][order class]
  frob::LookAhead la;            // second stream and events of the look-ahead LU (created on first use)
  double prof_ms[16] = {0};
  double prof_flops[16] = {0};
  double prof_bytes[16] = {0};
  long long prof_count[16] = {0};
};

namespace frob {

constexpr int INFO_SLOTS = 8;
constexpr int FROB_MAX_N = 16384;

// Bump allocator over the handle workspace; with a null base it only measures.
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(char* b) : base(b) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// scratch for the triangular solves / inverses / factorizations of order n
size_t solver_work_elems(int n);

// kernel classes for frob_profile_read
enum { PROF_GEMM_NNN = 0, PROF_BATCHED = 4, PROF_ADJOINT = 5, PROF_TRAIL_GEMM = 6 };
// Record an event pair around the launches issued between begin and end, on
// stream `s` (default: the handle's stream).
struct ProfScope {
  frob_handle* h;
  int cls;
  double flops, bytes;
  hipStream_t st;
  hipEvent_t e0 = nullptr;
  ProfScope(frob_handle* hh, int c, double fl, hipStream_t s = nullptr, double by = 0.0);
  ~ProfScope();
};
void prof_resolve(frob_handle* h);

// thrown when a call needs more workspace while its stream is being captured
struct CaptureGrowth {};

uint64_t splitmix64(uint64_t& x);
double draw_mu(frob_handle* h);
// Bytes an enclosing call keeps at the front of the workspace (0 outside one).
size_t ws_lead();
// Workspace bytes of frob_cinv_lu at order n.
size_t cinv_lu_ws(int n);
// The handle's workspace, grown to at least `bytes`.  Growth while the
// handle's stream is being captured throws CaptureGrowth (nothing is freed or
// allocated then); a workspace that a captured launch references is retired,
// not freed, when it is outgrown (mark_ws_captured).
void* ws_reserve(frob_handle* h, size_t bytes);
// Records that the handle's stream is being captured, if it is; returns whether.
bool mark_ws_captured(frob_handle* h);
// Resolves, once per device, the device address of the no-allocation batched
// entry point's scratch array (the device must be current).
void batched_scratch_init(int device);
// the handle's look-ahead stream and events, created on first use (null handle: none)
const LookAhead* lookahead(frob_handle* h);
void read_info(frob_handle* h);

// Newton-Schulz refinement X <- X + X (I - M X) with complex products done by
// Gauss's three-real-multiplication scheme (Proposition 2.2, tau = 1); the
// residual is formed in FP64, the correction product in precision `prec`.
size_t ns_ws_bytes(int n, int steps);
frob_status_t ns_refine(frob_handle* h, int n, const double* A, int lda, const double* B, int ldb, double* Xr,
                        double* Xi, int ldx, int max_steps, double tol, int prec, int flags, Carve& c,
                        frob_result_t* r);

}  // namespace frob
