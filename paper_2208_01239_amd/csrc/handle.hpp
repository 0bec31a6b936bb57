// handle.hpp -- the library handle and workspace carving (host side).
#pragma once

#include <cstdint>

#include "../../include/frobinv.h"
#include "common.hpp"

struct frob_handle {
  int device = 0;
  hipStream_t stream = nullptr;  // stream all work is enqueued on (null stream by default)
  void* ws = nullptr;            // grow-only device workspace
  size_t ws_cap = 0;
  int* dinfo = nullptr;          // device status words (factorization info)
  int* hinfo = nullptr;          // pinned host copy
  uint64_t rng = 0;              // splitmix64 state for the shift mu
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

// scratch for the triangular inverse recursion: (n/2 + 64) rows of n entries
inline int tmp_ld(int n) { return n; }
inline size_t tmp_elems(int n) { return (size_t)(n / 2 + 64) * (size_t)n + 64; }

uint64_t splitmix64(uint64_t& x);
double draw_mu(frob_handle* h);
void* ws_reserve(frob_handle* h, size_t bytes);
void read_info(frob_handle* h);

// Newton-Schulz refinement X <- X + X (I - M X) with complex products done by
// Gauss's three-real-multiplication scheme (Proposition 2.2, tau = 1).
size_t ns_ws_bytes(int n, int steps);
frob_status_t ns_refine(frob_handle* h, int n, const double* A, int lda, const double* B, int ldb, double* Xr,
                        double* Xi, int ldx, int steps, Carve& c, frob_result_t* r);

}  // namespace frob
