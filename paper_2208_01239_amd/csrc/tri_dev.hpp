// tri_dev.hpp -- device building block shared by the small triangular solve
// kernels: substitution with a lower triangle of order <= 64 held in LDS,
// applied to 64 right-hand sides at once by 256 threads.
//
// Thread tid works on right-hand side c = tid / 4 and owns its rows
// i = 4 m + g (g = tid % 4, m = 0 .. 15) in registers.  Rows are processed in
// blocks of four, one row per lane of the quad that shares c: the dependent
// part of a block is four quad broadcasts (DPP), the update of the remaining
// rows is independent FMAs whose LDS operands are the same for every c
// (broadcast reads).  An upper triangle is handled by the caller by reversing
// the index order, which turns it into a lower one.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace frob {

// f(integral_constant<int, I>) for I = B .. E-1, expanded at compile time, so
// that register-array indices inside f are constants even where the
// unroller would give up (large bodies) and fall back to indexed registers.
template <int B, int E>
struct StaticFor {
  template <class F>
  __device__ __forceinline__ static void run(const F& f) {
    f(std::integral_constant<int, B>{});
    StaticFor<B + 1, E>::run(f);
  }
};
template <int E>
struct StaticFor<E, E> {
  template <class F>
  __device__ __forceinline__ static void run(const F&) {}
};

// value held by lane (lane & ~3) + Q of the calling lane's quad
template <int Q>
__device__ __forceinline__ double quad_bcast(double v) {
  constexpr int ctrl = Q | (Q << 2) | (Q << 4) | (Q << 6);
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// A zero the compiler cannot see through.  Passed as `bfirst` it keeps one
// runtime test per block of the solve below, which stops the scheduler from
// hoisting every block's LDS reads to the top (256 VGPRs and spills).
__device__ __forceinline__ int opaque_zero() {
  int z;
  asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return z;
}

// Solve L x = b in place (x holds b on entry).  L: (4 NBLK) x (4 NBLK) lower
// triangle in LDS with row stride LDL (64 x 64 by default); rd[i] = 1 / L(i, i).
// Blocks before `bfirst` are skipped (their rows of x are zero for every lane
// of the wave and stay zero).
template <int LDL, int NBLK>
__device__ __forceinline__ void quad_lower_solve(const double* __restrict__ L, const double* __restrict__ rd,
                                                 double (&x)[NBLK], int g, int bfirst) {
  StaticFor<0, NBLK>::run([&](auto bc) {
    constexpr int b = decltype(bc)::value;
    if (b < bfirst) return;  // uniform per wave
    double xb = x[b];
    const double* Lr = L + (4 * b + g) * LDL + 4 * b;
    xb = (g == 0) ? xb * rd[4 * b] : xb;
    const double x0 = quad_bcast<0>(xb);
    if (g > 0) xb -= Lr[0] * x0;
    xb = (g == 1) ? xb * rd[4 * b + 1] : xb;
    const double x1 = quad_bcast<1>(xb);
    if (g > 1) xb -= Lr[1] * x1;
    xb = (g == 2) ? xb * rd[4 * b + 2] : xb;
    const double x2 = quad_bcast<2>(xb);
    if (g > 2) xb -= Lr[2] * x2;
    xb = (g == 3) ? xb * rd[4 * b + 3] : xb;
    const double x3 = quad_bcast<3>(xb);
    x[b] = xb;
    // rows below: one sweep per solved row, so consecutive FMAs are
    // independent (different rows) and pipeline instead of forming a chain
    const double xs[4] = {x0, x1, x2, x3};
    StaticFor<0, 4>::run([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      StaticFor<b + 1, NBLK>::run([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        x[m] = fma(-L[(4 * m + g) * LDL + 4 * b + q], xs[q], x[m]);
      });
    });
  });
}

}  // namespace frob
