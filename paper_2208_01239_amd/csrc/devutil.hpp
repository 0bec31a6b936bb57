// devutil.hpp -- small device helpers shared by the factorization kernels.
#pragma once

#include <climits>

#include "common.hpp"

namespace frob {

// Largest |v| of the wave with the lowest logical row on ties.  Returns the
// winning lane (or -1 if no lane has a candidate, e.g. an all-NaN column).
__device__ __forceinline__ int wave_argmax(double best, int bq, double& wbest, int& wq) {
  double m = best;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  wbest = m;
  if (!(m >= 0.0)) { wq = INT_MAX; return -1; }
  const unsigned long long tied = __ballot(best == m && bq != INT_MAX);
  if (__popcll(tied) == 1) {
    const int lane = __ffsll((long long)tied) - 1;
    wq = __builtin_amdgcn_readlane(bq, lane);
    return lane;
  }
  // several lanes hold the same value: lowest logical row wins
  int q = (best == m) ? bq : INT_MAX;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) q = min(q, __shfl_xor(q, off));
  wq = q;
  const unsigned long long own = __ballot(bq == q && best == m);
  return __ffsll((long long)own) - 1;
}

}  // namespace frob
