// common.hpp -- shared definitions for the gfx950 kernels and host drivers of
// libfrobinv (Frobenius inversion of complex matrices with real operations).
//
// Storage convention used by every kernel: dense row-major matrices with an
// explicit leading dimension.  An operand may carry a row-index array `rows`:
// its logical row i then lives in physical row rows[i].  This is how the LU
// factorizations pivot without moving data: partial pivoting permutes the
// index array only, and every consumer of the factors reads through it.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

namespace frob {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

struct HipError : std::runtime_error {
  hipError_t code;
  HipError(hipError_t c, const char* what) : std::runtime_error(what), code(c) {}
};

#define FROB_HIP(call)                                                                          \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      throw ::frob::HipError(e_, (std::string(#call) + ": " + hipGetErrorString(e_)).c_str()); \
  } while (0)

#define FROB_LAUNCH_CHECK() FROB_HIP(hipGetLastError())

// Triangular interpretation of a GEMM operand in its logical (op-applied)
// coordinates.  Entries outside the triangle read as zero; a unit triangle
// reads its diagonal as one.  Lets one GEMM kernel act as trmm / trsm step.
enum Tri : int { TRI_NONE = 0, TRI_LOWER = 1, TRI_LOWER_UNIT = 2, TRI_UPPER = 3, TRI_UPPER_UNIT = 4 };

// Real FP64 operand: element (i, k) of the stored (non-transposed) matrix is
// p[(rows ? rows[i] : i) * ld + k].  `p` already includes any column offset,
// and the row offset when `rows` is null.
struct DOp {
  const double* p;
  int ld;
  const int* rows;
};
struct DOut {
  double* p;
  int ld;
  const int* rows;   // output row indirection (may be null)
  const int* cols;   // output column scatter: logical column j -> cols[j] (may be null)
};

// Planar complex FP64 operand (separate real and imaginary arrays, same ld).
struct ZOp {
  const double* re;
  const double* im;
  int ld;
  const int* rows;
};
struct ZOut {
  double* re;
  double* im;
  int ld;
  const int* rows;
  const int* cols;
};

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

}  // namespace frob
