// newton.hip -- elementwise kernels of the Newton iterations built on the
// inversion (matrix sign, polar factor, Sylvester and Lyapunov equations).
//
//   sign:  X_{k+1} = (X_k + X_k^{-1}) / 2      (Section 5.3, eq. (iter))
//   polar: X_{k+1} = (X_k + X_k^{-H}) / 2      (Section 5.5, eq. (iter2))
//
// One kernel forms the new iterate in place and the two max norms of the
// stopping rule (eq. (maxnorm), the largest |entry| over both planes): of the
// change and of the new iterate.  Both are non-negative, so their IEEE bit
// patterns order like the values and one 64-bit atomic maximum per wave
// combines them.  The conjugate transpose of the polar step is read through
// a 32 x 32 LDS tile so that both the reads and the writes are coalesced.
#include "common.hpp"
#include "internal.hpp"

namespace frob {

namespace {

constexpr int NT = 32;   // tile side
constexpr int NR = 8;    // thread rows per tile (32 x 8 threads, 4 rows each)

__device__ __forceinline__ void wave_max_atomic(double v, unsigned long long* dst) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  if ((threadIdx.x + NT * threadIdx.y) % 64 == 0) atomicMax(dst, (unsigned long long)__double_as_longlong(v));
}

__global__ __launch_bounds__(NT * NR) void k_newton_step(int n, double* __restrict__ Xr, double* __restrict__ Xi,
                                                         int ldx, const double* __restrict__ Ir,
                                                         const double* __restrict__ Ii, int ldi, int herm,
                                                         unsigned long long* maxes) {
  __shared__ double tr[NT][NT + 1], ti[NT][NT + 1];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int bx = blockIdx.x * NT, by = blockIdx.y * NT;   // tile columns / rows of the iterate
  if (herm) {
    // (I^H)[i][j] = conj(I[j][i]): stage rows bx.. of I, columns by..
#pragma unroll
    for (int k = 0; k < NT / NR; ++k) {
      const int jj = ty + NR * k, r = bx + jj, c = by + tx;
      const bool ok = r < n && c < n;
      tr[jj][tx] = ok ? Ir[(long long)r * ldi + c] : 0.0;
      ti[jj][tx] = ok ? Ii[(long long)r * ldi + c] : 0.0;
    }
    __syncthreads();
  }
  double dmax = 0.0, xmax = 0.0;
#pragma unroll
  for (int k = 0; k < NT / NR; ++k) {
    const int ii = ty + NR * k, i = by + ii, j = bx + tx;
    if (i < n && j < n) {
      double vr, vi;
      if (herm) {
        vr = tr[tx][ii];
        vi = -ti[tx][ii];
      } else {
        vr = Ir[(long long)i * ldi + j];
        vi = Ii[(long long)i * ldi + j];
      }
      double* pr = Xr + (long long)i * ldx + j;
      double* pi = Xi + (long long)i * ldx + j;
      const double xr = *pr, xi = *pi;
      const double nr = 0.5 * (xr + vr), ni = 0.5 * (xi + vi);
      *pr = nr;
      *pi = ni;
      dmax = fmax(dmax, fmax(fabs(nr - xr), fabs(ni - xi)));
      xmax = fmax(xmax, fmax(fabs(nr), fabs(ni)));
    }
  }
  wave_max_atomic(dmax, maxes);
  wave_max_atomic(xmax, maxes + 1);
}

__global__ void k_zero_u64(unsigned long long* p) {
  if (threadIdx.x < 2) p[threadIdx.x] = 0ull;
}

// X = [[A, -C], [0, -B]] of order N = p + q (B = A^H when lyap)
__global__ void k_sylv_assemble(int p, int q, const double* __restrict__ Ar, const double* __restrict__ Ai, int lda,
                                const double* __restrict__ Br, const double* __restrict__ Bi, int ldb, int lyap,
                                const double* __restrict__ Cr, const double* __restrict__ Ci, int ldc,
                                double* __restrict__ Xr, double* __restrict__ Xi) {
  const int N = p + q;
  const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double vr = 0.0, vi = 0.0;
  if (i < p && j < p) {
    vr = Ar[(long long)i * lda + j];
    vi = Ai[(long long)i * lda + j];
  } else if (i < p) {
    vr = -Cr[(long long)i * ldc + (j - p)];
    vi = -Ci[(long long)i * ldc + (j - p)];
  } else if (j >= p) {
    const int r = i - p, c = j - p;
    if (lyap) {   // -(A^H)[r][c] = -conj(A[c][r])
      vr = -Ar[(long long)c * lda + r];
      vi = Ai[(long long)c * lda + r];
    } else {
      vr = -Br[(long long)r * ldb + c];
      vi = -Bi[(long long)r * ldb + c];
    }
  }
  Xr[(long long)i * N + j] = vr;
  Xi[(long long)i * N + j] = vi;
}

// Y = -(1/2) S[0:p, p:p+q]
__global__ void k_sylv_extract(int p, int q, const double* __restrict__ Sr, const double* __restrict__ Si,
                               double* __restrict__ Yr, double* __restrict__ Yi, int ldy) {
  const int N = p + q;
  const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= q) return;
  Yr[(long long)i * ldy + j] = -0.5 * Sr[(long long)i * N + p + j];
  Yi[(long long)i * ldy + j] = -0.5 * Si[(long long)i * N + p + j];
}

}  // namespace

void newton_step(hipStream_t s, int n, double* Xr, double* Xi, int ldx, const double* Ir, const double* Ii, int ldi,
                 bool herm, unsigned long long* maxes) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, maxes);
  FROB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_newton_step, dim3(ceil_div(n, NT), ceil_div(n, NT)), dim3(NT, NR), 0, s, n, Xr, Xi, ldx, Ir,
                     Ii, ldi, herm ? 1 : 0, maxes);
  FROB_LAUNCH_CHECK();
}

void sylvester_assemble(hipStream_t s, int p, int q, const double* Ar, const double* Ai, int lda, const double* Br,
                        const double* Bi, int ldb, bool lyap, const double* Cr, const double* Ci, int ldc,
                        double* Xr, double* Xi) {
  const int N = p + q;
  hipLaunchKernelGGL(k_sylv_assemble, dim3(ceil_div(N, 256), N), dim3(256), 0, s, p, q, Ar, Ai, lda, Br, Bi, ldb,
                     lyap ? 1 : 0, Cr, Ci, ldc, Xr, Xi);
  FROB_LAUNCH_CHECK();
}

void sylvester_extract(hipStream_t s, int p, int q, const double* Sr, const double* Si, double* Yr, double* Yi,
                       int ldy) {
  hipLaunchKernelGGL(k_sylv_extract, dim3(ceil_div(q, 256), p), dim3(256), 0, s, p, q, Sr, Si, Yr, Yi, ldy);
  FROB_LAUNCH_CHECK();
}

}  // namespace frob
