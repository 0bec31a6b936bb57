// elem.hip -- bandwidth-bound elementwise kernels (copies, shifts, column
// permutations, triangle mirroring).  Each thread handles consecutive columns
// of one row so that a wave64 reads and writes contiguous 512-byte segments.
#include "common.hpp"
#include "internal.hpp"

namespace frob {

namespace {

constexpr int EB = 256;

inline dim3 grid2d(int m, int n) { return dim3(ceil_div(n, EB), m); }

__global__ void k_iota(int n, int* p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

__global__ void k_fill_i32(int n, int v, int* p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_copy(int m, int n, const double* __restrict__ src, int lds, const int* __restrict__ rows,
                       double* __restrict__ dst, int ldd) {
  const int i = blockIdx.y, j = blockIdx.x * EB + threadIdx.x;
  if (j >= n) return;
  const int r = rows ? rows[i] : i;
  dst[(long long)i * ldd + j] = src[(long long)r * lds + j];
}

__global__ void k_fill(int m, int n, double v, double* __restrict__ dst, int ldd) {
  const int i = blockIdx.y, j = blockIdx.x * EB + threadIdx.x;
  if (j < n) dst[(long long)i * ldd + j] = v;
}

__global__ void k_identity(int n, double* __restrict__ dst, int ldd) {
  const int i = blockIdx.y, j = blockIdx.x * EB + threadIdx.x;
  if (j < n) dst[(long long)i * ldd + j] = (i == j) ? 1.0 : 0.0;
}

__global__ void k_axpby(int m, int n, double a, const double* __restrict__ X, int ldx, double b,
                        double* __restrict__ Y, int ldy) {
  const int i = blockIdx.y, j = blockIdx.x * EB + threadIdx.x;
  if (j >= n) return;
  double* y = Y + (long long)i * ldy + j;
  const double x = X[(long long)i * ldx + j];
  *y = (b == 0.0) ? a * x : a * x + b * *y;
}

// Z = a X + b Y
__global__ void k_lincomb(int m, int n, double a, const double* __restrict__ X, int ldx, double b,
                          const double* __restrict__ Y, int ldy, double* __restrict__ Z, int ldz) {
  const int i = blockIdx.y, j = blockIdx.x * EB + threadIdx.x;
  if (j >= n) return;
  Z[(long long)i * ldz + j] = a * X[(long long)i * ldx + j] + b * Y[(long long)i * ldy + j];
}

// Xr += P - Q, Xi += P + Q
__global__ void k_acc_rot(int m, int n, const double* __restrict__ P, int ldp, const double* __restrict__ Q, int ldq,
                          double* __restrict__ Xr, double* __restrict__ Xi, int ldx) {
  const int i = blockIdx.y, j = blockIdx.x * EB + threadIdx.x;
  if (j >= n) return;
  const double p = P[(long long)i * ldp + j], q = Q[(long long)i * ldq + j];
  Xr[(long long)i * ldx + j] += p - q;
  Xi[(long long)i * ldx + j] += p + q;
}

// R <- I - R (real and imaginary planes), sumsq += ||R||_F^2.  A block
// covers RESID_ROWS rows (one atomic per block: few enough that the atomics
// on the single accumulator do not serialize the kernel).
constexpr int RESID_ROWS = 8;
__global__ void k_resid_form(int n, double* __restrict__ Rr, double* __restrict__ Ri, int ld, double* sumsq) {
  double acc = 0.0;
  const int i1 = min(n, (int)(blockIdx.x + 1) * RESID_ROWS);
  for (int i = blockIdx.x * RESID_ROWS; i < i1; ++i) {
    double* pr = Rr + (long long)i * ld;
    double* pi = Ri + (long long)i * ld;
    for (int j = threadIdx.x; j < n; j += EB) {
      const double vr = (i == j ? 1.0 : 0.0) - pr[j], vi = -pi[j];
      pr[j] = vr;
      pi[j] = vi;
      acc = fma(vr, vr, fma(vi, vi, acc));
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  __shared__ double part[EB / 64];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < EB / 64; ++w) t += part[w];
    atomicAdd(sumsq, t);
  }
}

__global__ void k_rotate(int m, int n, double mu, const double* __restrict__ A, int lda,
                         const double* __restrict__ B, int ldb, double* X1, int ld1, double* X2, int ld2) {
  const int i = blockIdx.y, j = blockIdx.x * EB + threadIdx.x;
  if (j >= n) return;
  const double a = A[(long long)i * lda + j], b = B[(long long)i * ldb + j];
  X1[(long long)i * ld1 + j] = a - mu * b;
  X2[(long long)i * ld2 + j] = mu * a + b;
}

// (X1, X2) = (c A - s B, s A + c B)
__global__ void k_rot(int m, int n, double c, double sn, const double* __restrict__ A, int lda,
                      const double* __restrict__ B, int ldb, double* X1, int ld1, double* X2, int ld2) {
  const int i = blockIdx.y, j = blockIdx.x * EB + threadIdx.x;
  if (j >= n) return;
  const double a = A[(long long)i * lda + j], b = B[(long long)i * ldb + j];
  X1[(long long)i * ld1 + j] = c * a - sn * b;
  X2[(long long)i * ld2 + j] = sn * a + c * b;
}

// colsum[j] += sum over this block's rows of |a_ij|
constexpr int COL_ROWS = 64;
__global__ void k_colabs(int n, const double* __restrict__ a, int lda, double* colsum) {
  const int j = blockIdx.x * EB + threadIdx.x;
  if (j >= n) return;
  const int i0 = blockIdx.y * COL_ROWS, i1 = min(n, i0 + COL_ROWS);
  double acc = 0.0;
  for (int i = i0; i < i1; ++i) acc += fabs(a[(long long)i * lda + j]);
  atomicAdd(colsum + j, acc);
}

// *out = max_j colsum[j] (one block)
__global__ void k_maxabs(int n, const double* __restrict__ v, double* out) {
  double m = 0.0;
  for (int j = threadIdx.x; j < n; j += EB) m = fmax(m, v[j]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  __shared__ double part[EB / 64];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < EB / 64; ++w) t = fmax(t, part[w]);
    *out = t;
  }
}

__global__ void k_permute_cols(int m, int n, const double* __restrict__ src, int lds, const int* __restrict__ perm,
                               double* __restrict__ dst, int ldd) {
  const int i = blockIdx.y, j = blockIdx.x * EB + threadIdx.x;
  if (j >= n) return;
  dst[(long long)i * ldd + perm[j]] = src[(long long)i * lds + j];
}

__global__ void k_mirror_lower(int n, double* a, int lda, double sign) {
  const int i = blockIdx.y, j = blockIdx.x * EB + threadIdx.x;
  if (j < n && j > i) a[(long long)i * lda + j] = sign * a[(long long)j * lda + i];
}

__global__ void k_cvt_f32_f64(int m, int n, const float* __restrict__ src, int lds, double* __restrict__ dst, int ldd) {
  const int i = blockIdx.y, j = blockIdx.x * EB + threadIdx.x;
  if (j < n) dst[(long long)i * ldd + j] = (double)src[(long long)i * lds + j];
}

__global__ void k_cvt_f64_f32(int m, int n, const double* __restrict__ src, int lds, float* __restrict__ dst, int ldd) {
  const int i = blockIdx.y, j = blockIdx.x * EB + threadIdx.x;
  if (j < n) dst[(long long)i * ldd + j] = (float)src[(long long)i * lds + j];
}

// Gauss's three products P1 (in Z0), P2 (in Z1), P3 -> Z0 = P1 - tau P2, Z1 = P3 - P1 - P2
__global__ void k_gauss3_combine(long long cnt, double* __restrict__ Z0, double* __restrict__ Z1,
                                 const double* __restrict__ P3, double tau) {
  const long long e = (long long)blockIdx.x * EB + threadIdx.x;
  if (e >= cnt) return;
  const double p1 = Z0[e], p2 = Z1[e];
  Z0[e] = p1 - tau * p2;
  Z1[e] = P3[e] - p1 - p2;
}

__global__ void k_zero_upper(int n, double* a, int lda) {
  const int i = blockIdx.y, j = blockIdx.x * EB + threadIdx.x;
  if (j < n && j > i) a[(long long)i * lda + j] = 0.0;
}

}  // namespace

void resid_form_f64(hipStream_t s, int n, double* Rr, double* Ri, int ld, double* sumsq) {
  fill_f64(s, 1, 1, 0.0, sumsq, 1);
  hipLaunchKernelGGL(k_resid_form, dim3(ceil_div(n, RESID_ROWS)), dim3(EB), 0, s, n, Rr, Ri, ld, sumsq);
  FROB_LAUNCH_CHECK();
}

void iota_i32(hipStream_t s, int n, int* p) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_iota, dim3(ceil_div(n, EB)), dim3(EB), 0, s, n, p);
  FROB_LAUNCH_CHECK();
}

void fill_i32(hipStream_t s, int n, int v, int* p) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(ceil_div(n, EB)), dim3(EB), 0, s, n, v, p);
  FROB_LAUNCH_CHECK();
}

void copy_f64(hipStream_t s, int m, int n, const double* src, int lds, const int* rows, double* dst, int ldd) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_copy, grid2d(m, n), dim3(EB), 0, s, m, n, src, lds, rows, dst, ldd);
  FROB_LAUNCH_CHECK();
}

void fill_f64(hipStream_t s, int m, int n, double v, double* dst, int ldd) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_fill, grid2d(m, n), dim3(EB), 0, s, m, n, v, dst, ldd);
  FROB_LAUNCH_CHECK();
}

void identity_f64(hipStream_t s, int n, double* dst, int ldd) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_identity, grid2d(n, n), dim3(EB), 0, s, n, dst, ldd);
  FROB_LAUNCH_CHECK();
}

void axpby_f64(hipStream_t s, int m, int n, double a, const double* X, int ldx, double b, double* Y, int ldy) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_axpby, grid2d(m, n), dim3(EB), 0, s, m, n, a, X, ldx, b, Y, ldy);
  FROB_LAUNCH_CHECK();
}

void lincomb_f64(hipStream_t s, int m, int n, double a, const double* X, int ldx, double b, const double* Y, int ldy,
                 double* Z, int ldz) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_lincomb, grid2d(m, n), dim3(EB), 0, s, m, n, a, X, ldx, b, Y, ldy, Z, ldz);
  FROB_LAUNCH_CHECK();
}

void acc_rot_f64(hipStream_t s, int m, int n, const double* P, int ldp, const double* Q, int ldq, double* Xr,
                 double* Xi, int ldx) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_acc_rot, grid2d(m, n), dim3(EB), 0, s, m, n, P, ldp, Q, ldq, Xr, Xi, ldx);
  FROB_LAUNCH_CHECK();
}

void rotate_f64(hipStream_t s, int m, int n, double mu, const double* A, int lda, const double* B, int ldb,
                double* X1, int ld1, double* X2, int ld2) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_rotate, grid2d(m, n), dim3(EB), 0, s, m, n, mu, A, lda, B, ldb, X1, ld1, X2, ld2);
  FROB_LAUNCH_CHECK();
}

void rot_f64(hipStream_t s, int m, int n, double c, double sn, const double* A, int lda, const double* B, int ldb,
             double* X1, int ld1, double* X2, int ld2) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_rot, grid2d(m, n), dim3(EB), 0, s, m, n, c, sn, A, lda, B, ldb, X1, ld1, X2, ld2);
  FROB_LAUNCH_CHECK();
}

void norm1_f64(hipStream_t s, int n, const double* a, int lda, double* colsum, double* out) {
  fill_f64(s, 1, n, 0.0, colsum, n);
  hipLaunchKernelGGL(k_colabs, dim3(ceil_div(n, EB), ceil_div(n, COL_ROWS)), dim3(EB), 0, s, n, a, lda, colsum);
  FROB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_maxabs, dim3(1), dim3(EB), 0, s, n, colsum, out);
  FROB_LAUNCH_CHECK();
}

void permute_cols_f64(hipStream_t s, int m, int n, const double* src, int lds, const int* perm, double* dst,
                      int ldd) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_permute_cols, grid2d(m, n), dim3(EB), 0, s, m, n, src, lds, perm, dst, ldd);
  FROB_LAUNCH_CHECK();
}

void mirror_lower_f64(hipStream_t s, int n, double* a, int lda, double sign) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mirror_lower, grid2d(n, n), dim3(EB), 0, s, n, a, lda, sign);
  FROB_LAUNCH_CHECK();
}

void gauss3_combine_f64(hipStream_t s, long long cnt, double* Z0, double* Z1, const double* P3, double tau) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL(k_gauss3_combine, dim3((unsigned)((cnt + EB - 1) / EB)), dim3(EB), 0, s, cnt, Z0, Z1, P3, tau);
  FROB_LAUNCH_CHECK();
}

void convert_f32_f64(hipStream_t s, int m, int n, const float* src, int lds, double* dst, int ldd) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_cvt_f32_f64, grid2d(m, n), dim3(EB), 0, s, m, n, src, lds, dst, ldd);
  FROB_LAUNCH_CHECK();
}

void convert_f64_f32(hipStream_t s, int m, int n, const double* src, int lds, float* dst, int ldd) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_cvt_f64_f32, grid2d(m, n), dim3(EB), 0, s, m, n, src, lds, dst, ldd);
  FROB_LAUNCH_CHECK();
}

void zero_upper_f64(hipStream_t s, int n, double* a, int lda) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero_upper, grid2d(n, n), dim3(EB), 0, s, n, a, lda);
  FROB_LAUNCH_CHECK();
}

}  // namespace frob
