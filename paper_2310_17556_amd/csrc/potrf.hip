// Blocked right-looking FP64 Cholesky W = L L^T (Algorithm 1 step 2), in place on a row-major
// n x n matrix, lower triangle. Block size 64; per block column k:
//   1. potf2   one wave factors the 64 x 64 diagonal block in LDS (left-looking: lane i owns
//              row i and forms column j from dot products with the finished columns).
//   2. trsm    rows below the block: A_ik <- A_ik L_kk^-T, one lane per row, L_kk in LDS.
//   3. update  trailing lower triangle A_IJ -= A_Ik A_Jk^T in 64 x 64 tiles, panels in LDS.
// A pivot d with !(d > 0) (NaN included) stores the 1-based global index in *info and raises
// *flag; every later kernel sees the flag and returns at once, so the device work drains
// without touching the matrix further.
#include "dfisher_internal.h"

namespace dfi {
namespace {

constexpr int NB = 64;
constexpr int LDP = NB + 1;  // padded LDS row (doubles)

__global__ void __launch_bounds__(64)
potf2_kernel(double* __restrict__ A, int64_t n, int64_t k, int64_t* __restrict__ info, int32_t* __restrict__ flag) {
  __shared__ double a[NB * LDP];
  if (*(volatile int32_t*)flag) return;
  const int lane = threadIdx.x;
  const int64_t nb = min<int64_t>(NB, n - k);
  // Load the lower triangle of the diagonal block; pad beyond nb with the identity.
  for (int i = 0; i < NB; ++i) {
    const int j = lane;
    double val = 0.0;
    if (i < nb && j < nb) {
      if (j <= i) val = A[(k + i) * n + k + j];
    } else if (i == j) {
      val = 1.0;
    }
    a[i * LDP + j] = val;
  }
  __syncthreads();
  const int i = lane;
  for (int j = 0; j < NB; ++j) {
    // lane i >= j: s = a_ij - sum_{l<j} L_il L_jl
    double s = (i >= j) ? a[i * LDP + j] : 0.0;
    for (int l = 0; l < j; ++l) s -= a[i * LDP + l] * a[j * LDP + l];
    const double d = __shfl(s, j, 64);
    if (!(d > 0.0)) {
      if (lane == 0) {
        *info = k + j + 1;
        *flag = 1;
      }
      return;
    }
    const double ljj = sqrt(d);
    if (i == j) a[i * LDP + j] = ljj;
    else if (i > j) a[i * LDP + j] = s / ljj;
    __syncthreads();
  }
  for (int r = 0; r < nb; ++r) {
    if (lane <= r) A[(k + r) * n + k + lane] = a[r * LDP + lane];
  }
}

// Rows i in [k + NB, n): A[i][k .. k+NB) <- A[i][k .. k+NB) * L_kk^-T. One lane per row.
__global__ void __launch_bounds__(64)
trsm_kernel(double* __restrict__ A, int64_t n, int64_t k, const int32_t* __restrict__ flag) {
  __shared__ double Lk[NB * LDP];
  if (*(volatile const int32_t*)flag) return;
  const int lane = threadIdx.x;
  for (int r = 0; r < NB; ++r) Lk[r * LDP + lane] = (lane <= r) ? A[(k + r) * n + k + lane] : 0.0;
  __syncthreads();
  const int64_t i = k + NB + (int64_t)blockIdx.x * 64 + lane;
  if (i >= n) return;
  double x[NB];
  double* row = A + i * n + k;
#pragma unroll
  for (int j = 0; j < NB; ++j) x[j] = row[j];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    double s = x[j];
#pragma unroll
    for (int l = 0; l < j; ++l) s -= x[l] * Lk[j * LDP + l];
    x[j] = s / Lk[j * LDP + j];
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) row[j] = x[j];
}

// Trailing update of the lower triangle below/right of block column k: for tiles (I >= J) of the
// trailing matrix, A_IJ -= P_I P_J^T with P = A[:, k .. k+NB). 256 threads, 4 x 4 outputs each.
__global__ void __launch_bounds__(256)
update_kernel(double* __restrict__ A, int64_t n, int64_t k, const int32_t* __restrict__ flag) {
  __shared__ double PI[NB * LDP];
  __shared__ double PJ[NB * LDP];
  if (*(volatile const int32_t*)flag) return;
  const int64_t t = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int64_t J = t - I * (I + 1) / 2;
  const int64_t base = k + NB;
  const int64_t ri = base + I * NB, rj = base + J * NB;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < NB * NB; idx += 256) {
    const int r = idx / NB, c = idx % NB;
    PI[r * LDP + c] = (ri + r < n) ? A[(ri + r) * n + k + c] : 0.0;
    PJ[r * LDP + c] = (rj + r < n) ? A[(rj + r) * n + k + c] : 0.0;
  }
  __syncthreads();
  const int ty = tid / 16, tx = tid % 16;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int l = 0; l < NB; ++l) {
    double pi[4], pj[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) pi[a] = PI[(ty + 16 * a) * LDP + l];
#pragma unroll
    for (int b = 0; b < 4; ++b) pj[b] = PJ[(tx + 16 * b) * LDP + l];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = fma(pi[a], pj[b], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t gi = ri + ty + 16 * a;
    if (gi >= n) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t gj = rj + tx + 16 * b;
      if (gj > gi || gj >= n) continue;
      A[gi * n + gj] -= acc[a][b];
    }
  }
}

__global__ void zero_upper_kernel(double* __restrict__ A, int64_t n) {
  const int64_t nb = (n + 255) / 256;
  const int64_t i = (int64_t)blockIdx.x / nb;
  const int64_t j = ((int64_t)blockIdx.x - i * nb) * 256 + threadIdx.x;
  if (i < n && j < n && j > i) A[i * n + j] = 0.0;
}

__global__ void shift_copy_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t n, double tau) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx / n, j = idx - i * n;
  dst[idx] = src[idx] + ((i == j) ? tau : 0.0);
}

__global__ void axpy_kernel(double* __restrict__ y, const double* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += d[i];
}

__global__ void diag_max_kernel(const double* __restrict__ W, int64_t n, double* __restrict__ out) {
  __shared__ double red[256];
  double mx = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double d = W[i * n + i];
    mx = (d > mx) ? d : mx;
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void clear_status_kernel(int64_t* info, int32_t* flag) {
  *info = 0;
  *flag = 0;
}

}  // namespace

hipError_t potrf_launch(double* A, int64_t n, int64_t* info_dev, int32_t* flag_dev, hipStream_t st) {
  hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(1), 0, st, info_dev, flag_dev);
  for (int64_t k = 0; k < n; k += NB) {
    hipLaunchKernelGGL(potf2_kernel, dim3(1), dim3(64), 0, st, A, n, k, info_dev, flag_dev);
    const int64_t rest = n - k - NB;
    if (rest > 0) {
      const int64_t rb = (rest + 63) / 64;
      hipLaunchKernelGGL(trsm_kernel, dim3((unsigned)rb), dim3(64), 0, st, A, n, k, flag_dev);
      hipLaunchKernelGGL(update_kernel, dim3((unsigned)(rb * (rb + 1) / 2)), dim3(256), 0, st, A, n, k, flag_dev);
    }
  }
  return hipGetLastError();
}

hipError_t zero_upper(double* A, int64_t n, hipStream_t st) {
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(zero_upper_kernel, dim3((unsigned)(nb * n)), dim3(256), 0, st, A, n);
  return hipGetLastError();
}

hipError_t shift_copy(const double* src, double* dst, int64_t n, double tau, hipStream_t st) {
  const int64_t tot = n * n;
  hipLaunchKernelGGL(shift_copy_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, src, dst, n, tau);
  return hipGetLastError();
}

hipError_t axpy_inplace(double* y, const double* d, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, y, d, n);
  return hipGetLastError();
}

hipError_t diag_max(const double* W, int64_t n, double* out_dev, hipStream_t st) {
  hipLaunchKernelGGL(diag_max_kernel, dim3(1), dim3(256), 0, st, W, n, out_dev);
  return hipGetLastError();
}

}  // namespace dfi
