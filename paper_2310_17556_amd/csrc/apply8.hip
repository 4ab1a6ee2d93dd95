// Step 6 of Algorithm 1, x = (v - S^T y) / lambda, when y = y_c + z ends with a small refinement
// correction z: S^T y_c is carried exactly through the refinement passes (T), and the image of z
// is taken through the scaled-FP8 copy Q of S that the row pass wrote for the Gram (one byte per
// entry, a quarter of the bytes of S). Q = S + E with |E_ij| <= 2^-4 |S_ij| (E4M3 rounding under a
// power-of-two block scale), so the result differs from the exact image by E^T z, about 3 % of
// |S^T z| for rounding errors independent between entries; final_decide estimates that size
// against |S^T y| and falls back to the exact apply (the column pass over S) unless it is small.
// For a centered S the all-ones component of z, whose image through S is nearly zero but through
// Q is not (the rounding errors do not sum to zero over a column), is split off and taken exactly
// through the column sums S^T 1 that the residual pass wrote.
#include "dfisher_internal.h"

namespace dfi {
namespace {

constexpr int DT = 1024;   // final_decide: one workgroup
constexpr int AT = 256;    // fp8_apply: 64 row slots x 4 column quarters of a 64-column block

__device__ double tree_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = DT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ void t_axpy_kernel(double* __restrict__ T, const double* __restrict__ U, const double* __restrict__ alpha,
                              int64_t m, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) T[j] = fma(alpha[0], U[j], T[j]);
}

__global__ void __launch_bounds__(DT)
final_decide_kernel(int64_t n, double* __restrict__ y, const double* __restrict__ z, const double* __restrict__ b,
                    const double* __restrict__ d, double lambda, const int* __restrict__ cflag, double est_max,
                    float* __restrict__ zf, double* __restrict__ abar_out, int* __restrict__ use) {
  __shared__ double red[DT];
  const int tid = threadIdx.x;
  const int centered = cflag ? *cflag : 0;   // uniform
  double s = 0.0;
  if (centered)
    for (int64_t i = tid; i < n; i += DT) s += z[i];
  const double abar = centered ? tree_sum(s, red) / (double)n : 0.0;
  double a = 0.0, yb = 0.0, yy = 0.0;
  for (int64_t i = tid; i < n; i += DT) {
    const double zp = z[i] - abar;
    zf[i] = (float)zp;
    a = fma(d[i] * zp, zp, a);
    yb = fma(y[i], b[i], yb);
    yy = fma(y[i], y[i], yy);
  }
  const double A = tree_sum(a, red);
  const double YB = tree_sum(yb, red);
  const double YY = tree_sum(yy, red);
  const double sty = YB - lambda * YY;   // |S^T y|^2 of the iterate, as y.(W y) - lambda |y|^2 with W y ~ b
  const bool ok = sty > 0.0 && A >= 0.0 && A <= est_max * est_max * sty;   // false for NaN as well
  if (!ok)
    for (int64_t i = tid; i < n; i += DT) y[i] += z[i];
  if (tid == 0) {
    *abar_out = abar;
    *use = ok ? 1 : 0;
  }
}

// One workgroup per 64-column block: thread (row slot g, quarter c) takes 16 columns (one 16-byte
// load of codes per row) of the rows g, g + 64, ..., with FP32 products and sums (the term is a
// small correction: 1e-6 relative is far below what it needs); the 64 row slots are then added in
// a fixed order.
__global__ void __launch_bounds__(AT)
fp8_apply_kernel(const uint8_t* __restrict__ q, const uint8_t* __restrict__ sc, int64_t n, int64_t m,
                 const float* __restrict__ zf, const double* __restrict__ T, const double* __restrict__ cs,
                 const double* __restrict__ abar, const float* __restrict__ v, double lambda, void* __restrict__ x,
                 int x64, const int* __restrict__ use) {
  if (!*use) return;
  __shared__ float red[64][65];
  const int tid = threadIdx.x;
  const int g = tid >> 2, cq = tid & 3;
  const int64_t jb = blockIdx.x;
  const int64_t j0 = jb * 64 + cq * 16;   // this thread's first column
  const uint8_t* qb = q + jb * n * 64 + cq * 16;                     // row i at qb + 64 i
  const uint8_t* sb = sc + (j0 >> 7) * n * 4 + ((j0 >> 5) & 3);      // row i at sb + 4 i
  float acc[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) acc[u] = 0.f;
  auto row = [&](int64_t i) {
    const uint4 c4 = *reinterpret_cast<const uint4*>(qb + i * 64);
    const uint32_t e = sb[i * 4];
    const float w = zf[i] * __uint_as_float(e ? e << 23 : 0x00400000u);   // 2^(e - 127), also for e = 0
    const uint32_t wd[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)wd[k], false);   // bytes 0, 1
      const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)wd[k], true);    // bytes 2, 3
      acc[4 * k + 0] = fmaf(lo[0], w, acc[4 * k + 0]);
      acc[4 * k + 1] = fmaf(lo[1], w, acc[4 * k + 1]);
      acc[4 * k + 2] = fmaf(hi[0], w, acc[4 * k + 2]);
      acc[4 * k + 3] = fmaf(hi[1], w, acc[4 * k + 3]);
    }
  };
  int64_t i = g;
  for (; i + 192 < n; i += 256) {   // four rows per thread in flight
    row(i);
    row(i + 64);
    row(i + 128);
    row(i + 192);
  }
  for (; i < n; i += 64) row(i);
#pragma unroll
  for (int u = 0; u < 16; ++u) red[g][cq * 16 + u] = acc[u];
  __syncthreads();
  if (tid < 64) {
    const int64_t j = jb * 64 + tid;
    float sum = 0.f;
    for (int k = 0; k < 64; ++k) sum += red[k][tid];
    if (j < m) {
      const double ab = cs ? abar[0] * cs[j] : 0.0;
      const double xv = ((double)v[j] - T[j] - ab - (double)sum) / lambda;
      if (x64) static_cast<double*>(x)[j] = xv;
      else static_cast<float*>(x)[j] = (float)xv;
    }
  }
}

}  // namespace

hipError_t t_axpy(double* T, const double* U, const double* alpha, int64_t m, hipStream_t st, const int* skip) {
  hipLaunchKernelGGL(t_axpy_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, T, U, alpha, m, skip);
  return hipGetLastError();
}

hipError_t final_decide(int64_t n, double* y, const double* z, const double* b, const double* d, double lambda,
                        const int* centered, double est_max, float* zf, double* abar, int* use, hipStream_t st) {
  hipLaunchKernelGGL(final_decide_kernel, dim3(1), dim3(DT), 0, st, n, y, z, b, d, lambda, centered, est_max, zf, abar,
                     use);
  return hipGetLastError();
}

hipError_t fp8_apply(const uint8_t* q, const uint8_t* sc, int64_t ldq, int64_t n, int64_t m, const float* zf,
                     const double* T, const double* cs, const double* abar, const float* v, double lambda, void* x,
                     int x64, const int* use, hipStream_t st) {
  if ((ldq & 127) != 0 || ldq < m) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fp8_apply_kernel, dim3((unsigned)((m + 63) / 64)), dim3(AT), 0, st, q, sc, n, m, zf, T, cs, abar,
                     v, lambda, x, x64, use);
  return hipGetLastError();
}

}  // namespace dfi
