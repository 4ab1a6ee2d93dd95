// Front end of stochastic reconfiguration (Section 3) and the complex variant's vector work.
//
// Centering: the score matrix of SR is S = (O - mean O) / sqrt(n), the mean over the n samples
// (rows) of every parameter (column). The column sums come from the column pass (FP64, with
// y = 1); the kernels here write S_ij = fl32((O_ij - sum_j / n) / sqrt(n)), FP64 arithmetic and
// one rounding. A complex O (interleaved real and imaginary FP32 parts) is written in the stacked
// real form Z = [Re S; Im S] (2n x m), which is both the real-part variant's score matrix
// (F = Re[S^H S] = Z^T Z) and the planar form of S that the complex variant works on.
//
// Complex variant: with S = A + iB (Z = [A; B]) the system (S^H S + lambda I) x = v is the real
// system of the 2n x 2m matrix E = [[A, -B], [B, A]] with v = [Re v; Im v]. Its Gram is assembled
// from Z Z^T = [[A A^T, A B^T], [B A^T, B B^T]]:
//   E E^T = [[Wr, -Wi], [Wi, Wr]],  Wr = A A^T + B B^T,  Wi = B A^T - A B^T,
// and the products with E and E^T are products with Z of two vectors each, combined here.
#include "dfisher_internal.h"

#include <algorithm>
#include <cmath>

namespace dfi {
namespace {

constexpr int CT = 256;

// S_ij = fl32((O_ij - t_j / n) / rn), t = FP64 column sums of O; rows of O and S may coincide
// (same pointer and stride: each element is read and then written by the same thread).
__global__ void __launch_bounds__(CT) center_write_kernel(const float* O, int64_t n, int64_t m, int64_t ldo,
                                                          const double* __restrict__ t, double rn, float* S,
                                                          int64_t lds) {
  const int64_t j = (int64_t)blockIdx.x * CT + threadIdx.x;
  if (j >= m) return;
  const double mu = t[j] / (double)n;
  for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
    const double o = (double)O[i * ldo + j];
    S[i * lds + j] = (float)((o - mu) / rn);
  }
}

// Complex O (interleaved re, im; row stride ldo complex elements) -> Z rows i (real) and n + i
// (imaginary); t holds the interleaved column sums (t[2j] real, t[2j + 1] imaginary).
__global__ void __launch_bounds__(CT) center_write_complex_kernel(const float* __restrict__ O, int64_t n, int64_t m,
                                                                  int64_t ldo, const double* __restrict__ t, double rn,
                                                                  float* __restrict__ Z, int64_t ldz) {
  const int64_t j = (int64_t)blockIdx.x * CT + threadIdx.x;
  if (j >= m) return;
  const double mr = t[2 * j] / (double)n, mi = t[2 * j + 1] / (double)n;
  for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
    const float2 o = reinterpret_cast<const float2*>(O)[i * ldo + j];
    Z[i * ldz + j] = (float)(((double)o.x - mr) / rn);
    Z[(n + i) * ldz + j] = (float)(((double)o.y - mi) / rn);
  }
}

__global__ void fill_kernel(double* __restrict__ y, int64_t n, double value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = value;
}

// interleaved complex v (FP32 pairs) -> planar vr (first m), vi (next m)
__global__ void deinterleave_kernel(const float* __restrict__ v, int64_t m, float* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const float2 c = reinterpret_cast<const float2*>(v)[k];
  out[k] = c.x;
  out[m + k] = c.y;
}

// What (2n x 2n, row-major) = [[Wr, -Wi], [Wi, Wr]] + lambda I from G = Z Z^T (2n x 2n, both
// triangles): Wr_ij = G_ij + G_(n+i)(n+j), Wi_ij = G_(n+i)j - G_i(n+j).
__global__ void complex_embed_kernel(const double* __restrict__ G, int64_t n, double lambda, double* __restrict__ Wh) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j >= n) return;
  const int64_t N = 2 * n;
  const double wr = G[i * N + j] + G[(n + i) * N + n + j] + (i == j ? lambda : 0.0);
  const double wi = G[(n + i) * N + j] - G[i * N + n + j];
  Wh[i * N + j] = wr;
  Wh[(n + i) * N + n + j] = wr;
  Wh[(n + i) * N + j] = wi;
  Wh[i * N + n + j] = -wi;
}

// From P = Z u1 and Q = Z u2 (each 2n: [A u; B u]):
// out = rhs - lambda y + sgn [A u1 - B u2; B u1 + A u2]   (rhs, y may be null: treated as 0)
__global__ void complex_combine_kernel(const double* __restrict__ P, const double* __restrict__ Q, int64_t n,
                                       double sgn, const double* __restrict__ rhs, const double* __restrict__ y,
                                       double lambda, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double top = P[i] - Q[n + i];       // A u1 - B u2
  const double bot = P[n + i] + Q[i];       // B u1 + A u2
  double o1 = sgn * top, o2 = sgn * bot;
  if (rhs) {
    o1 += rhs[i];
    o2 += rhs[n + i];
  }
  if (y) {
    o1 -= lambda * y[i];
    o2 -= lambda * y[n + i];
  }
  out[i] = o1;
  out[n + i] = o2;
}

// [y1; y2] -> the two column-pass vectors [y1; y2] and [y2; -y1] (each 2n)
__global__ void complex_colvecs_kernel(const double* __restrict__ y, int64_t n, double* __restrict__ u1,
                                       double* __restrict__ u2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = y[i], b = y[n + i];
  u1[i] = a;
  u1[n + i] = b;
  u2[i] = b;
  u2[n + i] = -a;
}

// x_k = ((vr_k - T[16 k]) + i (vi_k - T[16 k + 1])) / lambda, interleaved, FP32 or FP64
template <bool F64>
__global__ void complex_apply_kernel(const float* __restrict__ v, const double* __restrict__ T, int64_t m, double lambda,
                                     void* __restrict__ x) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const float2 c = reinterpret_cast<const float2*>(v)[k];
  const double xr = ((double)c.x - T[k * MULTI_VECS]) / lambda;
  const double xi = ((double)c.y - T[k * MULTI_VECS + 1]) / lambda;
  if constexpr (F64) {
    static_cast<double*>(x)[2 * k] = xr;
    static_cast<double*>(x)[2 * k + 1] = xi;
  } else {
    static_cast<float*>(x)[2 * k] = (float)xr;
    static_cast<float*>(x)[2 * k + 1] = (float)xi;
  }
}

unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t center_write(const float* O, int64_t n, int64_t m, int64_t ldo, int cplx, const double* t, float* S,
                        int64_t lds, hipStream_t st) {
  const double rn = std::sqrt((double)n);
  const dim3 grid(blocks(m, CT), (unsigned)std::min<int64_t>(n, 64));
  if (cplx)
    hipLaunchKernelGGL(center_write_complex_kernel, grid, dim3(CT), 0, st, O, n, m, ldo, t, rn, S, lds);
  else
    hipLaunchKernelGGL(center_write_kernel, grid, dim3(CT), 0, st, O, n, m, ldo, t, rn, S, lds);
  return hipGetLastError();
}

hipError_t fill_value(double* y, int64_t n, double value, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel, dim3(blocks(n, 256)), dim3(256), 0, st, y, n, value);
  return hipGetLastError();
}

hipError_t deinterleave(const float* v, int64_t m, float* out, hipStream_t st) {
  hipLaunchKernelGGL(deinterleave_kernel, dim3(blocks(m, 256)), dim3(256), 0, st, v, m, out);
  return hipGetLastError();
}

hipError_t complex_embed(const double* G, int64_t n, double lambda, double* Wh, hipStream_t st) {
  hipLaunchKernelGGL(complex_embed_kernel, dim3(blocks(n, 256), (unsigned)n), dim3(256), 0, st, G, n, lambda, Wh);
  return hipGetLastError();
}

hipError_t complex_combine(const double* P, const double* Q, int64_t n, double sgn, const double* rhs, const double* y,
                           double lambda, double* out, hipStream_t st) {
  hipLaunchKernelGGL(complex_combine_kernel, dim3(blocks(n, 256)), dim3(256), 0, st, P, Q, n, sgn, rhs, y, lambda,
                     out);
  return hipGetLastError();
}

hipError_t complex_colvecs(const double* y, int64_t n, double* u1, double* u2, hipStream_t st) {
  hipLaunchKernelGGL(complex_colvecs_kernel, dim3(blocks(n, 256)), dim3(256), 0, st, y, n, u1, u2);
  return hipGetLastError();
}

hipError_t complex_apply(const float* v, const double* T, int64_t m, double lambda, void* x, int x_fp64,
                         hipStream_t st) {
  if (x_fp64)
    hipLaunchKernelGGL(complex_apply_kernel<true>, dim3(blocks(m, 256)), dim3(256), 0, st, v, T, m, lambda, x);
  else
    hipLaunchKernelGGL(complex_apply_kernel<false>, dim3(blocks(m, 256)), dim3(256), 0, st, v, T, m, lambda, x);
  return hipGetLastError();
}

}  // namespace dfi
