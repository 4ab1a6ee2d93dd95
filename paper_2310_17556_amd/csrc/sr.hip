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
//
// Centered preconditioner: a centered S has 1^T S = 0, so S S^T maps the all-ones vector to zero
// and W maps it to lambda times itself (for the complex embedding, the indicators of the real and
// the imaginary halves). A Gram formed from rounded inputs does not: for the scaled-FP8 Gram its
// error along that direction is ~1e-3 of the diagonal, far above lambda, which leaves the factor a
// poor preconditioner there and the refinement slow. The factored matrix is therefore
//   M = P W P + lambda U U^T,  P = I - U U^T,  U = [1_seg / sqrt(l)] for nseg equal segments of l,
// entrywise M_ij = W_ij - (r_i^(s_j) + r_j^(s_i)) / l + c^(s_i s_j) / l^2 + [s_i = s_j] lambda / l,
// with r_i^(s) = sum over j in segment s of W_ij and c^(st) = sum over i in s of r_i^(t) (FP64,
// fixed order). M agrees with W on the complement of the indicators and is exact on them; the
// refinement still works with the exact W, so only its convergence changes. W is left as it is
// when the computed Gram is far from centered along an indicator (project_update_kernel).
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

// Segment row sums r[s n + i] = sum over j in segment s (nseg <= 2: s = [j >= l]) of W_ij, W
// symmetric and read from its lower triangle, in two fixed-order steps. tile_sums_kernel: one
// workgroup per 64 x 64 tile (ti >= tj) of the lower triangle writes, per segment, the sums of
// its rows (over its columns j <= i) and of its columns (over its rows i > j, the transposed
// half); seg_reduce_kernel then adds, for row i of tile row I, the row sums of tiles (I, 0 .. I)
// and the column sums of tiles (I .. T - 1, I), in that order.
__global__ void __launch_bounds__(256) tile_sums_kernel(const double* __restrict__ W, int64_t n, int64_t l,
                                                        double* __restrict__ part) {
  __shared__ double tile[64][65];
  const int64_t t = blockIdx.x;
  int64_t ti = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  while (ti * (ti + 1) / 2 > t) --ti;
  const int64_t tj = t - ti * (ti + 1) / 2;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int a = e >> 6, b = e & 63;
    const int64_t i = ti * 64 + a, j = tj * 64 + b;
    tile[a][b] = (i < n && j <= i) ? W[i * n + j] : 0.0;
  }
  __syncthreads();
  const int k = threadIdx.x & 63;
  if (threadIdx.x < 64) {            // row k of the tile, over its columns
    double a0 = 0.0, a1 = 0.0;
    for (int b = 0; b < 64; ++b) {
      const double w = tile[k][b];
      if (tj * 64 + b < l) a0 += w; else a1 += w;
    }
    part[(t * 4 + 0) * 64 + k] = a0;
    part[(t * 4 + 1) * 64 + k] = a1;
  } else if (threadIdx.x < 128) {    // column k of the tile, over its rows strictly below the diagonal
    double a0 = 0.0, a1 = 0.0;
    const int a_first = (ti == tj) ? k + 1 : 0;
    for (int a = a_first; a < 64; ++a) {
      const double w = tile[a][k];
      if (ti * 64 + a < l) a0 += w; else a1 += w;
    }
    part[(t * 4 + 2) * 64 + k] = a0;
    part[(t * 4 + 3) * 64 + k] = a1;
  }
}

__global__ void __launch_bounds__(256) seg_reduce_kernel(const double* __restrict__ part, int64_t n, int64_t T,
                                                         int nseg, double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t I = i >> 6;
  const int a = (int)(i & 63);
  for (int s = 0; s < nseg; ++s) {
    double acc = 0.0;
    for (int64_t J = 0; J <= I; ++J) acc += part[((I * (I + 1) / 2 + J) * 4 + s) * 64 + a];
    for (int64_t K = I; K < T; ++K) acc += part[((K * (K + 1) / 2 + I) * 4 + 2 + s) * 64 + a];
    r[(int64_t)s * n + i] = acc;
  }
}

// c[s nseg + u] = sum over i in segment s of r[u n + i], and c[nseg nseg] = trace(W); one
// workgroup, fixed order
__device__ __forceinline__ double block_sum256(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double t = red[0];
  __syncthreads();
  return t;
}

__global__ void __launch_bounds__(256) seg_total_kernel(const double* __restrict__ W, const double* __restrict__ r,
                                                        int64_t n, int64_t l, int nseg, double* __restrict__ c) {
  __shared__ double red[256];
  for (int s = 0; s < nseg; ++s)
    for (int u = 0; u < nseg; ++u) {
      double acc = 0.0;
      for (int64_t i = threadIdx.x; i < l; i += 256) acc += r[(int64_t)u * n + (int64_t)s * l + i];
      const double t = block_sum256(acc, red);
      if (threadIdx.x == 0) c[s * nseg + u] = t;
    }
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) acc += W[i * n + i];
  const double t = block_sum256(acc, red);
  if (threadIdx.x == 0) c[nseg * nseg] = t;
}

// W <- M entrywise (lower triangle, or both when full), unless the declaration is implausible:
// the computed Gram's Rayleigh quotient along some indicator, c_ss / l - lambda, exceeds
// CENTER_GUARD times its mean diagonal. For a centered S that quotient is the Gram's rounding
// error along the indicator (about 1e-3 of the diagonal for the scaled-FP8 Gram); a clearly
// non-centered S would otherwise get a factor that is exact nowhere near W along it.
constexpr double CENTER_GUARD = 0.01;

__global__ void __launch_bounds__(256) project_update_kernel(double* __restrict__ W, int64_t n, int64_t l, int nseg,
                                                             const double* __restrict__ r, const double* __restrict__ c,
                                                             double lambda, int full, int64_t nb,
                                                             int* __restrict__ applied) {
  const double dbar = c[nseg * nseg] / (double)n - lambda;
  bool ok = true;
  for (int s = 0; s < nseg; ++s)
    if (!(c[s * nseg + s] / (double)l - lambda <= CENTER_GUARD * dbar)) ok = false;
  if (applied && blockIdx.x == 0 && threadIdx.x == 0) *applied = ok ? 1 : 0;
  if (!ok) return;
  const int64_t i = (int64_t)blockIdx.x / nb;
  const int64_t j = ((int64_t)blockIdx.x - i * nb) * 256 + threadIdx.x;
  if (j >= n || (!full && j > i)) return;
  const int64_t si = i < l ? 0 : 1, sj = j < l ? 0 : 1;   // nseg <= 2
  const double inv = 1.0 / (double)l;
  double w = W[i * n + j] - (r[sj * n + i] + r[si * n + j]) * inv + c[si * nseg + sj] * (inv * inv);
  if (si == sj) w += lambda * inv;
  W[i * n + j] = w;
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

size_t gram_project_work_bytes(int64_t n) {
  const int64_t T = (n + 63) / 64;
  return ((size_t)(T * (T + 1) / 2) * 4 * 64 + 8) * sizeof(double);
}

hipError_t gram_project(double* W, int64_t n, int nseg, double lambda, int full, double* work, double* r,
                        hipStream_t st, int* applied) {
  if (n < 1 || nseg < 1 || nseg > 2 || n % nseg != 0) return hipErrorInvalidValue;
  const int64_t l = n / nseg;
  const int64_t T = (n + 63) / 64;
  double* c = work + (size_t)(T * (T + 1) / 2) * 4 * 64;   // nseg^2 totals and the trace
  hipLaunchKernelGGL(tile_sums_kernel, dim3((unsigned)(T * (T + 1) / 2)), dim3(256), 0, st, W, n, l, work);
  hipLaunchKernelGGL(seg_reduce_kernel, dim3(blocks(n, 256)), dim3(256), 0, st, work, n, T, nseg, r);
  hipLaunchKernelGGL(seg_total_kernel, dim3(1), dim3(256), 0, st, W, r, n, l, nseg, c);
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(project_update_kernel, dim3((unsigned)(nb * n)), dim3(256), 0, st, W, n, l, nseg, r, c, lambda,
                     full, nb, applied);
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
