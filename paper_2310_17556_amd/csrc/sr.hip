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
// refinement still works with the exact W, so only its convergence changes.
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

// r[s n + i] = sum over j in segment s (nseg <= 2: s = [j >= l]) of W_ij, W symmetric and read from its lower
// triangle: row i up to the diagonal, then column i below it. A workgroup takes 64 rows; wave w
// sums rows i0 + w, i0 + w + 4, ... along the row (lanes strided, then a fixed butterfly), and all
// four waves read the column strip below (thread t: column i0 + t % 64, every fourth row from
// i0 + 1 + t / 64), combined in a fixed order.
__global__ void __launch_bounds__(256) seg_rowsum_kernel(const double* __restrict__ W, int64_t n, int64_t l, int nseg,
                                                         double* __restrict__ r) {
  __shared__ double part[4][64][2];
  __shared__ double rowp[64][2];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  for (int k = wave; k < 64; k += 4) {
    const int64_t i = i0 + k;
    double a0 = 0.0, a1 = 0.0;
    if (i < n) {
      for (int64_t j = lane; j <= i; j += 64) {
        const double w = W[i * n + j];
        if (j < l) a0 += w; else a1 += w;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off);
      a1 += __shfl_xor(a1, off);
    }
    if (lane == 0) {
      rowp[k][0] = a0;
      rowp[k][1] = a1;
    }
  }
  const int64_t c = i0 + lane;
  double b0 = 0.0, b1 = 0.0;
  if (c < n) {
    for (int64_t j = i0 + 1 + wave; j < n; j += 4) {
      if (j <= c) continue;
      const double w = W[j * n + c];
      if (j < l) b0 += w; else b1 += w;
    }
  }
  part[wave][lane][0] = b0;
  part[wave][lane][1] = b1;
  __syncthreads();
  if (wave == 0 && c < n) {
    for (int s = 0; s < nseg; ++s) {
      const double v = rowp[lane][s] + ((part[0][lane][s] + part[1][lane][s]) + (part[2][lane][s] + part[3][lane][s]));
      r[(int64_t)s * n + c] = v;
    }
  }
}

// c[s nseg + u] = sum over i in segment s of r[u n + i], one workgroup, fixed order
__global__ void __launch_bounds__(256) seg_total_kernel(const double* __restrict__ r, int64_t n, int64_t l, int nseg,
                                                        double* __restrict__ c) {
  __shared__ double red[256];
  for (int s = 0; s < nseg; ++s)
    for (int u = 0; u < nseg; ++u) {
      double acc = 0.0;
      for (int64_t i = threadIdx.x; i < l; i += 256) acc += r[(int64_t)u * n + (int64_t)s * l + i];
      red[threadIdx.x] = acc;
      __syncthreads();
      for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
      }
      if (threadIdx.x == 0) c[s * nseg + u] = red[0];
      __syncthreads();
    }
}

// W <- M entrywise (lower triangle, or both when full)
__global__ void __launch_bounds__(256) project_update_kernel(double* __restrict__ W, int64_t n, int64_t l, int nseg,
                                                             const double* __restrict__ r, const double* __restrict__ c,
                                                             double lambda, int full, int64_t nb) {
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

hipError_t gram_project(double* W, int64_t n, int nseg, double lambda, int full, double* r, double* c,
                        hipStream_t st) {
  if (n < 1 || nseg < 1 || nseg > 2 || n % nseg != 0) return hipErrorInvalidValue;
  const int64_t l = n / nseg;
  hipLaunchKernelGGL(seg_rowsum_kernel, dim3(blocks(n, 64)), dim3(256), 0, st, W, n, l, nseg, r);
  hipLaunchKernelGGL(seg_total_kernel, dim3(1), dim3(256), 0, st, r, n, l, nseg, c);
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(project_update_kernel, dim3((unsigned)(nb * n)), dim3(256), 0, st, W, n, l, nseg, r, c, lambda,
                     full, nb);
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
