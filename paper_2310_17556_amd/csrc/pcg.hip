// Vector steps of the FP64 refinement of W y = b (W = S S^T + lambda I, the n x n system of
// Algorithm 1) as conjugate gradients preconditioned by the factor of the computed Gram,
// M = L L^T ~ W. The product q = W p is matrix-free (one pass over S, elsewhere); these kernels
// do the n-vector work of one iteration: the two inner products, the step along p, the new
// direction. Every inner product is FP64 with a fixed summation order (strided per-thread sums,
// then a tree in LDS), so results do not depend on timing.
//
// Vectors come as segments of one concatenated array: segment s is [off_s, off_s + len_s), with
// off_s = seg[2 s], len_s = seg[2 s + 1] from a device table, or off_s = s * n, len_s = n when
// the table is null. A launch covers segments s0 .. s1 - 1 (one workgroup each); per-
// segment scalars (rz, rr) live at index s.
#include "dfisher_internal.h"

namespace dfi {
namespace {

constexpr int PT = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = PT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void segment(const int64_t* seg, int64_t n, int64_t s, int64_t& off, int64_t& len) {
  if (seg) {
    off = seg[2 * s];
    len = seg[2 * s + 1];
  } else {
    off = s * n;
    len = n;
  }
}

// p = z, rz = r . z
__global__ void __launch_bounds__(PT) pcg_init_kernel(const int64_t* __restrict__ seg, int64_t n, int64_t s0,
                                                      const double* __restrict__ r, const double* __restrict__ z,
                                                      double* __restrict__ p, double* __restrict__ rz) {
  __shared__ double red[PT];
  const int64_t s = s0 + blockIdx.x;
  int64_t off, len;
  segment(seg, n, s, off, len);
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += PT) {
    const double zi = z[off + i];
    p[off + i] = zi;
    acc = fma(r[off + i], zi, acc);
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) rz[s] = t;
}

// nq = -(W p) (as the residual pass with a zero right-hand side delivers it):
// alpha = rz / (p . W p); y += alpha p; r -= alpha W p; rr = r . r (if rr != null).
// A direction with p . W p not > 0 (p = 0 once the residual vanished) takes no step.
__global__ void __launch_bounds__(PT) pcg_step_kernel(const int64_t* __restrict__ seg, int64_t n, int64_t s0,
                                                      const double* __restrict__ p, const double* __restrict__ nq,
                                                      double* __restrict__ y, double* __restrict__ r,
                                                      const double* __restrict__ rz, double* __restrict__ rr) {
  __shared__ double red[PT];
  const int64_t s = s0 + blockIdx.x;
  int64_t off, len;
  segment(seg, n, s, off, len);
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += PT) acc = fma(p[off + i], -nq[off + i], acc);
  const double pq = block_sum(acc, red);
  const double a = (pq > 0.0 && rz[s] > 0.0) ? rz[s] / pq : 0.0;
  double acc2 = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += PT) {
    y[off + i] = fma(a, p[off + i], y[off + i]);
    const double ri = fma(a, nq[off + i], r[off + i]);
    r[off + i] = ri;
    acc2 = fma(ri, ri, acc2);
  }
  if (rr) {
    const double t = block_sum(acc2, red);
    if (threadIdx.x == 0) rr[s] = t;
  }
}

// rz' = r . z; beta = rz' / rz; p = z + beta p; rz = rz'
__global__ void __launch_bounds__(PT) pcg_dir_kernel(const int64_t* __restrict__ seg, int64_t n, int64_t s0,
                                                     const double* __restrict__ r, const double* __restrict__ z,
                                                     double* __restrict__ p, double* __restrict__ rz) {
  __shared__ double red[PT];
  const int64_t s = s0 + blockIdx.x;
  int64_t off, len;
  segment(seg, n, s, off, len);
  const double rzo = rz[s];   // read before the barriers of the sum; thread 0 overwrites it after
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += PT) acc = fma(r[off + i], z[off + i], acc);
  const double rzn = block_sum(acc, red);
  const double b = rzo > 0.0 ? rzn / rzo : 0.0;
  for (int64_t i = threadIdx.x; i < len; i += PT) p[off + i] = fma(b, p[off + i], z[off + i]);
  if (threadIdx.x == 0) rz[s] = rzn;
}

// y += z over the segments (the last correction, z = M^-1 r of the current residual)
__global__ void __launch_bounds__(PT) pcg_finish_kernel(const int64_t* __restrict__ seg, int64_t n, int64_t s0,
                                                        const double* __restrict__ z, double* __restrict__ y) {
  const int64_t s = s0 + blockIdx.x;
  int64_t off, len;
  segment(seg, n, s, off, len);
  for (int64_t i = threadIdx.x; i < len; i += PT) y[off + i] += z[off + i];
}

}  // namespace

hipError_t pcg_init(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, const double* r, const double* z, double* p,
                    double* rz, hipStream_t st) {
  if (s1 <= s0) return hipSuccess;
  hipLaunchKernelGGL(pcg_init_kernel, dim3((unsigned)(s1 - s0)), dim3(PT), 0, st, seg, n, s0, r, z, p, rz);
  return hipGetLastError();
}

hipError_t pcg_step(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, const double* p, const double* nq, double* y,
                    double* r, const double* rz, double* rr, hipStream_t st) {
  if (s1 <= s0) return hipSuccess;
  hipLaunchKernelGGL(pcg_step_kernel, dim3((unsigned)(s1 - s0)), dim3(PT), 0, st, seg, n, s0, p, nq, y, r, rz, rr);
  return hipGetLastError();
}

hipError_t pcg_dir(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, const double* r, const double* z, double* p,
                   double* rz, hipStream_t st) {
  if (s1 <= s0) return hipSuccess;
  hipLaunchKernelGGL(pcg_dir_kernel, dim3((unsigned)(s1 - s0)), dim3(PT), 0, st, seg, n, s0, r, z, p, rz);
  return hipGetLastError();
}

hipError_t pcg_finish(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, const double* z, double* y,
                      hipStream_t st) {
  if (s1 <= s0) return hipSuccess;
  hipLaunchKernelGGL(pcg_finish_kernel, dim3((unsigned)(s1 - s0)), dim3(PT), 0, st, seg, n, s0, z, y);
  return hipGetLastError();
}

}  // namespace dfi
