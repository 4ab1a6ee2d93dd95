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
                                                      double* __restrict__ p, double* __restrict__ rz,
                                                      const int* __restrict__ stop) {
  __shared__ double red[PT];
  const int64_t s = s0 + blockIdx.x;
  if (stop && stop[s]) return;
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
                                                      const double* __restrict__ rz, double* __restrict__ rr,
                                                      const int* __restrict__ stop, double* __restrict__ alpha) {
  __shared__ double red[PT];
  const int64_t s = s0 + blockIdx.x;
  if (stop && stop[s]) return;
  int64_t off, len;
  segment(seg, n, s, off, len);
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += PT) acc = fma(p[off + i], -nq[off + i], acc);
  const double pq = block_sum(acc, red);
  const double a = (pq > 0.0 && rz[s] > 0.0) ? rz[s] / pq : 0.0;
  if (alpha && threadIdx.x == 0) alpha[s] = a;
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
                                                     double* __restrict__ p, double* __restrict__ rz,
                                                     const int* __restrict__ stop) {
  __shared__ double red[PT];
  const int64_t s = s0 + blockIdx.x;
  if (stop && stop[s]) return;
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

// out[s] = x . x over segment s
__global__ void __launch_bounds__(PT) seg_sumsq_kernel(const int64_t* __restrict__ seg, int64_t n, int64_t s0,
                                                       const double* __restrict__ x, double* __restrict__ out) {
  __shared__ double red[PT];
  const int64_t s = s0 + blockIdx.x;
  int64_t off, len;
  segment(seg, n, s, off, len);
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += PT) acc = fma(x[off + i], x[off + i], acc);
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) out[s] = t;
}

// The stop test of one sweep for every running segment, on the device: rho = sqrt(rr / bb) (the
// relative residual of the current iterate), expect = rho max(floor, min(1, rho / prev)) when
// predicting, else rho; the segment stops when tol > 0 and expect <= tol, or at its sweep cap.
// A stopping segment takes its last correction (y += zc) and records its sweep count.
__global__ void __launch_bounds__(PT) pcg_decide_kernel(const int64_t* __restrict__ seg, int64_t n, int64_t s0, int sweep,
                                                        PcgControl c, const double* __restrict__ zc,
                                                        double* __restrict__ y) {
  const int64_t s = s0 + blockIdx.x;
  if (c.stop[s]) return;
  const double bb = c.bb[s], rr = c.rr[s];
  const double rho = bb > 0.0 ? sqrt(rr / bb) : (rr > 0.0 ? INFINITY : 0.0);
  const double pv = c.prev[s];
  const double ratio = pv > 0.0 ? fmin(1.0, rho / pv) : 0.0;
  const double expect = c.predict ? rho * fmax(c.floor, ratio) : rho;
  const bool met = c.tol > 0.0 && expect <= c.tol;
  const bool last = sweep >= c.cap[s];
  __syncthreads();   // every thread has read the scalars before thread 0 updates them
  if (threadIdx.x == 0) {
    c.prev[s] = rho;
    c.resid[s] = rho;
  }
  if (!(met || last)) return;
  int64_t off, len;
  segment(seg, n, s, off, len);
  if (!c.keep)
    for (int64_t i = threadIdx.x; i < len; i += PT) y[off + i] += zc[off + i];
  if (threadIdx.x == 0) {
    c.stop[s] = 1;
    c.done[s] = sweep;
    c.met[s] = met ? 1 : 0;
  }
}

// stop[s] = (cap[s] < 1), prev = 1, done = 0, resid = -1, met = 0
__global__ void pcg_control_init_kernel(int64_t nseg, PcgControl c) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  c.stop[s] = c.cap[s] < 1 ? 1 : 0;
  c.prev[s] = 1.0;
  c.done[s] = 0;
  c.resid[s] = -1.0;
  c.met[s] = 0;
}

}  // namespace

hipError_t seg_sumsq(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, const double* x, double* out,
                     hipStream_t st) {
  if (s1 <= s0) return hipSuccess;
  hipLaunchKernelGGL(seg_sumsq_kernel, dim3((unsigned)(s1 - s0)), dim3(PT), 0, st, seg, n, s0, x, out);
  return hipGetLastError();
}

hipError_t pcg_decide(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, int sweep, const PcgControl& c,
                      const double* zc, double* y, hipStream_t st) {
  if (s1 <= s0) return hipSuccess;
  hipLaunchKernelGGL(pcg_decide_kernel, dim3((unsigned)(s1 - s0)), dim3(PT), 0, st, seg, n, s0, sweep, c, zc, y);
  return hipGetLastError();
}

hipError_t pcg_control_init(int64_t nseg, const PcgControl& c, hipStream_t st) {
  if (nseg < 1) return hipSuccess;
  hipLaunchKernelGGL(pcg_control_init_kernel, dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, st, nseg, c);
  return hipGetLastError();
}

hipError_t pcg_init(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, const double* r, const double* z, double* p,
                    double* rz, hipStream_t st, const int* stop) {
  if (s1 <= s0) return hipSuccess;
  hipLaunchKernelGGL(pcg_init_kernel, dim3((unsigned)(s1 - s0)), dim3(PT), 0, st, seg, n, s0, r, z, p, rz, stop);
  return hipGetLastError();
}

hipError_t pcg_step(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, const double* p, const double* nq, double* y,
                    double* r, const double* rz, double* rr, hipStream_t st, const int* stop, double* alpha) {
  if (s1 <= s0) return hipSuccess;
  hipLaunchKernelGGL(pcg_step_kernel, dim3((unsigned)(s1 - s0)), dim3(PT), 0, st, seg, n, s0, p, nq, y, r, rz, rr,
                     stop, alpha);
  return hipGetLastError();
}

hipError_t pcg_dir(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, const double* r, const double* z, double* p,
                   double* rz, hipStream_t st, const int* stop) {
  if (s1 <= s0) return hipSuccess;
  hipLaunchKernelGGL(pcg_dir_kernel, dim3((unsigned)(s1 - s0)), dim3(PT), 0, st, seg, n, s0, r, z, p, rz, stop);
  return hipGetLastError();
}

hipError_t pcg_finish(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, const double* z, double* y,
                      hipStream_t st) {
  if (s1 <= s0) return hipSuccess;
  hipLaunchKernelGGL(pcg_finish_kernel, dim3((unsigned)(s1 - s0)), dim3(PT), 0, st, seg, n, s0, z, y);
  return hipGetLastError();
}

}  // namespace dfi
