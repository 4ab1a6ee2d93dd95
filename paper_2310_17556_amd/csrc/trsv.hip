// Triangular solves with the Cholesky factor L (row-major n x n FP64, lower): the L^-1 and L^-T
// applications of the right-to-left evaluation of S^T L^-T L^-1 S v (Section 2, after Algorithm 1).
//
// One workgroup of 1024 threads (16 waves) walks 64-row blocks. For each block:
//   * the off-diagonal contribution is a dense product over the already solved part, spread over
//     all 16 waves (forward: row dot products, lanes striding the row; backward: the rows below
//     the block, each lane owning one column of the block);
//   * the 64 x 64 diagonal triangle is solved by one wave with register broadcasts (__shfl),
//     its coefficients staged in LDS.
// The solution vector lives in LDS, so n is limited by LDS capacity (TRSV_MAX_N).
#include "dfisher_internal.h"

namespace dfi {
namespace {

constexpr int NB = 64;
constexpr int LDP = NB + 1;
constexpr int NW = 16;  // waves

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// y = L^-1 b
__global__ void __launch_bounds__(64 * NW)
trsv_fwd_kernel(const double* __restrict__ L, int64_t n, const double* b, double* y) {
  extern __shared__ double sm[];
  double* z = sm;               // n
  double* rhs = z + n;          // NB
  double* D = rhs + NB;         // NB * LDP
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t nblk = (n + NB - 1) / NB;
  for (int64_t kb = 0; kb < nblk; ++kb) {
    const int64_t r0 = kb * NB;
    const int nb = (int)min<int64_t>(NB, n - r0);
    // rhs_i = b_i - sum_{c < r0} L_ic z_c ; wave w takes rows w, w + 16, ...
    for (int r = wave; r < nb; r += NW) {
      const double* Lr = L + (r0 + r) * n;
      double acc = 0.0;
      for (int64_t c = lane; c < r0; c += 64) acc = fma(Lr[c], z[c], acc);
      acc = wave_sum(acc);
      if (lane == 0) rhs[r] = b[r0 + r] - acc;
    }
    // diagonal block into LDS
    for (int idx = threadIdx.x; idx < NB * NB; idx += 64 * NW) {
      const int r = idx / NB, c = idx % NB;
      D[r * LDP + c] = (r < nb && c <= r) ? L[(r0 + r) * n + r0 + c] : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
      double val = (lane < nb) ? rhs[lane] : 0.0;
      double zi = 0.0;
      for (int c = 0; c < nb; ++c) {
        const double zc = __shfl(val / D[lane * LDP + lane], c, 64);
        if (lane == c) zi = zc;
        if (lane > c) val = fma(-D[lane * LDP + c], zc, val);
      }
      if (lane < nb) {
        z[r0 + lane] = zi;
      }
    }
    __syncthreads();
  }
  for (int64_t i = threadIdx.x; i < n; i += 64 * NW) y[i] = z[i];
}

// y = L^-T b : y_i = (b_i - sum_{k > i} L_ki y_k) / L_ii, blocks from the last to the first.
__global__ void __launch_bounds__(64 * NW)
trsv_bwd_kernel(const double* __restrict__ L, int64_t n, const double* b, double* y) {
  extern __shared__ double sm[];
  double* z = sm;               // n (solution)
  double* part = z + n;         // NW * NB
  double* D = part + NW * NB;   // NB * LDP
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t nblk = (n + NB - 1) / NB;
  for (int64_t kb = nblk - 1; kb >= 0; --kb) {
    const int64_t r0 = kb * NB;
    const int nb = (int)min<int64_t>(NB, n - r0);
    const int64_t rend = r0 + nb;
    // part_w[j] = sum over rows k >= rend handled by wave w of L_k,(r0+j) z_k
    double acc = 0.0;
    if (lane < nb) {
      for (int64_t k = rend + wave; k < n; k += NW) acc = fma(L[k * n + r0 + lane], z[k], acc);
    }
    part[wave * NB + lane] = acc;
    for (int idx = threadIdx.x; idx < NB * NB; idx += 64 * NW) {
      const int r = idx / NB, c = idx % NB;
      D[r * LDP + c] = (r < nb && c <= r) ? L[(r0 + r) * n + r0 + c] : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
      double s = 0.0;
      for (int w = 0; w < NW; ++w) s += part[w * NB + lane];
      double val = (lane < nb) ? b[r0 + lane] - s : 0.0;
      double yi = 0.0;
      for (int c = nb - 1; c >= 0; --c) {
        const double yc = __shfl(val / D[lane * LDP + lane], c, 64);
        if (lane == c) yi = yc;
        if (lane < c) val = fma(-D[c * LDP + lane], yc, val);
      }
      if (lane < nb) z[r0 + lane] = yi;
    }
    __syncthreads();
  }
  for (int64_t i = threadIdx.x; i < n; i += 64 * NW) y[i] = z[i];
}

}  // namespace

size_t trsv_lds_bytes(int64_t n, int trans) {
  return (size_t)(n + (trans ? NW * NB : NB) + NB * LDP) * sizeof(double);
}

// The solves keep the solution vector in LDS; allow up to the full 160 KB of a CDNA4 CU.
hipError_t trsv_prepare() {
  const int bytes = 160 * 1024;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&trsv_fwd_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&trsv_bwd_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t trsv_launch(const double* L, int64_t n, int trans, const double* b, double* y, hipStream_t st) {
  const size_t shm = trsv_lds_bytes(n, trans);
  if (trans == 0)
    hipLaunchKernelGGL(trsv_fwd_kernel, dim3(1), dim3(64 * NW), shm, st, L, n, b, y);
  else
    hipLaunchKernelGGL(trsv_bwd_kernel, dim3(1), dim3(64 * NW), shm, st, L, n, b, y);
  return hipGetLastError();
}

}  // namespace dfi
