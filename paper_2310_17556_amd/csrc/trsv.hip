// Triangular solves with the Cholesky factor L (row-major n x n FP64, lower): the L^-1 and L^-T
// applications of the right-to-left evaluation of S^T L^-T L^-1 S v (Section 2, after Algorithm 1).
//
// Blocked by 64-row blocks, in two parts:
//   * diag_inv: the inverse of every 64 x 64 diagonal block D_k = L_kk^-1 (one workgroup per
//     block, all blocks in parallel; lane c forms column c by forward substitution). For a
//     factorisation this is computed once and reused by every solve.
//   * one launch per block step. Forward step k: every workgroup forms z_k = D_k r_k (a 64 x 64
//     matrix-vector product; r_k is final because all earlier steps have updated it), workgroup 0
//     stores z_k, and each workgroup then updates its own 64-row block J > k of the right-hand
//     side, r_J -= L_Jk z_k. Backward step k (from the last block): y_k = D_k^T r_k, then
//     r_J -= L_kJ^T y_k for the blocks J < k, which read row block k of L (contiguous rows).
// Every launch reads only the panel it needs; the whole solve reads the lower triangle once.
// Batched form: grid dimension y indexes right-hand sides (vector j at offset j n); vector j uses
// factor j / nper (L + (j / nper) sL, Dinv + (j / nper) sD), so several right-hand sides of one
// factor and several factors share every launch.
#include "dfisher_internal.h"

namespace dfi {
namespace {

constexpr int NB = 64;
constexpr int LDP = NB + 1;

// D_k = inverse of the lower-triangular 64 x 64 block L_kk (identity-padded past n).
// One 64-lane workgroup per block; lane c computes column c: x_c = e_c, x_i = -(sum_{c<=l<i} L_il x_l)/L_ii.
__global__ void __launch_bounds__(64)
diag_inv_kernel(const double* __restrict__ L, int64_t n, double* __restrict__ Dinv, int64_t sL, int64_t sD,
                const TrsvJob* __restrict__ jobs) {
  __shared__ double Lk[NB * LDP];
  if (jobs) {
    const TrsvJob& j = jobs[blockIdx.y];
    L = j.L;
    Dinv = j.Dinv;
    n = j.n;
    if ((int64_t)blockIdx.x * NB >= n) return;
  } else {
    L += (int64_t)blockIdx.y * sL;
    Dinv += (int64_t)blockIdx.y * sD;
  }
  const int64_t k = blockIdx.x;
  const int64_t r0 = k * NB;
  const int c = threadIdx.x;
  for (int r = 0; r < NB; ++r) {
    double val = 0.0;
    if (r0 + r < n && r0 + c < n) {
      if (c <= r) val = L[(r0 + r) * n + r0 + c];
    } else if (r == c) {
      val = 1.0;
    }
    Lk[r * LDP + c] = val;
  }
  __syncthreads();
  double x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    double s = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int l = 0; l < i; ++l) s -= Lk[i * LDP + l] * x[l];   // x_l = 0 for l < c
    x[i] = (i >= c) ? s / Lk[i * LDP + i] : 0.0;
  }
  double* D = Dinv + k * NB * NB;
#pragma unroll
  for (int i = 0; i < NB; ++i) D[i * NB + c] = x[i];   // D[i][c] = (L_kk^-1)_ic
}

// Forward step k. r: right-hand side being reduced in place (FP64, length n); z: output.
// Grid: 1 + number of row blocks below k (at least 1). 256 threads.
__global__ void __launch_bounds__(256)
fwd_step_kernel(const double* __restrict__ L, int64_t n, const double* __restrict__ Dinv, int64_t k,
                double* __restrict__ r, double* __restrict__ z, int64_t sL, int64_t sD, int64_t nper,
                const TrsvJob* __restrict__ jobs) {
  __shared__ double zk[NB];
  __shared__ double part[4][NB];
  __shared__ double lp[NB * LDP];   // this workgroup's piece of the panel, lp[i * LDP + c] = L[J NB + i][k NB + c]
  if (jobs) {
    const TrsvJob& j = jobs[blockIdx.y];
    L = j.L;
    Dinv = j.Dinv;
    n = j.n;
    r = j.r;
    z = j.out;
    const int64_t nblk = (n + NB - 1) / NB;
    if (k >= nblk || (int64_t)blockIdx.x >= nblk - k) return;   // grid sized for the largest system
  } else {
    const int64_t j = blockIdx.y, f = j / nper;
    L += f * sL;
    Dinv += f * sD;
    r += j * n;
    z += j * n;
  }
  const int tid = threadIdx.x;
  const int64_t r0 = k * NB;
  const int nb = (int)min<int64_t>(NB, n - r0);
  // This workgroup's piece of the panel L_Jk (row block J = k + blockIdx.x) is loaded first: it does
  // not depend on z_k, so its latency overlaps z_k's. Thread (c, g) loads column c of rows
  // 16 g .. 16 g + 15, so each load instruction reads 512 contiguous bytes of one row; the piece
  // goes through LDS to the row-wise products below.
  const int64_t rowJ = (k + blockIdx.x) * NB;
  const int lc = tid & 63, lg = tid >> 6;
  double lv[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int64_t rw = rowJ + lg * 16 + u;
    lv[u] = (blockIdx.x > 0 && rw < n && lc < nb) ? L[rw * n + r0 + lc] : 0.0;
  }
  // z_k = D_k r_k: 4 groups of 64 threads each take 16 columns of D_k (read from its transpose)
  {
    const int i = tid & 63, g = tid >> 6;
    const double* D = Dinv + k * NB * NB;
    double s = 0.0;
    // the 32 loads first (columns past nb read column 0 of r and are skipped), then the sum in
    // column order
    const int c0 = g * 16;
    double dv[16], rv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      dv[u] = D[i * NB + c0 + u];
      rv[u] = r[r0 + (c0 + u < nb ? c0 + u : 0)];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) s = (c0 + u < nb) ? fma(dv[u], rv[u], s) : s;
    part[g][i] = s;
  }
  __syncthreads();
  if (tid < NB) zk[tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
  __syncthreads();
  if (blockIdx.x == 0) {
    if (tid < nb) z[r0 + tid] = zk[tid];
    return;
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) lp[(lg * 16 + u) * LDP + lc] = lv[u];
  __syncthreads();
  // r_J -= L_Jk z_k: 4 threads per row, 16 columns each
  const int64_t row = rowJ + (tid >> 2);
  const int q = tid & 3;
  const double* lr = &lp[(tid >> 2) * LDP + q * 16];
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) s = fma(lr[u], zk[q * 16 + u], s);
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  if (q == 0 && row < n) r[row] -= s;
}

// Backward step k. Grid: 1 + k (block k itself and the blocks J < k). 256 threads.
__global__ void __launch_bounds__(256)
bwd_step_kernel(const double* __restrict__ L, int64_t n, const double* __restrict__ Dinv, int64_t k,
                double* __restrict__ r, double* __restrict__ y, int64_t sL, int64_t sD, int64_t nper,
                const TrsvJob* __restrict__ jobs) {
  __shared__ double yk[NB];
  __shared__ double part[4][NB];
  if (jobs) {
    const TrsvJob& j = jobs[blockIdx.y];
    L = j.L;
    Dinv = j.Dinv;
    n = j.n;
    r = j.r;
    y = j.out;
    if (k >= (n + NB - 1) / NB) return;   // this system's backward sweep starts at its own last block
  } else {
    const int64_t j = blockIdx.y, f = j / nper;
    L += f * sL;
    Dinv += f * sD;
    r += j * n;
    y += j * n;
  }
  const int tid = threadIdx.x;
  const int64_t r0 = k * NB;
  const int nb = (int)min<int64_t>(NB, n - r0);
  // This workgroup's piece of row block k of L (columns of block J = blockIdx.x - 1; thread (c, g)
  // takes rows 16 g .. 16 g + 15 of column c), loaded before y_k so the two latencies overlap.
  const int64_t J = (int64_t)blockIdx.x - 1;
  const int cc = tid & 63, gg = tid >> 6;
  double lv[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) lv[u] = (J >= 0 && gg * 16 + u < nb) ? L[(r0 + gg * 16 + u) * n + J * NB + cc] : 0.0;
  // y_k = D_k^T r_k
  {
    const int i = tid & 63, g = tid >> 6;
    const double* D = Dinv + k * NB * NB;
    double s = 0.0;
    // the 32 loads first (columns past nb read column 0 of r and are skipped), then the sum in
    // column order
    const int c0 = g * 16;
    double dv[16], rv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      dv[u] = D[(c0 + u) * NB + i];
      rv[u] = r[r0 + (c0 + u < nb ? c0 + u : 0)];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) s = (c0 + u < nb) ? fma(dv[u], rv[u], s) : s;
    part[g][i] = s;
  }
  __syncthreads();
  if (tid < NB) yk[tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
  __syncthreads();
  if (blockIdx.x == 0) {
    if (tid < nb) y[r0 + tid] = yk[tid];
    return;
  }
  // r_J -= L_kJ^T y_k for J = blockIdx.x - 1 < k: column c of block J gets sum_i L[r0+i][J*64+c] y_k[i]
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) s = fma(lv[u], yk[gg * 16 + u], s);
  __syncthreads();
  part[gg][cc] = s;
  __syncthreads();
  if (tid < NB) r[J * NB + tid] -= part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
}

__global__ void copy_vec_kernel(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

}  // namespace

size_t trsv_dinv_bytes(int64_t n) { return (size_t)((n + NB - 1) / NB) * NB * NB * sizeof(double); }

hipError_t trsv_diag_inv_batched(const double* L, int64_t sL, int64_t n, int64_t nfac, double* Dinv, hipStream_t st) {
  if (nfac < 1 || nfac > 65535) return hipErrorInvalidValue;
  const int64_t nblk = (n + NB - 1) / NB;
  hipLaunchKernelGGL(diag_inv_kernel, dim3((unsigned)nblk, (unsigned)nfac), dim3(64), 0, st, L, n, Dinv, sL,
                     (int64_t)(trsv_dinv_bytes(n) / sizeof(double)), (const TrsvJob*)nullptr);
  return hipGetLastError();
}

hipError_t trsv_diag_inv(const double* L, int64_t n, double* Dinv, hipStream_t st) {
  return trsv_diag_inv_batched(L, n * n, n, 1, Dinv, st);
}

hipError_t trsv_launch_batched(const double* L, int64_t sL, const double* Dinv, int64_t n, int64_t nvec, int64_t nper,
                               int trans, const double* b, double* y, double* work, hipStream_t st) {
  if (nvec < 1 || nvec > 65535 || nper < 1) return hipErrorInvalidValue;
  const int64_t nblk = (n + NB - 1) / NB;
  const int64_t sD = (int64_t)(trsv_dinv_bytes(n) / sizeof(double));
  const unsigned nv = (unsigned)nvec;
  const int64_t tot = n * nvec;
  hipLaunchKernelGGL(copy_vec_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, b, work, tot);
  if (trans == 0) {
    for (int64_t k = 0; k < nblk; ++k)
      hipLaunchKernelGGL(fwd_step_kernel, dim3((unsigned)(nblk - k), nv), dim3(256), 0, st, L, n, Dinv, k, work, y, sL,
                         sD, nper, (const TrsvJob*)nullptr);
  } else {
    for (int64_t k = nblk - 1; k >= 0; --k)
      hipLaunchKernelGGL(bwd_step_kernel, dim3((unsigned)(k + 1), nv), dim3(256), 0, st, L, n, Dinv, k, work, y, sL,
                         sD, nper, (const TrsvJob*)nullptr);
  }
  return hipGetLastError();
}

hipError_t trsv_diag_inv_grouped(const TrsvJob* jobs_dev, int64_t njobs, int64_t nmax, hipStream_t st) {
  if (njobs < 1 || njobs > 65535) return hipErrorInvalidValue;
  const int64_t nblk = (nmax + NB - 1) / NB;
  hipLaunchKernelGGL(diag_inv_kernel, dim3((unsigned)nblk, (unsigned)njobs), dim3(64), 0, st, (const double*)nullptr,
                     (int64_t)0, (double*)nullptr, (int64_t)0, (int64_t)0, jobs_dev);
  return hipGetLastError();
}

hipError_t trsv_launch_grouped(const TrsvJob* jobs_dev, int64_t njobs, int64_t nmax, int trans, hipStream_t st) {
  if (njobs < 1 || njobs > 65535) return hipErrorInvalidValue;
  const int64_t nblk = (nmax + NB - 1) / NB;
  const unsigned nj = (unsigned)njobs;
  if (trans == 0) {
    for (int64_t k = 0; k < nblk; ++k)
      hipLaunchKernelGGL(fwd_step_kernel, dim3((unsigned)(nblk - k), nj), dim3(256), 0, st, (const double*)nullptr,
                         (int64_t)0, (const double*)nullptr, k, (double*)nullptr, (double*)nullptr, (int64_t)0,
                         (int64_t)0, (int64_t)1, jobs_dev);
  } else {
    for (int64_t k = nblk - 1; k >= 0; --k)
      hipLaunchKernelGGL(bwd_step_kernel, dim3((unsigned)(k + 1), nj), dim3(256), 0, st, (const double*)nullptr,
                         (int64_t)0, (const double*)nullptr, k, (double*)nullptr, (double*)nullptr, (int64_t)0,
                         (int64_t)0, (int64_t)1, jobs_dev);
  }
  return hipGetLastError();
}

// y = L^-1 b (trans = 0) or L^-T b (trans = 1). work: n doubles (the reduced right-hand side).
// b may alias y; work must not alias either.
hipError_t trsv_launch(const double* L, const double* Dinv, int64_t n, int trans, const double* b, double* y,
                       double* work, hipStream_t st) {
  return trsv_launch_batched(L, n * n, Dinv, n, 1, 1, trans, b, y, work, st);
}

}  // namespace dfi
