// Triangular solves with the Cholesky factor L (row-major n x n FP64, lower): the L^-1 and L^-T
// applications of the right-to-left evaluation of S^T L^-T L^-1 S v (Section 2, after Algorithm 1).
//
// Blocked by 64-row blocks, in two parts:
//   * diag_inv: the inverse of every 64 x 64 diagonal block D_k = L_kk^-1 (one workgroup per
//     block, all blocks in parallel; lane c forms column c by forward substitution). For a
//     factorisation this is computed once and reused by every solve.
//   * one launch per two block steps. Forward step k alone would be: every workgroup forms
//     z_k = D_k r_k (a 64 x 64 matrix-vector product; r_k is final because all earlier steps have
//     updated it), workgroup 0 stores z_k, and each workgroup then updates its own 64-row block
//     J > k of the right-hand side, r_J -= L_Jk z_k. A launch takes blocks k and k + 1 together:
//     every workgroup also forms r_{k+1} - L_{k+1,k} z_k and z_{k+1} from it, and the updates
//     subtract both panels. Backward (from the last block): y_k = D_k^T r_k, then r_J -= L_kJ^T y_k
//     for the blocks J < k, which read row block k of L (contiguous rows), likewise two blocks per
//     launch. Every value is formed by the same products in the same order as with one block per
//     launch; a launch costs a few microseconds however little it does, and the solve is a chain
//     of them, so halving their number halves most of its time.
// Every launch reads only the panel it needs; the whole solve reads the lower triangle once.
// Batched form: grid dimension y indexes right-hand sides (vector j at offset j n); vector j uses
// factor j / nper (L + (j / nper) sL, Dinv + (j / nper) sD), so several right-hand sides of one
// factor and several factors share every launch.
#include "dfisher_internal.h"

#include <algorithm>

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
  // the transposed copy after all blocks, for the forward steps' reads (lanes along i)
  double* Dt = Dinv + ((n + NB - 1) / NB + k) * NB * NB;
#pragma unroll
  for (int i = 0; i < NB; ++i) Dt[c * NB + i] = x[i];  // Dt[c][i] = (L_kk^-1)_ic
}

// Forward double step s: blocks a = 2 s and b = 2 s + 1 (b may lie past the last block) in one
// launch. Every workgroup forms z_a = D_a r_a, then r_b - L_ba z_a and z_b = D_b (r_b - L_ba z_a),
// each exactly as the single step of its block would (same products, same order); workgroup 0
// stores z_a and z_b, and workgroup x >= 1 updates row block J = b + x with both panels,
// r_J -= L_Ja z_a, then r_J -= L_Jb z_b. r: right-hand side being reduced in place (FP64, length
// n); z: output. Grid: 1 + number of row blocks below b (at least 1). 256 threads.
__global__ void __launch_bounds__(256)
fwd_step2_kernel(const double* __restrict__ L, int64_t n, const double* __restrict__ Dinv, int64_t s,
                 double* __restrict__ r, double* __restrict__ z, int64_t sL, int64_t sD, int64_t nper,
                 const TrsvJob* __restrict__ jobs) {
  __shared__ double za[NB], zb[NB], rbv[NB];
  __shared__ double part[4][NB];
  __shared__ double lpa[NB * LDP];   // this workgroup's piece of panel a: lpa[i * LDP + c] = L[J NB + i][a NB + c]
  __shared__ double lpb[NB * LDP];   // the same rows of panel b
  double* const lab = lpa;           // L_ba, read before the panel pieces are stored
  if (jobs) {
    const TrsvJob& j = jobs[blockIdx.y];
    L = j.L;
    Dinv = j.Dinv;
    n = j.n;
    r = j.r;
    z = j.out;
  } else {
    const int64_t j = blockIdx.y, f = j / nper;
    L += f * sL;
    Dinv += f * sD;
    r += j * n;
    z += j * n;
  }
  const int64_t nblk = (n + NB - 1) / NB;
  const int64_t a = 2 * s, b = a + 1;
  const bool hasb = b < nblk;
  // grouped launches size the grid for the largest system
  if (a >= nblk || (int64_t)blockIdx.x >= (hasb ? nblk - b : 1)) return;
  const int tid = threadIdx.x;
  const int64_t ra = a * NB, rb = b * NB;
  const int nba = (int)min<int64_t>(NB, n - ra);
  const int nbb = hasb ? (int)min<int64_t>(NB, n - rb) : 0;
  // Every load first: this workgroup's pieces of panels a and b (row block J = b + x), L_ba, D_a,
  // D_b, r_a. Thread (c, g) loads column c of rows 16 g .. 16 g + 15 (512 contiguous bytes of a row
  // per instruction); the pieces go through LDS to the row-wise products.
  const int64_t rowJ = (b + (int64_t)blockIdx.x) * NB;
  const int lc = tid & 63, lg = tid >> 6;
  double va[16], vb[16], vab[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int64_t rw = rowJ + lg * 16 + u;
    const bool own = blockIdx.x > 0 && rw < n;
    va[u] = (own && lc < nba) ? L[rw * n + ra + lc] : 0.0;
    vb[u] = (own && lc < nbb) ? L[rw * n + rb + lc] : 0.0;
    const int64_t rwb = rb + lg * 16 + u;
    vab[u] = (hasb && rwb < n && lc < nba) ? L[rwb * n + ra + lc] : 0.0;
  }
  // the old values of r_b (for row tid / 4 of block b) and of this workgroup's row of block J:
  // nothing in this launch writes them before they are used
  const int64_t rowJt = rowJ + (tid >> 2);
  const double rbold = ((tid >> 2) < nbb) ? r[rb + (tid >> 2)] : 0.0;
  const double rJold = (blockIdx.x > 0 && rowJt < n) ? r[rowJt] : 0.0;
  // z_a = D_a r_a: 4 groups of 64 threads each take 16 columns of D_a (columns past nba read
  // column 0 of r and are skipped), then the sum in column order. D is read from its transposed
  // copy, so that the 64 lanes of a load read one contiguous row.
  const int i = tid & 63, g = tid >> 6;
  const int c0 = g * 16;
  double dva[16], rva[16], dvb[16];
  {
    const double* Dt = Dinv + nblk * NB * NB;
    const double* Da = Dt + a * NB * NB;
    const double* Db = Dt + (hasb ? b : a) * NB * NB;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      dva[u] = Da[(c0 + u) * NB + i];
      rva[u] = r[ra + (c0 + u < nba ? c0 + u : 0)];
      dvb[u] = Db[(c0 + u) * NB + i];
    }
  }
  double sa = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) sa = (c0 + u < nba) ? fma(dva[u], rva[u], sa) : sa;
  part[g][i] = sa;
#pragma unroll
  for (int u = 0; u < 16; ++u) lab[(lg * 16 + u) * LDP + lc] = vab[u];
  __syncthreads();
  if (tid < NB) za[tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
  __syncthreads();
  // r_b - L_ba z_a: 4 threads per row, 16 columns each (block b's update in the single step)
  {
    const int row = tid >> 2, q = tid & 3;
    const double* lr = &lab[row * LDP + q * 16];
    double t = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) t = fma(lr[u], za[q * 16 + u], t);
    t += __shfl_xor(t, 1, 64);
    t += __shfl_xor(t, 2, 64);
    if (q == 0) rbv[row] = rbold - t;
  }
  __syncthreads();
  // z_b = D_b (r_b - L_ba z_a), as z_a
  double sb = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) sb = (c0 + u < nbb) ? fma(dvb[u], rbv[c0 + u], sb) : sb;
  part[g][i] = sb;
  __syncthreads();
  if (tid < NB) zb[tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
  __syncthreads();
  if (blockIdx.x == 0) {
    if (tid < nba) z[ra + tid] = za[tid];
    if (tid < nbb) z[rb + tid] = zb[tid];
    return;
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    lpa[(lg * 16 + u) * LDP + lc] = va[u];
    lpb[(lg * 16 + u) * LDP + lc] = vb[u];
  }
  __syncthreads();
  // r_J -= L_Ja z_a, then r_J -= L_Jb z_b: 4 threads per row, 16 columns each
  const int64_t row = rowJ + (tid >> 2);
  const int q = tid & 3;
  const double* l1 = &lpa[(tid >> 2) * LDP + q * 16];
  const double* l2 = &lpb[(tid >> 2) * LDP + q * 16];
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    s1 = fma(l1[u], za[q * 16 + u], s1);
    s2 = fma(l2[u], zb[q * 16 + u], s2);
  }
  s1 += __shfl_xor(s1, 1, 64);
  s1 += __shfl_xor(s1, 2, 64);
  s2 += __shfl_xor(s2, 1, 64);
  s2 += __shfl_xor(s2, 2, 64);
  if (q == 0 && row < n) {
    double v = rJold;
    v -= s1;
    v -= s2;
    r[row] = v;
  }
}

// Backward double step t: blocks h = nblk - 1 - 2 t and l = h - 1 (l = -1 when h = 0) in one launch,
// counted from each system's own last block. Every workgroup forms y_h = D_h^T r_h, then
// r_l - L_hl^T y_h and y_l = D_l^T (r_l - L_hl^T y_h), each as the single step of its block would;
// workgroup 0 stores y_h and y_l, and workgroup x >= 1 updates block J = x - 1 < l with both,
// r_J -= L_hJ^T y_h, then r_J -= L_lJ^T y_l (row blocks h and l of L: contiguous rows). Grid: 1 + l
// (at least 1). 256 threads.
__global__ void __launch_bounds__(256)
bwd_step2_kernel(const double* __restrict__ L, int64_t n, const double* __restrict__ Dinv, int64_t t,
                 double* __restrict__ r, double* __restrict__ y, int64_t sL, int64_t sD, int64_t nper,
                 const TrsvJob* __restrict__ jobs) {
  __shared__ double yh[NB], yl[NB], rl[NB];
  __shared__ double part[4][NB];
  if (jobs) {
    const TrsvJob& j = jobs[blockIdx.y];
    L = j.L;
    Dinv = j.Dinv;
    n = j.n;
    r = j.r;
    y = j.out;
  } else {
    const int64_t j = blockIdx.y, f = j / nper;
    L += f * sL;
    Dinv += f * sD;
    r += j * n;
    y += j * n;
  }
  const int64_t nblk = (n + NB - 1) / NB;
  const int64_t h = nblk - 1 - 2 * t;
  const int64_t l = h - 1;
  const bool hasl = l >= 0;
  if (h < 0 || (int64_t)blockIdx.x >= (hasl ? 1 + l : 1)) return;
  const int tid = threadIdx.x;
  const int64_t h0 = h * NB, l0 = (hasl ? l : h) * NB;
  const int nbh = (int)min<int64_t>(NB, n - h0);   // block l (< h) is whole
  // Every load first: this workgroup's pieces of row blocks h and l (columns of block J = x - 1;
  // thread (c, g) takes rows 16 g .. 16 g + 15 of column c), L_hl, D_h, D_l, r_h.
  const int64_t J = (int64_t)blockIdx.x - 1;
  const int cc = tid & 63, gg = tid >> 6;
  double vh[16], vl[16], vhl[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int rr = gg * 16 + u;
    vh[u] = (J >= 0 && rr < nbh) ? L[(h0 + rr) * n + J * NB + cc] : 0.0;
    vl[u] = (J >= 0) ? L[(l0 + rr) * n + J * NB + cc] : 0.0;
    vhl[u] = (hasl && rr < nbh) ? L[(h0 + rr) * n + l0 + cc] : 0.0;
  }
  // the old values of r_l and of block J (entry tid < 64): nothing in this launch writes them
  // before they are used
  const double rlold = (hasl && tid < NB) ? r[l0 + tid] : 0.0;
  const double rJold = (J >= 0 && tid < NB) ? r[J * NB + tid] : 0.0;
  // y_h = D_h^T r_h: 4 groups of 64 threads each take 16 columns (columns past nbh read column 0
  // of r and are skipped), then the sum in column order
  const int i = tid & 63, g = tid >> 6;
  const int c0 = g * 16;
  double dvh[16], rvh[16], dvl[16];
  {
    const double* Dh = Dinv + h * NB * NB;
    const double* Dl = Dinv + (hasl ? l : h) * NB * NB;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      dvh[u] = Dh[(c0 + u) * NB + i];
      rvh[u] = r[h0 + (c0 + u < nbh ? c0 + u : 0)];
      dvl[u] = Dl[(c0 + u) * NB + i];
    }
  }
  double s0 = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) s0 = (c0 + u < nbh) ? fma(dvh[u], rvh[u], s0) : s0;
  part[g][i] = s0;
  __syncthreads();
  if (tid < NB) yh[tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
  __syncthreads();
  // r_l - L_hl^T y_h: column c of block l gets sum_i L[h0 + i][l0 + c] y_h[i]
  {
    double tq = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) tq = fma(vhl[u], yh[gg * 16 + u], tq);
    part[gg][cc] = tq;
  }
  __syncthreads();
  if (tid < NB) rl[tid] = rlold - (part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid]);
  __syncthreads();
  // y_l = D_l^T (r_l - L_hl^T y_h) (block l whole: every column counts)
  double s1 = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) s1 = fma(dvl[u], rl[c0 + u], s1);
  part[g][i] = s1;
  __syncthreads();
  if (tid < NB) yl[tid] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
  __syncthreads();
  if (blockIdx.x == 0) {
    if (tid < nbh) y[h0 + tid] = yh[tid];
    if (hasl && tid < NB) y[l0 + tid] = yl[tid];
    return;
  }
  // r_J -= L_hJ^T y_h, then r_J -= L_lJ^T y_l, each as column sums over the block's rows
  double p1 = 0.0, p2 = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    p1 = fma(vh[u], yh[gg * 16 + u], p1);
    p2 = fma(vl[u], yl[gg * 16 + u], p2);
  }
  part[gg][cc] = p1;
  __syncthreads();
  double v = 0.0;
  if (tid < NB) v = rJold - (part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid]);
  __syncthreads();
  part[gg][cc] = p2;
  __syncthreads();
  if (tid < NB) r[J * NB + tid] = v - (part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid]);
}

__global__ void copy_vec_kernel(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

}  // namespace

// Grids of the double steps for a system of nblk blocks: forward step s, 1 + the blocks below
// 2 s + 1; backward step t, 1 + the blocks below nblk - 2 - 2 t.
static int64_t fwd2_grid(int64_t nblk, int64_t s) { return std::max<int64_t>(1, nblk - (2 * s + 1)); }
static int64_t bwd2_grid(int64_t nblk, int64_t t) { return 1 + std::max<int64_t>(0, nblk - 2 - 2 * t); }

// the diagonal-block inverses, then their transposes
size_t trsv_dinv_bytes(int64_t n) { return 2 * (size_t)((n + NB - 1) / NB) * NB * NB * sizeof(double); }

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
    for (int64_t s = 0; 2 * s < nblk; ++s)
      hipLaunchKernelGGL(fwd_step2_kernel, dim3((unsigned)fwd2_grid(nblk, s), nv), dim3(256), 0, st, L, n, Dinv, s, work,
                         y, sL, sD, nper, (const TrsvJob*)nullptr);
  } else {
    for (int64_t t = 0; 2 * t < nblk; ++t)
      hipLaunchKernelGGL(bwd_step2_kernel, dim3((unsigned)bwd2_grid(nblk, t), nv), dim3(256), 0, st, L, n, Dinv, t, work,
                         y, sL, sD, nper, (const TrsvJob*)nullptr);
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
  // every system starts its backward sweep at its own last block, so the largest sets the grids
  if (trans == 0) {
    for (int64_t s = 0; 2 * s < nblk; ++s)
      hipLaunchKernelGGL(fwd_step2_kernel, dim3((unsigned)fwd2_grid(nblk, s), nj), dim3(256), 0, st,
                         (const double*)nullptr, (int64_t)0, (const double*)nullptr, s, (double*)nullptr,
                         (double*)nullptr, (int64_t)0, (int64_t)0, (int64_t)1, jobs_dev);
  } else {
    for (int64_t t = 0; 2 * t < nblk; ++t)
      hipLaunchKernelGGL(bwd_step2_kernel, dim3((unsigned)bwd2_grid(nblk, t), nj), dim3(256), 0, st,
                         (const double*)nullptr, (int64_t)0, (const double*)nullptr, t, (double*)nullptr,
                         (double*)nullptr, (int64_t)0, (int64_t)0, (int64_t)1, jobs_dev);
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
