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

#include <algorithm>

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

// ---------------------------------------------------------------- many vectors (batched call)
// The same final step for nvec vectors at once: the passes carry T_v = S^T y_v per vector (in the
// multi-vector passes' layout, groups of 16 vectors interleaved by column), every vector's last
// correction z_v is taken through the codes as one product C = Z Q (nvec x n times n x m) on the
// bf16 matrix cores: a code times its row's power-of-two scale is exactly a bf16 number, z_v is
// rounded to bf16 (2^-9 relative, far inside the 3 % the codes already cost), and the products
// are summed in FP32.

// Tacc[g][j][c] += alpha[16 g + c] Uacc[g][j][c] for the vectors that exist (16 g + c < nvec)
__global__ void t_axpy_multi_kernel(double* __restrict__ T, const double* __restrict__ U,
                                    const double* __restrict__ alpha, int64_t m, int64_t nvec) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ngroups = (nvec + 15) / 16;
  if (idx >= ngroups * m * 16) return;
  const int64_t g = idx / (m * 16);
  const int c = (int)(idx & 15);
  const int64_t v = g * 16 + c;
  if (v < nvec) T[idx] = fma(alpha[v], U[idx], T[idx]);
}

constexpr int MT = 256;   // multi_decide: one workgroup per vector

__device__ double tree_sum_mt(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = MT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Vector v = blockIdx.x: abar_v, zb_v = bf16(z_v - abar_v) (zeros from n to ldz), use_v as in
// final_decide; y is left alone (the flag kernel decides for all vectors together).
__global__ void __launch_bounds__(MT)
multi_decide_kernel(int64_t n, const double* __restrict__ Y, const double* __restrict__ Z,
                    const double* __restrict__ B, const double* __restrict__ d, const double* __restrict__ lamv,
                    int64_t nrhs, const int* __restrict__ cflag, double est_max, __bf16* __restrict__ zb, int64_t ldz,
                    double* __restrict__ abar, int* __restrict__ usev) {
  __shared__ double red[MT];
  const int64_t v = blockIdx.x;
  const int tid = threadIdx.x;
  const double* y = Y + v * n;
  const double* z = Z + v * n;
  const double* b = B + v * n;
  const double lambda = lamv[v / nrhs];
  const int centered = cflag ? *cflag : 0;
  double s = 0.0;
  if (centered)
    for (int64_t i = tid; i < n; i += MT) s += z[i];
  const double ab = centered ? tree_sum_mt(s, red) / (double)n : 0.0;
  double a = 0.0, yb = 0.0, yy = 0.0;
  for (int64_t i = tid; i < ldz; i += MT) {
    double zp = 0.0;
    if (i < n) {
      zp = z[i] - ab;
      a = fma(d[i] * zp, zp, a);
      yb = fma(y[i], b[i], yb);
      yy = fma(y[i], y[i], yy);
    }
    zb[v * ldz + i] = (__bf16)(float)zp;
  }
  const double A = tree_sum_mt(a, red);
  const double YB = tree_sum_mt(yb, red);
  const double YY = tree_sum_mt(yy, red);
  const double sty = YB - lambda * YY;
  const bool ok = sty > 0.0 && A >= 0.0 && A <= est_max * est_max * sty;
  if (tid == 0) {
    abar[v] = ab;
    usev[v] = ok ? 1 : 0;
  }
}

// flag[0] = 1 when every vector may take the codes (one workgroup)
__global__ void __launch_bounds__(MT) multi_flag_kernel(const int* __restrict__ usev, int64_t nvec,
                                                         int* __restrict__ flag) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int64_t v = threadIdx.x; v < nvec; v += MT)
    if (!usev[v]) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0) flag[0] = bad ? 0 : 1;
}

// Y += Z (every vector) unless flag[0]: the exact passes then take the corrected iterates
__global__ void multi_condaxpy_kernel(double* __restrict__ Y, const double* __restrict__ Z, int64_t len,
                                      const int* __restrict__ flag) {
  if (flag[0]) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) Y[i] += Z[i];
}

struct SmallVals {
  double v[32];
};
__global__ void put_values_kernel(double* __restrict__ out, SmallVals vals, int count) {
  if ((int)threadIdx.x < count) out[threadIdx.x] = vals.v[threadIdx.x];
}

// The product C = Z Q for 128 vectors x BC columns per workgroup, rows in chunks of 64: the
// chunk's bf16 z (128 x 64) and the decoded codes, transposed to column-major (BC x 64, each code
// times its row's scale, exactly a bf16 number), go through LDS; wave w owns vectors 32 w .. 32 w +
// 31 and all BC columns (BC / 32 accumulators of 32 x 32), fed by v_mfma_f32_32x32x16_bf16 with the
// same k assignment for both operands (lanes 0-31 k = kk .. kk + 7, lanes 32-63 k = 16 + kk ..,
// kk = 0, 8 of each 32-row half). Then x_v,j = (V_r,j - T_v,j - abar_v cs_j - C_v,j) / lambda_f.
constexpr int BV = 128, BC = 128, BK = 64, BLD = BK + 8;   // LDS rows of 72 bf16 (144 bytes)
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__global__ void __launch_bounds__(256)
bf16_apply_kernel(const uint8_t* __restrict__ q, const uint8_t* __restrict__ sc, int64_t n, int64_t m, int64_t ldq,
                  const __bf16* __restrict__ zb, int64_t ldz, int64_t nvec, const double* __restrict__ Tacc,
                  const double* __restrict__ Ulast, const double* __restrict__ alpha,
                  const double* __restrict__ cs, const double* __restrict__ abar, const double* __restrict__ lamv,
                  int64_t nrhs, const float* __restrict__ V, int64_t ldv, void* __restrict__ X, int64_t ldx, int x64,
                  const int* __restrict__ use) {
  if (!*use) return;
  __shared__ __align__(16) __bf16 zs[BV * BLD];
  __shared__ __align__(16) __bf16 bt[BC * BLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int64_t j0 = (int64_t)blockIdx.x * BC;
  const int64_t v0 = (int64_t)blockIdx.y * BV;
  f32x16_t acc[BC / 32];
#pragma unroll
  for (int nb = 0; nb < BC / 32; ++nb)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[nb][e] = 0.f;
  // the next chunk's z and codes are loaded into registers while the products of this one run
  constexpr int CQ = BC / 4, OCT = 256 / CQ, NP = BK / 8 / OCT;
  static_assert(BK / 8 % OCT == 0, "the chunk's row octets are a whole number of passes");
  uint4 zn[4];
  uint32_t wn[NP][8], en[NP][8];
  auto load_chunk = [&](int64_t i0) {
    const int v = tid >> 1, hh = tid & 1;   // z: row v of the chunk, 32 bf16 (64 bytes) per thread
    if (v0 + v < nvec) {
      const uint4* src = reinterpret_cast<const uint4*>(zb + (v0 + v) * ldz + i0 + hh * 32);
#pragma unroll
      for (int u = 0; u < 4; ++u) zn[u] = src[u];
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) zn[u] = make_uint4(0u, 0u, 0u, 0u);
    }
    // codes: thread (column quad tid % CQ, row octets tid / CQ + OCT rr), 4 codes and a scale byte per row
    const int64_t jq = j0 + 4 * (tid % CQ);
#pragma unroll
    for (int rr = 0; rr < NP; ++rr)
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t i = i0 + (tid / CQ + OCT * rr) * 8 + r;
        wn[rr][r] = 0u;
        en[rr][r] = 0u;
        if (i < n && jq < ldq) {
          wn[rr][r] = *reinterpret_cast<const uint32_t*>(q + ((jq >> 6) * n + i) * 64 + (jq & 63));
          en[rr][r] = sc[((jq >> 7) * n + i) * 4 + ((jq >> 5) & 3)];
        }
      }
  };
  auto store_chunk = [&]() {
    const int v = tid >> 1, hh = tid & 1;
    uint4* dst = reinterpret_cast<uint4*>(zs + v * BLD + hh * 32);
#pragma unroll
    for (int u = 0; u < 4; ++u) dst[u] = zn[u];
#pragma unroll
    for (int rr = 0; rr < NP; ++rr) {
      const int ro = tid / CQ + OCT * rr;
      float vals[4][8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        // 2^(e - 127), also for e = 0 (rows past n hold zero codes)
        const uint32_t e = en[rr][r];
        const float sf = __uint_as_float(e ? e << 23 : 0x00400000u);
        const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)wn[rr][r], false);
        const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)wn[rr][r], true);
        vals[0][r] = lo[0] * sf;
        vals[1][r] = lo[1] * sf;
        vals[2][r] = hi[0] * sf;
        vals[3][r] = hi[1] * sf;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        bf16x8_t b8;
#pragma unroll
        for (int r = 0; r < 8; ++r) b8[r] = (__bf16)vals[c][r];   // exact: at most 4 significant bits
        *reinterpret_cast<bf16x8_t*>(bt + (4 * (tid % CQ) + c) * BLD + ro * 8) = b8;
      }
    }
  };
  load_chunk(0);
  for (int64_t i0 = 0; i0 < n; i0 += BK) {
    __syncthreads();   // the previous chunk's operands have been read
    store_chunk();
    __syncthreads();
    if (i0 + BK < n) load_chunk(i0 + BK);
#pragma unroll
    for (int kb = 0; kb < BK; kb += 32)
#pragma unroll
      for (int kk = 0; kk < 16; kk += 8) {
        const int ko = kb + half * 16 + kk;
        const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(zs + (32 * wave + l32) * BLD + ko);
#pragma unroll
        for (int nb = 0; nb < BC / 32; ++nb) {
          const bf16x8_t bb = *reinterpret_cast<const bf16x8_t*>(bt + (32 * nb + l32) * BLD + ko);
          acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc[nb], 0, 0, 0);
        }
      }
  }
  // lane l, register r = 4 k + e: vector 8 k + 4 (l / 32) + e of the wave's 32, column l % 32. Its
  // T is entry 8 (k % 2) + 4 (l / 32) + e of column j's 16 in group 2 w + k / 2 (of the block's
  // vectors): the lane reads two 32-byte pieces of each of two 128-byte rows of T.
  const int64_t ngroups = (nvec + 15) / 16;
#pragma unroll
  for (int nb = 0; nb < BC / 32; ++nb) {
    const int64_t j = j0 + 32 * nb + l32;
    if (j >= m) continue;
    const double csj = cs ? cs[j] : 0.0;
    double t16[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t g = (v0 >> 4) + 2 * wave + (k >> 1);
      if (g < ngroups) {
        const int64_t o = (g * m + j) * 16 + 8 * (k & 1) + 4 * half;
        const double2* tp = reinterpret_cast<const double2*>(Tacc + o);
        const double2 a = tp[0], b = tp[1];
        t16[4 * k + 0] = a.x;
        t16[4 * k + 1] = a.y;
        t16[4 * k + 2] = b.x;
        t16[4 * k + 3] = b.y;
        if (Ulast) {   // the last direction's S^T p, not yet added: T + alpha_v U
          const double2* up = reinterpret_cast<const double2*>(Ulast + o);
          const double2 ua = up[0], ub = up[1];
          const int64_t vb = 16 * g + 8 * (k & 1) + 4 * half;
          t16[4 * k + 0] = fma(alpha[min(vb + 0, nvec - 1)], ua.x, t16[4 * k + 0]);
          t16[4 * k + 1] = fma(alpha[min(vb + 1, nvec - 1)], ua.y, t16[4 * k + 1]);
          t16[4 * k + 2] = fma(alpha[min(vb + 2, nvec - 1)], ub.x, t16[4 * k + 2]);
          t16[4 * k + 3] = fma(alpha[min(vb + 3, nvec - 1)], ub.y, t16[4 * k + 3]);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) t16[4 * k + e] = 0.0;
      }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t v = v0 + 32 * wave + 8 * (r >> 2) + 4 * half + (r & 3);
      if (v >= nvec) continue;
      const double t = t16[r];
      const double xv = ((double)V[(v % nrhs) * ldv + j] - t - abar[v] * csj - (double)acc[nb][r]) / lamv[v / nrhs];
      if (x64) static_cast<double*>(X)[v * ldx + j] = xv;
      else static_cast<float*>(X)[v * ldx + j] = (float)xv;
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


hipError_t t_axpy_multi(double* T, const double* U, const double* alpha, int64_t m, int64_t nvec, hipStream_t st) {
  const int64_t tot = (nvec + 15) / 16 * m * 16;
  hipLaunchKernelGGL(t_axpy_multi_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, T, U, alpha, m, nvec);
  return hipGetLastError();
}

hipError_t put_values(double* out, const double* vals, int64_t count, hipStream_t st) {
  for (int64_t c0 = 0; c0 < count; c0 += 32) {
    SmallVals sv{};
    const int k = (int)std::min<int64_t>(32, count - c0);
    for (int i = 0; i < k; ++i) sv.v[i] = vals[c0 + i];
    hipLaunchKernelGGL(put_values_kernel, dim3(1), dim3(32), 0, st, out + c0, sv, k);
  }
  return hipGetLastError();
}

hipError_t multi_final8(const uint8_t* q, const uint8_t* sc, int64_t ldq, int64_t n, int64_t m, int64_t nvec,
                        int64_t nrhs, double* Y, const double* Z, const double* B, const double* d,
                        const double* lamv, const int* centered, double est_max, void* zbv, int64_t ldz,
                        double* abar, int* usev, int* flag, const double* Tacc, const double* Ulast,
                        const double* alpha, const double* cs, const float* V, int64_t ldv, void* X, int64_t ldx,
                        int x64, hipStream_t st) {
  if ((ldq & 127) != 0 || ldq < m || ldz < n || (ldz & 63) != 0 || nvec < 1 || nvec > 65535 * (int64_t)BV)
    return hipErrorInvalidValue;
  __bf16* zb = static_cast<__bf16*>(zbv);
  hipLaunchKernelGGL(multi_decide_kernel, dim3((unsigned)nvec), dim3(MT), 0, st, n, Y, Z, B, d, lamv, nrhs, centered,
                     est_max, zb, ldz, abar, usev);
  hipLaunchKernelGGL(multi_flag_kernel, dim3(1), dim3(MT), 0, st, usev, nvec, flag);
  const int64_t len = nvec * n;
  hipLaunchKernelGGL(multi_condaxpy_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, Y, Z, len, flag);
  const dim3 grid((unsigned)((m + BC - 1) / BC), (unsigned)((nvec + BV - 1) / BV));
  hipLaunchKernelGGL(bf16_apply_kernel, grid, dim3(256), 0, st, q, sc, n, m, ldq, (const __bf16*)zb, ldz, nvec, Tacc,
                     Ulast, alpha, cs, (const double*)abar, lamv, nrhs, V, ldv, X, ldx, x64, (const int*)flag);
  return hipGetLastError();
}

}  // namespace dfi
