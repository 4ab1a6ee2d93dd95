// HBM-streaming passes over S for the right-to-left evaluation of x = (v - S^T L^-T L^-1 S v)/lambda
// (Section 2, the inlined form of Algorithm 1 steps 3-4). Every pass reads S exactly once with
// 16-byte loads; products of FP32 values are accumulated in FP64.
//
// Row pass   b = S v (and/or the exact squared row norms d_i = |s_i|^2, the diagonal of S S^T).
//            A wave owns RPW rows and a group of columns; it walks the group in sub-chunks of
//            2048 columns (8 x 16-byte loads per lane, each load covering 1 KB of one row),
//            keeps the sub-chunk of v in registers and reuses it for all RPW rows, and keeps one
//            FP64 accumulator per row per lane. At the end each row is reduced across the wave
//            and one FP64 partial per (row, column group) is stored; a second kernel adds the
//            column groups in fixed order.
// Column pass t = S^T y. A workgroup owns 1024 consecutive columns (one float4 per lane) and
//            walks the rows; y_i is wave-uniform. When m is small the rows are split across
//            workgroups and FP64 partials are added in fixed order by a finalize kernel.
#include "dfisher_internal.h"

#include <cstdlib>

#include <algorithm>

namespace dfi {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int RP_WAVES = 4;     // waves per workgroup (each its own row group)
constexpr int RP_RPW = 8;       // rows per wave (few enough registers for 4 waves per SIMD)
constexpr int RP_U = 8;         // float4 loads per lane per row and sub-chunk
constexpr int RP_SUB = 64 * 4 * RP_U;  // 2048 columns per sub-chunk

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Block scale exponent of the scaled-FP8 form: the smallest e with amax <= 448 * 2^e, clamped to
// [-127, 127] (e = -127 for amax == 0). With amax = f 2^E, 1 <= f < 2: amax <= 1.75 * 2^(8+e)
// holds for e = E - 8 when f <= 1.75, else e = E - 7. Exact, from the FP32 bit pattern.
__device__ __forceinline__ int mx_scale_exp(float amax) {
  const uint32_t u = __float_as_uint(amax);
  const int ebits = (int)((u >> 23) & 0xFF);
  if (ebits == 0) return -127;                       // zero or FP32-subnormal block maximum
  const int E = ebits - 127;
  const uint32_t mant = u & 0x7FFFFF;
  int e = E - 8 + ((mant > 0x600000u) ? 1 : 0);       // 1.75 = 1 + 0x600000 / 2^23
  return e < -127 ? -127 : (e > 127 ? 127 : e);
}

// 2^-e as a float, for e in [-127, 127] (2^127 is the largest; 2^-127 is an FP32 subnormal).
__device__ __forceinline__ float pow2_neg(int e) { return ldexpf(1.0f, -e); }

// Four consecutive vector entries; an FP32 vector stays FP32 (widened where it is used).
template <typename VT>
struct Vec4;
template <>
struct Vec4<float> {
  f32x4 x;
};
template <>
struct Vec4<double> {
  double x[4];
};

template <typename VT>
__device__ __forceinline__ void load_vec4(const VT* __restrict__ v, int64_t col, int64_t m, bool vec, Vec4<VT>& out) {
  if constexpr (sizeof(VT) == 4) {
    if (vec && col + 4 <= m) {
      out.x = *reinterpret_cast<const f32x4*>(v + col);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) out.x[e] = (col + e < m) ? v[col + e] : 0.f;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) out.x[e] = (col + e < m) ? v[col + e] : 0.0;
  }
}

__device__ __forceinline__ void load_s4(const float* __restrict__ p, int64_t col, int64_t m, bool vec, f32x4& out) {
  if (vec && col + 4 <= m) {
    out = *reinterpret_cast<const f32x4*>(p);
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e] = (col + e < m) ? p[e] : 0.f;
  }
}

// Grid: x = row blocks of RP_WAVES * RP_RPW rows, y = column groups of `cg` columns (multiple
// of RP_SUB). part layout: part_b[g * n + i], part_d[(ngroups + g) * n + i].
// QM = 1 also writes the scaled-FP8 form of S, row-major, for every column k < ldq (zero input
// beyond m; needs the vectorised path): codes q[i * ldq + k] (E4M3, round to nearest even) and
// scale exponents sc[i * (ldq / 32) + k / 32] (E8M0 byte e + 127) per 32-column block; a block is
// 8 consecutive lanes of one 16-byte load. (The Gram's column-blocked operands come from
// rowpass_prep_kernel.)
template <typename VT, bool WANT_B, bool WANT_D, int QM>
__global__ void __launch_bounds__(64 * RP_WAVES)
rowpass_kernel(const float* __restrict__ S, int64_t n, int64_t m, int64_t lds, const VT* __restrict__ v,
               int64_t cg, int64_t ngroups, double* __restrict__ part, int vec, uint8_t* __restrict__ q,
               uint8_t* __restrict__ sc, int64_t ldq) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = ((int64_t)blockIdx.x * RP_WAVES + wave) * RP_RPW;
  const int64_t g = blockIdx.y;
  const int64_t c0 = g * cg;
  const int64_t c1 = min(m, c0 + cg);
  if (row0 >= n) return;
  const int nr = (int)min<int64_t>(RP_RPW, n - row0);

  double ab[RP_RPW], ad[RP_RPW];
#pragma unroll
  for (int r = 0; r < RP_RPW; ++r) { ab[r] = 0.0; ad[r] = 0.0; }

  for (int64_t cs = c0; cs < c1; cs += RP_SUB) {
    Vec4<VT> vv[RP_U];
    if constexpr (WANT_B) {
#pragma unroll
      for (int u = 0; u < RP_U; ++u) load_vec4<VT>(v, cs + 256 * u + 4 * lane, c1, (vec & 2) != 0, vv[u]);
    }
#pragma unroll
    for (int r = 0; r < RP_RPW; ++r) {
      if (r < nr) {
        const float* rowp = S + (row0 + r) * lds;
        f32x4 sv[RP_U];
#pragma unroll
        for (int u = 0; u < RP_U; ++u) {
          const int64_t col = cs + 256 * u + 4 * lane;
          load_s4(rowp + col, col, c1, (vec & 1) != 0, sv[u]);
        }
#pragma unroll
        for (int u = 0; u < RP_U; ++u)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const double s = (double)sv[u][e];
            if constexpr (WANT_B) ab[r] = fma(s, (double)vv[u].x[e], ab[r]);
            if constexpr (WANT_D) ad[r] = fma(s, s, ad[r]);
          }
        if constexpr (QM == 1) {
#pragma unroll
          for (int u = 0; u < RP_U; ++u) {
            const int64_t col = cs + 256 * u + 4 * lane;
            float amax = fmaxf(fmaxf(fabsf(sv[u][0]), fabsf(sv[u][1])), fmaxf(fabsf(sv[u][2]), fabsf(sv[u][3])));
            amax = fmaxf(amax, __shfl_xor(amax, 1, 64));
            amax = fmaxf(amax, __shfl_xor(amax, 2, 64));
            amax = fmaxf(amax, __shfl_xor(amax, 4, 64));
            const int ex = mx_scale_exp(amax);
            const float inv = pow2_neg(ex);
            // |sv * inv| <= 448 by the choice of ex; the conversion rounds to nearest even
            int packed = __builtin_amdgcn_cvt_pk_fp8_f32(sv[u][0] * inv, sv[u][1] * inv, 0, false);
            packed = __builtin_amdgcn_cvt_pk_fp8_f32(sv[u][2] * inv, sv[u][3] * inv, packed, true);
            if (col < ldq) {
              *reinterpret_cast<int*>(q + (row0 + r) * ldq + col) = packed;
              if ((lane & 7) == 0) sc[(row0 + r) * (ldq >> 5) + (col >> 5)] = (uint8_t)(ex + 127);
            }
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RP_RPW; ++r) {
    if (r < nr) {
      if constexpr (WANT_B) {
        const double t = wave_sum(ab[r]);
        if (lane == 0) part[g * n + row0 + r] = t;
      }
      if constexpr (WANT_D) {
        const double t = wave_sum(ad[r]);
        if (lane == 0) part[(ngroups + g) * n + row0 + r] = t;
      }
    }
  }
}

// b_i = sum_g part_b[g][i] (or r0_i - lam y_i - sum_g part_b[g][i]); d_i = sum_g part_d[g][i].
// 16 rows and 16 group lanes per 256-thread workgroup: lane s adds groups s, s + 16, ... in order,
// and the 16 lane sums are combined by a fixed pairwise tree in LDS (many groups at small n).
__device__ __forceinline__ void reduce_body(const double* __restrict__ part, int64_t n, int64_t ngroups, int want_b,
                                            int want_d, double* __restrict__ b, double* __restrict__ d,
                                            const double* __restrict__ r0, const double* __restrict__ y, double lam,
                                            const int* __restrict__ skip, int64_t blk) {
  __shared__ double red[2][16][17];
  if (skip && *skip) return;   // a problem whose refinement has stopped (uniform)
  const int tid = threadIdx.x;
  const int ri = tid & 15, sl = tid >> 4;
  const int64_t i = blk * 16 + ri;
  double sb = 0.0, sd = 0.0;
  if (i < n) {
    for (int64_t g = sl; g < ngroups; g += 16) {
      if (want_b) sb += part[g * n + i];
      if (want_d) sd += part[(ngroups + g) * n + i];
    }
  }
  red[0][sl][ri] = sb;
  red[1][sl][ri] = sd;
  __syncthreads();
#pragma unroll
  for (int w = 8; w > 0; w >>= 1) {
    if (sl < w) {
      red[0][sl][ri] += red[0][sl + w][ri];
      red[1][sl][ri] += red[1][sl + w][ri];
    }
    __syncthreads();
  }
  if (sl == 0 && i < n) {
    if (want_b) b[i] = r0 ? (r0[i] - lam * y[i]) - red[0][0][ri] : red[0][0][ri];
    if (want_d) d[i] = red[1][0][ri];
  }
}

__global__ void __launch_bounds__(256)
rowpass_reduce_kernel(const double* __restrict__ part, int64_t n, int64_t ngroups, int want_b, int want_d,
                      double* __restrict__ b, double* __restrict__ d, const double* __restrict__ r0,
                      const double* __restrict__ y, double lam, const int* __restrict__ skip) {
  reduce_body(part, n, ngroups, want_b, want_d, b, d, r0, y, lam, skip, blockIdx.x);
}

// The refinement residuals of many problems in one launch: job j owns blocks [blk0_j, blk0_j +
// ceil(n_j / 16)) and forms out = rhs - lam u - sum over its workgroups' partials, as
// refine_pass_reduce does for one problem.
__global__ void __launch_bounds__(256)
refine_reduce_grouped_kernel(const ReduceJob* __restrict__ jobs, int njobs) {
  const int64_t w = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].blk0 <= w) lo = mid;
    else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  const ReduceJob& j = jobs[lo];
  const int64_t bl = w - j.blk0;
  if (bl < 0 || bl * 16 >= j.n) return;
  reduce_body(j.part, j.n, j.ngroups, 1, 0, j.out, nullptr, j.rhs, j.u, j.lam, j.skip, bl);
}

// ---------------------------------------------------------------------------- column pass
constexpr int CP_THREADS = 256;
constexpr int CP_COLS = CP_THREADS * 4;  // 1024 columns per workgroup
constexpr int CP_UNROLL = 8;

template <int MODE>
__device__ __forceinline__ void colpass_store(void* out, const float* v, double lam, int64_t col, int64_t m,
                                              const double (&t)[4], bool vec) {
  // MODE 0: x = (v - t) / lam as FP32; 1: as FP64; 2: t as FP64; 3: t as FP32.
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (col + e >= m) break;
    if constexpr (MODE == 2) {
      static_cast<double*>(out)[col + e] = t[e];
    } else if constexpr (MODE == 3) {
      static_cast<float*>(out)[col + e] = (float)t[e];
    } else {
      const double x = ((double)v[col + e] - t[e]) / lam;
      if constexpr (MODE == 0) static_cast<float*>(out)[col + e] = (float)x;
      else static_cast<double*>(out)[col + e] = x;
    }
  }
  (void)vec;
}

// Grid: x = column blocks of CP_COLS, y = row splits of `rps` rows. nsplit == 1 stores the final
// result; otherwise FP64 partial sums go to part[split * m + col].
template <int MODE>
__global__ void __launch_bounds__(CP_THREADS)
colpass_kernel(const float* __restrict__ S, int64_t n, int64_t m, int64_t lds, const double* __restrict__ y,
               const float* v, double lam, void* out, double* __restrict__ part, int64_t rps, int vec,
               const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t col = (int64_t)blockIdx.x * CP_COLS + 4 * threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * rps;
  const int64_t r1 = min(n, r0 + rps);
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  const bool full = vec && (col + 4 <= m);
  if (col < m) {
    int64_t i = r0;
    for (; i + CP_UNROLL <= r1; i += CP_UNROLL) {
      f32x4 sv[CP_UNROLL];
      double yy[CP_UNROLL];
#pragma unroll
      for (int u = 0; u < CP_UNROLL; ++u) {
        const float* p = S + (i + u) * lds + col;
        if (full) sv[u] = *reinterpret_cast<const f32x4*>(p);
        else {
#pragma unroll
          for (int e = 0; e < 4; ++e) sv[u][e] = (col + e < m) ? p[e] : 0.f;
        }
        yy[u] = y[i + u];
      }
#pragma unroll
      for (int u = 0; u < CP_UNROLL; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = fma((double)sv[u][e], yy[u], t[e]);
    }
    for (; i < r1; ++i) {
      const float* p = S + i * lds + col;
      f32x4 s;
      if (full) s = *reinterpret_cast<const f32x4*>(p);
      else {
#pragma unroll
        for (int e = 0; e < 4; ++e) s[e] = (col + e < m) ? p[e] : 0.f;
      }
      const double yi = y[i];
#pragma unroll
      for (int e = 0; e < 4; ++e) t[e] = fma((double)s[e], yi, t[e]);
    }
  }
  if (col >= m) return;
  if (part == nullptr) {
    colpass_store<MODE>(out, v, lam, col, m, t, vec);
  } else {
    double* pp = part + (int64_t)blockIdx.y * m;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (col + e < m) pp[col + e] = t[e];
  }
}

template <int MODE>
__global__ void colpass_finalize_kernel(const double* __restrict__ part, int64_t nsplit, int64_t m, const float* v,
                                        double lam, void* out, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  double t = 0.0;
  for (int64_t s = 0; s < nsplit; ++s) t += part[s * m + k];
  if constexpr (MODE == 2) {
    static_cast<double*>(out)[k] = t;
  } else if constexpr (MODE == 3) {
    static_cast<float*>(out)[k] = (float)t;
  } else {
    const double x = ((double)v[k] - t) / lam;
    if constexpr (MODE == 0) static_cast<float*>(out)[k] = (float)x;
    else static_cast<double*>(out)[k] = x;
  }
}

// Row pass that also writes the Gram's operands in their column-blocked layouts (QM = 3: scaled-FP8
// codes in 64-column blocks + scale bytes; QM = 2: split-BF16 planes in 16-column blocks). A wave
// owns RP_RPW = 8 consecutive rows and walks its column group 256 columns at a time (one 16-byte
// load per lane and row). The converted values of the 8 rows go to a per-wave LDS buffer laid out
// like the global blocks, so each global store covers one block's 8 consecutive rows: 512 bytes
// of codes, or 256 bytes of a plane, contiguous. b = S v (if WANT_B) and d_i = |s_i|^2 accumulate in
// FP64 as in rowpass_kernel. Needs the vectorised path (16-byte aligned rows); every column below
// ldq (zero input past m) is written.
constexpr int RPREP_COLS = 256;
constexpr int RPREP_STAGE = RP_RPW * RPREP_COLS * 4;   // bytes per wave: 8 rows x 256 columns x (hi + lo)

template <bool WANT_B, int QM>
__global__ void __launch_bounds__(64 * RP_WAVES)
rowpass_prep_kernel(const float* __restrict__ S, int64_t n, int64_t m, int64_t lds, const float* __restrict__ v,
                    int64_t cg, double* __restrict__ part, int vec, uint8_t* __restrict__ q, uint8_t* __restrict__ sc,
                    int64_t ldq) {
  __shared__ __align__(16) uint8_t stage_all[RP_WAVES][RPREP_STAGE];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint8_t* stg = stage_all[wave];
  const int64_t row0 = ((int64_t)blockIdx.x * RP_WAVES + wave) * RP_RPW;
  const int64_t g = blockIdx.y;
  const int64_t ngroups = gridDim.y;
  const int64_t c0 = g * cg;
  const int64_t c1 = min(m, c0 + cg);
  if (row0 >= n) return;
  const int nr = (int)min<int64_t>(RP_RPW, n - row0);

  double ab[RP_RPW], ad[RP_RPW];
#pragma unroll
  for (int r = 0; r < RP_RPW; ++r) { ab[r] = 0.0; ad[r] = 0.0; }

  for (int64_t cs = c0; cs < c1; cs += RPREP_COLS) {
    const int64_t col = cs + 4 * lane;
    f32x4 vv = {0.f, 0.f, 0.f, 0.f};
    if constexpr (WANT_B) load_s4(v + col, col, c1, (vec & 2) != 0, vv);
    f32x4 sv[RP_RPW];
#pragma unroll
    for (int r = 0; r < RP_RPW; ++r) {
      sv[r] = (f32x4){0.f, 0.f, 0.f, 0.f};
      if (r < nr) load_s4(S + (row0 + r) * lds + col, col, c1, (vec & 1) != 0, sv[r]);
    }
#pragma unroll
    for (int r = 0; r < RP_RPW; ++r)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double s = (double)sv[r][e];
        if constexpr (WANT_B) ab[r] = fma(s, (double)vv[e], ab[r]);
        ad[r] = fma(s, s, ad[r]);
      }
    if constexpr (QM == 3) {
      // codes of row r, columns col..col+3: block b = lane / 16 (64 columns), row r inside it
#pragma unroll
      for (int r = 0; r < RP_RPW; ++r) {
        float amax = fmaxf(fmaxf(fabsf(sv[r][0]), fabsf(sv[r][1])), fmaxf(fabsf(sv[r][2]), fabsf(sv[r][3])));
        amax = fmaxf(amax, __shfl_xor(amax, 1, 64));
        amax = fmaxf(amax, __shfl_xor(amax, 2, 64));
        amax = fmaxf(amax, __shfl_xor(amax, 4, 64));
        const int ex = mx_scale_exp(amax);
        const float inv = pow2_neg(ex);
        // |sv * inv| <= 448 by the choice of ex; the conversion rounds to nearest even
        int packed = __builtin_amdgcn_cvt_pk_fp8_f32(sv[r][0] * inv, sv[r][1] * inv, 0, false);
        packed = __builtin_amdgcn_cvt_pk_fp8_f32(sv[r][2] * inv, sv[r][3] * inv, packed, true);
        *reinterpret_cast<int*>(stg + ((lane >> 4) * RP_RPW + r) * 64 + (lane & 15) * 4) = packed;
        if ((lane & 7) == 0 && r < nr && col < ldq)
          sc[(((col >> 7) * n + row0 + r) << 2) + ((col >> 5) & 3)] = (uint8_t)(ex + 127);
      }
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      // 4 blocks x (8 rows x 64 bytes): lane l stores bytes 8 (l % 8) .. of row l / 8
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int64_t bc = cs + 64 * b;   // first column of the block
        const int r = lane >> 3;
        const uint64_t w = *reinterpret_cast<const uint64_t*>(stg + (b * RP_RPW + r) * 64 + (lane & 7) * 8);
        if (r < nr && bc < ldq)
          *reinterpret_cast<uint64_t*>(q + (((bc >> 6) * n + row0 + r) << 6) + (lane & 7) * 8) = w;
      }
    } else {
      // planes of row r, columns col..col+3: block b = lane / 4 (16 columns); hi at [0, 4 KB), lo after
#pragma unroll
      for (int r = 0; r < RP_RPW; ++r) {
        bf16x4 h, l;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const __bf16 hb = (__bf16)sv[r][e];        // round to nearest even
          h[e] = hb;
          l[e] = (__bf16)(sv[r][e] - (float)hb);
        }
        const int off = ((lane >> 2) * RP_RPW + r) * 32 + (lane & 3) * 8;
        *reinterpret_cast<bf16x4*>(stg + off) = h;
        *reinterpret_cast<bf16x4*>(stg + RPREP_STAGE / 2 + off) = l;
      }
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      // per plane 16 blocks x (8 rows x 32 bytes); one store covers two blocks: lanes 0-31 block
      // 2i, lanes 32-63 block 2i + 1; lane l stores bytes 8 (l % 4) .. of row (l % 32) / 4
      __bf16* hi = reinterpret_cast<__bf16*>(q);
      __bf16* lo = reinterpret_cast<__bf16*>(sc);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int b = 2 * i + (lane >> 5);
        const int r = (lane & 31) >> 2;
        const int64_t bc = cs + 16 * b;
        const int soff = (b * RP_RPW + r) * 32 + (lane & 3) * 8;
        const uint64_t wh = *reinterpret_cast<const uint64_t*>(stg + soff);
        const uint64_t wl = *reinterpret_cast<const uint64_t*>(stg + RPREP_STAGE / 2 + soff);
        if (r < nr && bc < ldq) {
          const int64_t e0 = (((bc >> 4) * n + row0 + r) << 4) + (lane & 3) * 4;   // element offset
          *reinterpret_cast<uint64_t*>(hi + e0) = wh;
          *reinterpret_cast<uint64_t*>(lo + e0) = wl;
        }
      }
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // the buffer is rewritten next iteration
  }
#pragma unroll
  for (int r = 0; r < RP_RPW; ++r) {
    if (r < nr) {
      if constexpr (WANT_B) {
        const double t = wave_sum(ab[r]);
        if (lane == 0) part[g * n + row0 + r] = t;
      }
      const double t = wave_sum(ad[r]);
      if (lane == 0) part[(ngroups + g) * n + row0 + r] = t;
    }
  }
}

// ---------------------------------------------------------------------------- fused refinement pass
// u = S (S^T y) with one read of S: the product of the exact S S^T with y that the refinement
// residual needs, without forming t = S^T y in memory. A workgroup of FR_WAVES waves holds a block
// of FR_COLS = 16 columns over all n rows in registers (one 16-byte load per lane; a wave covers 16
// rows per load, lane 4 r + q holding columns 4 q .. 4 q + 3 of row r), forms t_c = sum_i S_ic y_i
// for the block's columns (FP64 products and sums, reduced over the 16 lanes of a column and then
// over the waves in fixed order through LDS), and adds S_ic t_c to per-lane FP64 row accumulators.
// Two workgroups of one XCD (w mod 8, in dispatch order) walk a contiguous region of blocks side
// by side, so the two halves of each 128-byte line of a row are read through the same L2 at about
// the same time, and the regions of the pairs spread the reads in flight over the row. At
// the end each row's accumulators are reduced over its 4 lanes and stored as one partial per
// workgroup, part[g * n + i], which rowpass_reduce_kernel adds in fixed order. NCH loads per lane
// cover n <= 16 FR_WAVES NCH rows. Only whole 16-column blocks are streamed here.
constexpr int FR_COLS = 16;
constexpr int FR_WAVES = 8;    // 2 waves per SIMD: 256 registers per lane for 32 loads in flight
constexpr int FR_GROUP = 2;    // workgroups (of one XCD) walking adjacent blocks side by side

template <int NCH>
__global__ void __launch_bounds__(64 * FR_WAVES)
refine_pass_kernel(const float* __restrict__ S, int64_t n, int64_t m, int64_t lds, const double* __restrict__ y,
                   double* __restrict__ part, const int* __restrict__ skip) {
  constexpr int ROWS = 16 * FR_WAVES;   // rows per load step of the workgroup
  if (skip && *skip) return;   // a problem whose refinement has stopped (uniform): no read of S
  __shared__ double ys[ROWS * NCH];
  // Per-wave partials of t and t itself. Single buffers suffice: a block's partials are read
  // before its second barrier, which every wave passes before writing the next block's.
  __shared__ double tp[FR_WAVES][FR_COLS];
  __shared__ double tf[FR_COLS];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane & 3;
  const int rbase = wave * 16 + (lane >> 2);
  for (int idx = tid; idx < ROWS * NCH; idx += 64 * FR_WAVES) ys[idx] = idx < n ? y[idx] : 0.0;
  __syncthreads();
  double acc[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) acc[c] = 0.0;
  const int64_t nblk = m / FR_COLS;   // full blocks; the m % 16 last columns go to refine_tail_kernel
  // addresses: wave-uniform base + a 32-bit lane offset (the plan checks 16 lds * 4 < 2^31)
  const uint32_t loff = (uint32_t)(((lane >> 2) * lds + 4 * q) * 4);
  // Block of this workgroup in round s. Workgroup w = 8 l + x (x = its XCD, G = grid) has slot
  // x (G / 8) + l; slots 2 p and 2 p + 1 (one XCD when G / 8 is even) form pair p, which walks its
  // own contiguous region of R blocks two at a time: the two halves of each 128-byte line go
  // through one L2 at about the same time, and the pairs' regions spread the reads in flight over
  // the whole row. (With every workgroup on consecutive blocks, the reads in flight would all lie
  // in one 16 KB window of columns, rows a large power of two apart in the usual layout: the same
  // low address bits everywhere, which is hard on the HBM channel interleave.) Other grids take
  // blocks s G + slot.
  const int64_t G = gridDim.x;
  const int64_t slot = (G & 7) == 0 ? (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3) : (int64_t)blockIdx.x;
  const bool grouped = (G % (8 * FR_GROUP)) == 0;
  const int64_t R = grouped ? FR_GROUP * ((nblk + G - 1) / G) : 0;
  const int64_t grp = slot / FR_GROUP, mem = slot % FR_GROUP;
  auto block_of = [&](int64_t s) { return grouped ? grp * R + FR_GROUP * s + mem : s * G + slot; };
  auto valid = [&](int64_t s) { return (!grouped || FR_GROUP * s + mem < R) && block_of(s) < nblk; };
  // Load c of a block: rows c ROWS + 16 wave .. + 15, as a buffer load from a wave-uniform base
  // (the block's first column in row c ROWS + 16 wave) with the 32-bit lane offset. The buffer's
  // records end at row n, so rows past n read zeros; for a wave whose rows of this load all lie
  // past n, or with !any (no next block), it has no records at all and the load touches no
  // memory. The loop needs no branch around a load.
  // n, re-declared opaque every block (see the loop): each load's record count is formed where it
  // is used instead of NCH of them being kept in scalar registers
  // 32-bit scalars (n <= 4096, 16 lds * 4 < 2^31): few scalar registers per load
  int nrows = (int)n;
  const int rowbytes = (int)(lds * 4);
  auto load = [&](int64_t blk, int c, bool any) -> f32x4 {
    const int r0 = c * ROWS + wave * 16;
    const int rin = any ? min(16, nrows - r0) : 0;   // rows of this load below n (uniform)
    const bool in = rin > 0;
    const float* base = S + (in ? (int64_t)r0 : 0) * lds + blk * FR_COLS;
    // records end at row r0 + rin: lanes of rows past n read zeros (their offsets start there)
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), 0, in ? rin * rowbytes : 0, 0x00020000);
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)loff, 0, 0));
  };
  // Software pipeline without extra registers: the loads of block s + 1 are issued during the
  // second product of block s, each into the register its block-s data has just left, so HBM
  // streams while the matrix of one block is reduced and applied.
  f32x4 sv[NCH];
  int64_t s = 0;
  bool more = valid(0);   // uniform
  if (more) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) sv[c] = load(block_of(0), c, true);
  }
  // a do-while with the test at the bottom: no copies of the loop-carried accumulators
  if (more) do {
    const int64_t nxt = block_of(s + 1);
    more = valid(s + 1);
    asm volatile("" : "+s"(nrows));
    double tq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const double yr = ys[c * ROWS + rbase];
#pragma unroll
      for (int e = 0; e < 4; ++e) tq[e] = fma((double)sv[c][e], yr, tq[e]);
    }
#pragma unroll
    for (int o = 4; o < 64; o <<= 1)
#pragma unroll
      for (int e = 0; e < 4; ++e) tq[e] += __shfl_xor(tq[e], o, 64);
    if ((lane >> 2) == 0) {
#pragma unroll
      for (int e = 0; e < 4; ++e) tp[wave][4 * q + e] = tq[e];
    }
    __syncthreads();
    // wave 0 adds the waves' partials in fixed order: lane (col, g) sums waves 2 g and 2 g + 1,
    // then the four groups are combined pairwise (commutative adds: every lane gets the same bits)
    static_assert(FR_WAVES == 8, "the partial sum below takes 4 groups of 2 waves");
    if (wave == 0) {
      const int col = lane & 15, g = lane >> 4;
      double sg = tp[2 * g][col] + tp[2 * g + 1][col];
      sg += __shfl_xor(sg, 16, 64);
      sg += __shfl_xor(sg, 32, 64);
      if (lane < FR_COLS) tf[lane] = sg;
    }
    __syncthreads();
    double t[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) t[e] = tf[4 * q + e];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      asm volatile("" : "+v"(sv[c]));   // convert again rather than keep 2 NCH FP64 copies live
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[c] = fma((double)sv[c][e], t[e], acc[c]);
      sv[c] = load(more ? nxt : 0, c, more);
      __builtin_amdgcn_sched_barrier(0);   // keep the load behind the products that free its register
    }
    ++s;
  } while (more);
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    double v = acc[c];
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    const int64_t row = (int64_t)c * ROWS + rbase;
    if (q == 0 && row < n) part[(int64_t)blockIdx.x * n + row] = v;
  }
}

// ------------------------------------------------------------ fused refinement pass, whole lines
// The same product u = S (S^T y) with whole 128-byte lines: a block is 32 columns, a row's 128
// bytes are read by 8 lanes (16 bytes each), and a workgroup holds NCH loads per lane, 64 NCH
// rows. For n <= 64 NCH (NCH = 8, 16, 32 for n <= 512, 1024, 2048) one workgroup holds a whole
// block, and the workgroups walk contiguous regions of blocks. For 2048 < n <= 4096 (SPLIT)
// the two workgroups of a pair (one XCD: w and w + 8) hold its two row halves in
// registers (rows [0, 2048) and [2048, n); 32 loads of 16 bytes per lane, a row's 128 bytes over 8
// lanes). Each half's column partials t_c^(h) = sum over its rows of S_ic y_i are formed in a fixed
// order (lanes, then waves through LDS) and published in global memory; the workgroup waits,
// bounded, for its partner's, and both form t_c = t_c^(0) + t_c^(1) (same bits in both). Every
// block's partials have their own slot (nothing is overwritten during a launch), filled before
// each launch with XCH_EMPTY, a NaN whose payload no arithmetic produces (a NaN from S keeps the
// low 29 bits of its widened FP32 payload zero; a generated NaN has a zero payload), so the partner
// polls the values themselves: one memory round trip from the store to the reader instead of a
// store, a wait for its completion, a counter and a second load. A wait that runs out (the partner
// not resident, or far behind) is not an error: the workgroup computes the partner's partial itself
// from S, in the same order, so the result never depends on timing. Rows of the other half get zero
// partials, so the fixed-order reduction over workgroups is unchanged.
constexpr int FS_COLS = 32;
constexpr int FS_HALF = 2048;        // rows of the first half (64 rows per load step x 32 loads)
constexpr int FS_SPIN = 4096;        // polls (s_sleep 2 each, ~0.2 ms in all) before computing it here
constexpr uint64_t XCH_EMPTY = 0x7FF80000DEADBEEFull;   // an exchange slot not written yet

// The pass of workgroup w of gridx (the kernel body; the grouped form below runs it for a
// problem's share of a launch over many problems).
template <int NCH, bool SPLIT, bool CS>
__device__ __forceinline__ void refine_line_body(const float* __restrict__ S, int64_t n, int64_t m, int64_t lds,
                                                 const double* __restrict__ y, double* __restrict__ part,
                                                 double* __restrict__ xch, int64_t R, int spin,
                                                 const int* __restrict__ skip, double* __restrict__ tout,
                                                 double* __restrict__ csout, int64_t w, int64_t gridx) {
  constexpr int ROWS = 8 * FR_WAVES;   // rows per load step of the workgroup (8 per wave)
  static_assert(!SPLIT || NCH * ROWS == FS_HALF, "a split block's first half is one workgroup's rows");
  if (skip && *skip) return;
  __shared__ double ys[ROWS * NCH];
  __shared__ double tp[FR_WAVES][2 * FS_COLS];   // per wave: column partials of S^T y, then of S^T 1
  __shared__ double tf[2 * FS_COLS];
  __shared__ int got;
  constexpr bool wcs = CS;                        // also the column sums S^T 1 into csout
  constexpr int nl = CS ? 2 * FS_COLS : FS_COLS;  // lanes of wave 0 that carry a column value
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane & 7;                       // columns 4 q .. 4 q + 3 of the block
  const int rloc = wave * 8 + (lane >> 3);      // row within a load step
  // SPLIT: pair of two members on one XCD; else every workgroup walks its own region
  const int64_t pair = SPLIT ? (w & 7) * (gridx >> 4) + ((w >> 3) >> 1) : w;
  const int h = SPLIT ? (int)((w >> 3) & 1) : 0;
  const int64_t row0 = h ? FS_HALF : 0;
  const int64_t nh = SPLIT ? (h ? n - FS_HALF : min<int64_t>(n, FS_HALF)) : n;   // rows of this workgroup
  const int64_t prow0 = h ? 0 : FS_HALF;                                          // the partner's half
  const int64_t pnh = h ? FS_HALF : n - FS_HALF;
  for (int idx = tid; idx < ROWS * NCH; idx += 64 * FR_WAVES) ys[idx] = idx < nh ? y[row0 + idx] : 0.0;
  __syncthreads();
  double acc[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) acc[c] = 0.0;
  // the last block may be partial (m % 32 columns): its columns past m are zeroed after the load
  // (they are the next row's or the padding's values, or zeros past the buffer's records)
  const int64_t nblk = (m + FS_COLS - 1) / FS_COLS;
  const int64_t nfull = m / FS_COLS;
  const int cq = 4 * (lane & 7);   // this lane's first column within a block
  auto mask_tail = [&](f32x4& v, int64_t blk) {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (blk * FS_COLS + cq + e < m) ? v[e] : 0.f;
  };
  const int64_t b0 = pair * R, b1 = min(nblk, b0 + R);
  const uint32_t loff = (uint32_t)(((lane >> 3) * lds + 4 * q) * 4);
  const int rowbytes = (int)(lds * 4);
  // load c of block blk for the rows [base, base + cnt): rows past cnt read zeros (buffer records)
  auto load = [&](int64_t blk, int64_t base, int64_t cnt, int c, bool any) -> f32x4 {
    const int r0 = c * ROWS + wave * 8;
    const int rin = any ? (int)min<int64_t>(8, cnt - r0) : 0;
    const bool in = rin > 0;
    const float* bp = S + (in ? base + r0 : 0) * lds + blk * FS_COLS;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(bp), 0, in ? rin * rowbytes : 0, 0x00020000);
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)loff, 0, 0));
  };
  // column partials of one half from per-lane sums tq (4 columns per lane; with the column sums,
  // cq likewise): lanes of equal q, then the waves in a fixed order; the result lands in tp / is
  // read back by wave 0, lanes 0 .. 31 (S^T y) and 32 .. 63 (S^T 1)
  auto reduce_cols = [&](double* tq, f32x4 cq) {
#pragma unroll
    for (int o = 8; o < 64; o <<= 1)
#pragma unroll
      for (int e = 0; e < 4; ++e) tq[e] += __shfl_xor(tq[e], o, 64);
    if constexpr (CS) {
#pragma unroll
      for (int o = 8; o < 64; o <<= 1)
#pragma unroll
        for (int e = 0; e < 4; ++e) cq[e] += __shfl_xor(cq[e], o, 64);
    }
    if ((lane >> 3) == 0) {
#pragma unroll
      for (int e = 0; e < 4; ++e) tp[wave][4 * q + e] = tq[e];
      if constexpr (CS) {
#pragma unroll
        for (int e = 0; e < 4; ++e) tp[wave][FS_COLS + 4 * q + e] = (double)cq[e];
      }
    }
    __syncthreads();
    double v = 0.0;
    if (wave == 0 && lane < nl)
      v = ((tp[0][lane] + tp[1][lane]) + (tp[2][lane] + tp[3][lane])) +
          ((tp[4][lane] + tp[5][lane]) + (tp[6][lane] + tp[7][lane]));
    __syncthreads();
    return v;
  };
  f32x4 sv[NCH];
  int64_t blk = b0;
  bool more = blk < b1;
  if (more) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) sv[c] = load(blk, row0, nh, c, true);
  }
  if (more) do {
    const int64_t k = blk - b0;           // this block's index in the pair's walk
    if (blk == nfull) {                   // the partial last block (uniform)
#pragma unroll
      for (int c = 0; c < NCH; ++c) mask_tail(sv[c], blk);
    }
    const bool nmore = blk + 1 < b1;
    double tq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const double yr = ys[c * ROWS + rloc];
#pragma unroll
      for (int e = 0; e < 4; ++e) tq[e] = fma((double)sv[c][e], yr, tq[e]);
    }
    // the column sums over this lane's rows and then over the lanes in FP32 (they scale a small
    // correction term: 1e-5 relative is plenty), over the waves in FP64
    f32x4 cq = {0.f, 0.f, 0.f, 0.f};
    if constexpr (CS) {
#pragma unroll
      for (int c = 0; c < NCH; ++c) cq += sv[c];
    }
    const double own = reduce_cols(tq, cq);
    double tcol = 0.0;   // wave 0, lane < nl: this block's final value of column lane % 32
    if constexpr (!SPLIT) {
      if (wave == 0 && lane < nl) tf[lane] = own;
      tcol = own;
      (void)k;
    } else {
    double* slot = xch + ((pair * R + k) * 2) * (2 * FS_COLS);   // [h = 0 | h = 1] x (32 + 32 columns)
    // Publication without fences (an agent-scope fence writes back and invalidates the whole L2 of
    // the XCD, every block, for every workgroup): the partials are agent-scope relaxed atomics
    // (device-coherent accesses that skip the non-coherent caches), and the partner polls the
    // slot's values until none is XCH_EMPTY; each value is one 8-byte store, so a value read is
    // whole.
    double pv = 0.0;   // wave 0, lane < nl: the partner's value of this lane's column
    if (wave == 0) {
      if (lane < nl) __hip_atomic_store(slot + h * 2 * FS_COLS + lane, own, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int ok = 0;
      for (int it = 0; it < spin; ++it) {
        bool ready = true;
        if (lane < nl) {
          pv = __hip_atomic_load(slot + (1 - h) * 2 * FS_COLS + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ready = (uint64_t)__double_as_longlong(pv) != XCH_EMPTY;
        }
        if (__all(ready)) {   // wave-uniform
          ok = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      if (lane == 0) got = ok;
    }
    __syncthreads();
    double other = 0.0;
    if (got) {
      if (wave == 0 && lane < nl) other = pv;
    } else {
      // the partner's partials, computed here in its order (one load in flight per lane: rare path)
      double pq[4] = {0.0, 0.0, 0.0, 0.0};
      f32x4 pc = {0.f, 0.f, 0.f, 0.f};
      for (int c = 0; c < NCH; ++c) {
        f32x4 v = load(blk, prow0, pnh, c, true);
        if (blk == nfull) mask_tail(v, blk);
        const int64_t pr = (int64_t)c * ROWS + rloc;
        const double yr = pr < pnh ? y[prow0 + pr] : 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) pq[e] = fma((double)v[e], yr, pq[e]);
        if constexpr (CS) pc += v;
      }
      other = reduce_cols(pq, pc);
    }
    tcol = h == 0 ? own + other : other + own;
    if (wave == 0 && lane < nl) tf[lane] = tcol;
    }
    // the block's columns of S^T y (and S^T 1) to memory when asked: one writer per block
    if (wave == 0 && lane < nl && (!SPLIT || h == 0)) {
      const int64_t col = blk * FS_COLS + (lane & (FS_COLS - 1));
      if (col < m) {
        if (lane < FS_COLS) {
          if (tout) tout[col] = tcol;
        } else {
          csout[col] = tcol;
        }
      }
    }
    __syncthreads();
    double t[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) t[e] = tf[4 * q + e];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      asm volatile("" : "+v"(sv[c]));
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[c] = fma((double)sv[c][e], t[e], acc[c]);
      sv[c] = load(nmore ? blk + 1 : 0, row0, nh, c, nmore);
      __builtin_amdgcn_sched_barrier(0);
    }
    more = nmore;
    ++blk;
  } while (more);
  // row partials: this half's rows from the accumulators, zeros for the other half
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    double v = acc[c];
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    const int64_t r = (int64_t)c * ROWS + rloc;
    if (q == 0 && r < nh) part[w * n + row0 + r] = v;
  }
  if constexpr (SPLIT)
    for (int64_t i = tid; i < n - nh; i += 64 * FR_WAVES) part[w * n + (h ? i : FS_HALF + i)] = 0.0;
}

template <int NCH, bool SPLIT, bool CS>
__global__ void __launch_bounds__(64 * FR_WAVES)
refine_line_kernel(const float* __restrict__ S, int64_t n, int64_t m, int64_t lds, const double* __restrict__ y,
                   double* __restrict__ part, double* __restrict__ xch, int64_t R,
                   int spin, const int* __restrict__ skip, double* __restrict__ tout, double* __restrict__ csout) {
  refine_line_body<NCH, SPLIT, CS>(S, n, m, lds, y, part, xch, R, spin, skip, tout, csout, blockIdx.x, gridDim.x);
}

// Many problems' whole-line passes (n <= 2048, one workgroup per block) in one launch: job j owns
// workgroups [wg0_j, wg0_j + ngroups_j) and runs them exactly as its own launch would (the same
// partition of its blocks, its own partials), so the results are those of one launch per problem.
// A launch per problem pays a ramp-up and a tail per problem; small problems do not fill the
// device. Jobs are sorted by wg0; a workgroup finds its job by bisection (uniform, scalar loads).
template <int NCH, bool CS>
__global__ void __launch_bounds__(64 * FR_WAVES)
refine_line_grouped_kernel(const LineJob* __restrict__ jobs, int njobs) {
  const int64_t w = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].wg0 <= w) lo = mid;
    else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  const LineJob& j = jobs[lo];
  const int64_t wl = w - j.wg0;
  if (wl < 0 || wl >= j.ngroups) return;
  refine_line_body<NCH, false, CS>(j.S, j.n, j.m, j.lds, j.u, j.part, nullptr, j.R, 0, j.skip, j.tout, j.csout, wl,
                                   j.ngroups);
}

// The last m % TW (< TW, TW = the block width) columns of the fused pass, as one more group of
// partials: t_c = sum_i S_ic y_i for those columns (per-thread FP64 partials over rows tid,
// tid + 256, ..., then added in fixed order through LDS), then part[i] = sum_c S_ic t_c. One
// workgroup of 256 threads.
template <int TW>
__global__ void __launch_bounds__(256)
refine_tail_kernel(const float* __restrict__ S, int64_t n, int64_t m, int64_t lds, const double* __restrict__ y,
                   int64_t c0, double* __restrict__ part, const int* __restrict__ skip) {
  __shared__ double red[256][TW];
  __shared__ double tc[TW];
  if (skip && *skip) return;
  const int tid = threadIdx.x;
  const int nt = (int)(m - c0);   // 1 .. TW - 1
  double p[TW];
#pragma unroll
  for (int c = 0; c < TW; ++c) p[c] = 0.0;
  for (int64_t i = tid; i < n; i += 256) {
    const double yi = y[i];
#pragma unroll
    for (int c = 0; c < TW; ++c)
      if (c < nt) p[c] = fma((double)S[i * lds + c0 + c], yi, p[c]);
  }
#pragma unroll
  for (int c = 0; c < TW; ++c) red[tid][c] = p[c];
  __syncthreads();
  if (tid < TW) {
    double sum = 0.0;
    for (int k = 0; k < 256; ++k) sum += red[k][tid];
    tc[tid] = sum;
  }
  __syncthreads();
  for (int64_t i = tid; i < n; i += 256) {
    double u = 0.0;
    for (int c = 0; c < nt; ++c) u = fma((double)S[i * lds + c0 + c], tc[c], u);
    part[i] = u;
  }
}

__global__ void fill_u64_kernel(uint64_t* __restrict__ a, int64_t k, uint64_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) a[i] = v;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

RowPassPlan rowpass_plan(int64_t n, int64_t m, int64_t lds) {
  RowPassPlan p{};
  p.n = n;
  p.m = m;
  p.lds = lds;
  const int64_t rowblocks = (n + RP_WAVES * RP_RPW - 1) / (RP_WAVES * RP_RPW);
  // aim for ~8192 waves in flight over the whole grid
  const int64_t target_groups = std::max<int64_t>(1, 2048 / rowblocks);
  const int64_t max_groups = (m + RP_SUB - 1) / RP_SUB;
  p.nchunk = std::max<int64_t>(1, std::min(target_groups, max_groups));
  int64_t cg = (m + p.nchunk - 1) / p.nchunk;
  cg = (cg + RP_SUB - 1) / RP_SUB * RP_SUB;
  p.chunk = cg;
  p.nchunk = (m + cg - 1) / cg;
  p.part_bytes = (size_t)2 * (size_t)p.nchunk * (size_t)n * sizeof(double);
  return p;
}

hipError_t rowpass_launch(const RowPassPlan& p, const float* S, const float* v, const double* vd, bool want_b,
                          bool want_d, double* part, hipStream_t st, uint8_t* q, uint8_t* sc, int64_t ldq,
                          bool blocked) {
  // bit 0: rows of S are 16-byte aligned; bit 1: the vector is 16-byte aligned as well
  const bool vec = ((p.lds & 3) == 0) && aligned16(S);
  const bool vecv = vec && (v ? aligned16(v) : true) && (vd ? aligned16(vd) : true);
  const dim3 grid((unsigned)((p.n + RP_WAVES * RP_RPW - 1) / (RP_WAVES * RP_RPW)), (unsigned)p.nchunk);
  const dim3 block(64 * RP_WAVES);
  const int iv = (vec ? 1 : 0) | (vecv ? 2 : 0);
  if (q) {
    // fused quantisation: b = S v (optional), row norms, and the scaled-FP8 copy of S
    if (!vec || !want_d || vd || (ldq & 63) != 0 || ldq < p.m) return hipErrorInvalidValue;
    if (blocked && (ldq & 127) != 0) return hipErrorInvalidValue;
    if (blocked && want_b)
      hipLaunchKernelGGL((rowpass_prep_kernel<true, 3>), grid, block, 0, st, S, p.n, p.m, p.lds, v, p.chunk, part, iv, q, sc, ldq);
    else if (blocked)
      hipLaunchKernelGGL((rowpass_prep_kernel<false, 3>), grid, block, 0, st, S, p.n, p.m, p.lds, (const float*)nullptr, p.chunk, part, iv, q, sc, ldq);
    else if (want_b)
      hipLaunchKernelGGL((rowpass_kernel<float, true, true, 1>), grid, block, 0, st, S, p.n, p.m, p.lds, v, p.chunk, p.nchunk, part, iv, q, sc, ldq);
    else
      hipLaunchKernelGGL((rowpass_kernel<float, false, true, 1>), grid, block, 0, st, S, p.n, p.m, p.lds, (const float*)nullptr, p.chunk, p.nchunk, part, iv, q, sc, ldq);
    return hipGetLastError();
  }
  uint8_t* nq = nullptr;
  if (want_b && vd) {
    if (want_d)
      hipLaunchKernelGGL((rowpass_kernel<double, true, true, 0>), grid, block, 0, st, S, p.n, p.m, p.lds, vd, p.chunk, p.nchunk, part, iv, nq, nq, ldq);
    else
      hipLaunchKernelGGL((rowpass_kernel<double, true, false, 0>), grid, block, 0, st, S, p.n, p.m, p.lds, vd, p.chunk, p.nchunk, part, iv, nq, nq, ldq);
  } else if (want_b) {
    if (want_d)
      hipLaunchKernelGGL((rowpass_kernel<float, true, true, 0>), grid, block, 0, st, S, p.n, p.m, p.lds, v, p.chunk, p.nchunk, part, iv, nq, nq, ldq);
    else
      hipLaunchKernelGGL((rowpass_kernel<float, true, false, 0>), grid, block, 0, st, S, p.n, p.m, p.lds, v, p.chunk, p.nchunk, part, iv, nq, nq, ldq);
  } else if (want_d) {
    hipLaunchKernelGGL((rowpass_kernel<float, false, true, 0>), grid, block, 0, st, S, p.n, p.m, p.lds, (const float*)nullptr, p.chunk, p.nchunk, part, iv, nq, nq, ldq);
  }
  return hipGetLastError();
}

hipError_t rowpass_launch_split(const RowPassPlan& p, const float* S, const float* v, double* part, uint16_t* hi,
                                uint16_t* lo, int64_t ldh, hipStream_t st) {
  const bool vec = ((p.lds & 3) == 0) && aligned16(S);
  const bool vecv = vec && (v ? aligned16(v) : true);
  if (!vec || (ldh & 63) != 0 || ldh < p.m) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((p.n + RP_WAVES * RP_RPW - 1) / (RP_WAVES * RP_RPW)), (unsigned)p.nchunk);
  const dim3 block(64 * RP_WAVES);
  const int iv = 1 | (vecv ? 2 : 0);
  uint8_t* qh = reinterpret_cast<uint8_t*>(hi);
  uint8_t* ql = reinterpret_cast<uint8_t*>(lo);
  if (v)
    hipLaunchKernelGGL((rowpass_prep_kernel<true, 2>), grid, block, 0, st, S, p.n, p.m, p.lds, v, p.chunk, part, iv, qh, ql, ldh);
  else
    hipLaunchKernelGGL((rowpass_prep_kernel<false, 2>), grid, block, 0, st, S, p.n, p.m, p.lds, (const float*)nullptr, p.chunk, part, iv, qh, ql, ldh);
  return hipGetLastError();
}

hipError_t rowpass_reduce(const RowPassPlan& p, const double* part, bool want_b, bool want_d, double* b, double* d,
                          const double* r0, const double* y, double lam, hipStream_t st) {
  const dim3 grid((unsigned)((p.n + 15) / 16));
  hipLaunchKernelGGL(rowpass_reduce_kernel, grid, dim3(256), 0, st, part, p.n, p.nchunk, want_b ? 1 : 0,
                     want_d ? 1 : 0, b, d, r0, y, lam, (const int*)nullptr);
  return hipGetLastError();
}

ColPassPlan colpass_plan(int64_t n, int64_t m) {
  ColPassPlan p{};
  const int64_t cblocks = (m + CP_COLS - 1) / CP_COLS;
  int64_t nsplit = 1;
  // split the rows when there are too few column blocks to fill the device
  if (cblocks < 2048) nsplit = std::min<int64_t>((2048 + cblocks - 1) / cblocks, std::max<int64_t>(1, n / 64));
  p.nsplit = std::max<int64_t>(1, nsplit);
  p.rps = (n + p.nsplit - 1) / p.nsplit;
  p.nsplit = (n + p.rps - 1) / p.rps;
  p.part_bytes = p.nsplit > 1 ? (size_t)p.nsplit * (size_t)m * sizeof(double) : 0;
  return p;
}

hipError_t colpass_launch(const ColPassPlan& p, const float* S, int64_t n, int64_t m, int64_t lds, const double* y,
                          const float* v, double lambda, void* out, int mode, double* part, hipStream_t st,
                          const int* skip) {
  const bool vec = ((lds & 3) == 0) && aligned16(S);
  const dim3 grid((unsigned)((m + CP_COLS - 1) / CP_COLS), (unsigned)p.nsplit);
  double* pp = p.nsplit > 1 ? part : nullptr;
  const int iv = vec ? 1 : 0;
  switch (mode) {
    case 0: hipLaunchKernelGGL(colpass_kernel<0>, grid, dim3(CP_THREADS), 0, st, S, n, m, lds, y, v, lambda, out, pp, p.rps, iv, skip); break;
    case 1: hipLaunchKernelGGL(colpass_kernel<1>, grid, dim3(CP_THREADS), 0, st, S, n, m, lds, y, v, lambda, out, pp, p.rps, iv, skip); break;
    case 3: hipLaunchKernelGGL(colpass_kernel<3>, grid, dim3(CP_THREADS), 0, st, S, n, m, lds, y, v, lambda, out, pp, p.rps, iv, skip); break;
    default: hipLaunchKernelGGL(colpass_kernel<2>, grid, dim3(CP_THREADS), 0, st, S, n, m, lds, y, v, lambda, out, pp, p.rps, iv, skip); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p.nsplit == 1) return e;
  const dim3 g2((unsigned)((m + 255) / 256));
  switch (mode) {
    case 0: hipLaunchKernelGGL(colpass_finalize_kernel<0>, g2, dim3(256), 0, st, part, p.nsplit, m, v, lambda, out, skip); break;
    case 1: hipLaunchKernelGGL(colpass_finalize_kernel<1>, g2, dim3(256), 0, st, part, p.nsplit, m, v, lambda, out, skip); break;
    case 3: hipLaunchKernelGGL(colpass_finalize_kernel<3>, g2, dim3(256), 0, st, part, p.nsplit, m, v, lambda, out, skip); break;
    default: hipLaunchKernelGGL(colpass_finalize_kernel<2>, g2, dim3(256), 0, st, part, p.nsplit, m, v, lambda, out, skip); break;
  }
  return hipGetLastError();
}

RefinePassPlan refine_pass_plan(int64_t n, int64_t m, int64_t lds, const float* S, bool split_ok) {
  RefinePassPlan p{};
  p.n = n;
  const int64_t rows = 16 * FR_WAVES;
  p.nch = n <= 8 * rows ? 8 : (n <= 16 * rows ? 16 : (n <= 32 * rows ? 32 : 0));
  const int64_t nfull = m / FR_COLS;
  p.usable = p.nch > 0 && nfull > 0 && ((lds & 3) == 0) && aligned16(S) &&
             16 * lds * 4 < ((int64_t)1 << 31);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  // whole-line kernels (32-column blocks): one workgroup per block for n <= 2048; rows split over a
  // pair of workgroups for 2048 < n <= 4096 when every compute unit holds one workgroup and the
  // pairs fit the XCD layout
  const int64_t nblk32 = (m + FS_COLS - 1) / FS_COLS;   // the last one may be partial (masked in the kernel)
  p.split = split_ok && p.usable && p.nch == 32 && n > FS_HALF && (cus % 16) == 0 && nblk32 >= cus / 2;
  if (p.split) {
    const int64_t npairs = cus / 2;
    p.line = true;
    p.ngroups = cus;
    p.R = (nblk32 + npairs - 1) / npairs;
    p.tail = false;
    const size_t groups = (size_t)(p.ngroups + (p.tail ? 1 : 0)) * (size_t)n;
    p.xch_off = groups;
    p.xch_len = (size_t)npairs * (size_t)p.R * 2 * (2 * FS_COLS);
    p.part_bytes = (p.xch_off + p.xch_len) * sizeof(double);
    return p;
  }
  if (p.usable && n <= FS_HALF && nblk32 >= 1) {
    p.line = true;
    p.lnch = n <= 512 ? 8 : (n <= 1024 ? 16 : 32);
    const int64_t per_cu = p.lnch == 8 ? 3 : (p.lnch == 16 ? 2 : 1);
    p.ngroups = std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * per_cu, nblk32));
    p.R = (nblk32 + p.ngroups - 1) / p.ngroups;
    p.tail = false;
    p.part_bytes = (size_t)p.ngroups * (size_t)n * sizeof(double);
    return p;
  }
  // workgroups per compute unit as the registers allow (8 waves each: 6, 4 and 2 waves per SIMD fit
  // for 8, 16 and 32 loads per lane): with small n one block is little data, and several blocks
  // per compute unit keep enough bytes in flight
  const int64_t per_cu = p.nch == 8 ? 3 : (p.nch == 16 ? 2 : 1);
  p.ngroups = std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * per_cu, nfull));
  p.tail = (m % FR_COLS) != 0;
  p.part_bytes = p.usable ? (size_t)(p.ngroups + (p.tail ? 1 : 0)) * (size_t)n * sizeof(double) : 0;
  return p;
}

hipError_t refine_pass_launch(const RefinePassPlan& p, const float* S, int64_t n, int64_t m, int64_t lds,
                              const double* y, double* part, hipStream_t st, const int* skip, int spin, double* tout,
                              double* csout) {
  if (!p.usable || p.n != n) return hipErrorInvalidValue;
  if ((tout || csout) && !p.line) return hipErrorInvalidValue;   // only the whole-line kernels write them
  const dim3 grid((unsigned)p.ngroups), block(64 * FR_WAVES);
  if (p.split) {   // every exchange slot starts as XCH_EMPTY (a fill kernel: capturable)
    const int64_t nx = (int64_t)p.xch_len;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<uint64_t*>(part + p.xch_off), nx, XCH_EMPTY);
    if (spin < 0) {   // DFISHER_PAIR_SPIN overrides the default bound (0: never wait for the partner)
      const char* e = std::getenv("DFISHER_PAIR_SPIN");
      spin = e ? std::max(0, std::atoi(e)) : FS_SPIN;
    }
    if (csout)
      hipLaunchKernelGGL((refine_line_kernel<32, true, true>), grid, block, 0, st, S, n, m, lds, y, part,
                         part + p.xch_off, p.R, spin, skip, tout, csout);
    else
      hipLaunchKernelGGL((refine_line_kernel<32, true, false>), grid, block, 0, st, S, n, m, lds, y, part,
                         part + p.xch_off, p.R, spin, skip, tout, csout);
  } else if (p.line) {
    switch (p.lnch) {
      case 8:
        if (csout)
          hipLaunchKernelGGL((refine_line_kernel<8, false, true>), grid, block, 0, st, S, n, m, lds, y, part,
                             (double*)nullptr, p.R, 0, skip, tout, csout);
        else
          hipLaunchKernelGGL((refine_line_kernel<8, false, false>), grid, block, 0, st, S, n, m, lds, y, part,
                             (double*)nullptr, p.R, 0, skip, tout, csout);
        break;
      case 16:
        if (csout)
          hipLaunchKernelGGL((refine_line_kernel<16, false, true>), grid, block, 0, st, S, n, m, lds, y, part,
                             (double*)nullptr, p.R, 0, skip, tout, csout);
        else
          hipLaunchKernelGGL((refine_line_kernel<16, false, false>), grid, block, 0, st, S, n, m, lds, y, part,
                             (double*)nullptr, p.R, 0, skip, tout, csout);
        break;
      default:
        if (csout)
          hipLaunchKernelGGL((refine_line_kernel<32, false, true>), grid, block, 0, st, S, n, m, lds, y, part,
                             (double*)nullptr, p.R, 0, skip, tout, csout);
        else
          hipLaunchKernelGGL((refine_line_kernel<32, false, false>), grid, block, 0, st, S, n, m, lds, y, part,
                             (double*)nullptr, p.R, 0, skip, tout, csout);
        break;
    }
  }
  if (p.line) return hipGetLastError();   // the line kernels take the partial last block themselves
  switch (p.nch) {
    case 8: hipLaunchKernelGGL(refine_pass_kernel<8>, grid, block, 0, st, S, n, m, lds, y, part, skip); break;
    case 16: hipLaunchKernelGGL(refine_pass_kernel<16>, grid, block, 0, st, S, n, m, lds, y, part, skip); break;
    default: hipLaunchKernelGGL(refine_pass_kernel<32>, grid, block, 0, st, S, n, m, lds, y, part, skip); break;
  }
  if (p.tail)
    hipLaunchKernelGGL(refine_tail_kernel<FR_COLS>, dim3(1), dim3(256), 0, st, S, n, m, lds, y, m / FR_COLS * FR_COLS,
                       part + p.ngroups * n, skip);
  return hipGetLastError();
}

hipError_t refine_pass_reduce(const RefinePassPlan& p, const double* part, double* r, const double* b,
                              const double* y, double lam, hipStream_t st, const int* skip) {
  hipLaunchKernelGGL(rowpass_reduce_kernel, dim3((unsigned)((p.n + 15) / 16)), dim3(256), 0, st, part, p.n,
                     p.ngroups + (p.tail ? 1 : 0), 1, 0, r, (double*)nullptr, b, y, lam, skip);
  return hipGetLastError();
}

hipError_t refine_line_grouped_launch(const LineJob* jobs_dev, int njobs, int nch, bool cs, int64_t nwg,
                                      hipStream_t st) {
  if (njobs < 1 || nwg < 1 || nwg > 0x7FFFFFFF) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nwg), block(64 * FR_WAVES);
  switch (nch) {
    case 8:
      if (cs) hipLaunchKernelGGL((refine_line_grouped_kernel<8, true>), grid, block, 0, st, jobs_dev, njobs);
      else hipLaunchKernelGGL((refine_line_grouped_kernel<8, false>), grid, block, 0, st, jobs_dev, njobs);
      break;
    case 16:
      if (cs) hipLaunchKernelGGL((refine_line_grouped_kernel<16, true>), grid, block, 0, st, jobs_dev, njobs);
      else hipLaunchKernelGGL((refine_line_grouped_kernel<16, false>), grid, block, 0, st, jobs_dev, njobs);
      break;
    case 32:
      if (cs) hipLaunchKernelGGL((refine_line_grouped_kernel<32, true>), grid, block, 0, st, jobs_dev, njobs);
      else hipLaunchKernelGGL((refine_line_grouped_kernel<32, false>), grid, block, 0, st, jobs_dev, njobs);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t refine_reduce_grouped(const ReduceJob* jobs_dev, int njobs, int64_t nblk, hipStream_t st) {
  if (njobs < 1 || nblk < 1 || nblk > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(refine_reduce_grouped_kernel, dim3((unsigned)nblk), dim3(256), 0, st, jobs_dev, njobs);
  return hipGetLastError();
}

}  // namespace dfi
