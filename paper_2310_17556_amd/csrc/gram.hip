// Gram W = S S^T + lambda I_n on the CDNA4 matrix cores (Algorithm 1 step 1; the O(n^2 m)
// term that dominates the cost of the method, Section 2).
//
// Work decomposition
//   * Only lower-triangle 256 x 256 tiles of W are computed (W is symmetric).
//   * The contraction dimension (m, the parameters) is split into k-slices. A work item is
//     (tile, slice); it accumulates S_I S_J^T over its slice in FP32 matrix-core accumulators
//     and stores the FP32 partial tile. gram_reduce then adds the slices in FP64 in a fixed
//     order (deterministic, and the FP32 error stays that of one slice).
//   * XCD-aware mapping: workgroups are dealt round-robin to the 8 XCDs, so workgroup w runs on
//     XCD w % 8. Each XCD gets its own group of slices, and consecutive workgroups on an XCD
//     take different tiles of the same slice: tiles that run together read the same columns
//     of S, which then come from that XCD's L2 instead of HBM.
//   * Each workgroup has 8 waves in a 2 x 4 layout; a wave owns a 128 x 64 sub-tile as
//     4 x 2 blocks of 32 x 32 MFMA accumulators (128 FP32 accumulators per lane).
//   * Per k-step, 32 columns of the row panels S_I and S_J are loaded from global memory into
//     registers (prefetched one step ahead) and written to LDS; for split-BF16 they are split
//     into hi/lo bf16 on the way. Diagonal tiles load one panel and use it twice.
//
// k-ordering inside a step: an MFMA consumes k-values that depend on the lane half h = lane/32.
// Both operands use the same assignment (half h takes columns 16h .. 16h+15 of the step), so
// every product S_ik S_jk is formed exactly once and the sum over k is unchanged.
#include "dfisher_internal.h"

#include <algorithm>

namespace dfi {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int T = GRAM_TILE;      // 256
constexpr int KS = GRAM_KSTEP;    // 32
constexpr int WM = 2, WN = 4;             // wave grid inside the tile
constexpr int NTHR = 64 * WM * WN;        // 512
constexpr int BMW = T / WM, BNW = T / WN; // 128 x 64 per wave
constexpr int IM = BMW / 32, IN = BNW / 32;
constexpr int LOADS = T * KS / 4 / NTHR;  // float4 loads per thread per panel = 4
constexpr int ROWS_PER_LOAD = NTHR / (KS / 4);  // 64

// LDS row strides (elements). +16 bytes of padding per row keeps the 16-byte fragment reads
// of 16 consecutive rows on distinct bank groups.
constexpr int F32_STRIDE = KS + 4;    // 36 floats = 144 B
constexpr int BF_STRIDE = KS + 8;     // 40 bf16   = 80 B

__device__ __forceinline__ void tri_index(int64_t t, int64_t& ti, int64_t& tj) {
  // t -> (ti, tj), ti >= tj, t = ti (ti + 1) / 2 + tj
  int64_t r = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  ti = r;
  tj = t - r * (r + 1) / 2;
}

// Global -> register staging for one 256-row panel and one k-step.
// Thread t loads rows (t / 8) + 64 i, columns 4 (t % 8) .. +3 of the step.
template <bool VEC>
__device__ __forceinline__ void load_panel(const float* __restrict__ S, int64_t lds, int64_t n,
                                           int64_t row0, int64_t kcol, int64_t kend, f32x4 (&r)[LOADS]) {
  const int t = threadIdx.x;
  const int c = 4 * (t & 7);
  const int64_t col = kcol + c;
#pragma unroll
  for (int i = 0; i < LOADS; ++i) {
    const int64_t row = row0 + (t >> 3) + ROWS_PER_LOAD * i;
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (row < n) {
      const float* p = S + row * lds + col;
      if (VEC && col + 4 <= kend) {
        v = *reinterpret_cast<const f32x4*>(p);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (col + e < kend) v[e] = p[e];
      }
    }
    r[i] = v;
  }
}

template <int PREC>
struct Lds;

// FP32 operands: one panel of T rows x KS columns per operand.
template <>
struct Lds<0> {
  float a[T * F32_STRIDE];
  float b[T * F32_STRIDE];
};
// split-BF16 operands: hi and lo panels per operand.
template <>
struct Lds<1> {
  __bf16 ahi[T * BF_STRIDE];
  __bf16 alo[T * BF_STRIDE];
  __bf16 bhi[T * BF_STRIDE];
  __bf16 blo[T * BF_STRIDE];
};

__device__ __forceinline__ void store_f32(float* panel, const f32x4 (&r)[LOADS]) {
  const int t = threadIdx.x;
  const int c = 4 * (t & 7);
#pragma unroll
  for (int i = 0; i < LOADS; ++i) {
    const int row = (t >> 3) + ROWS_PER_LOAD * i;
    *reinterpret_cast<f32x4*>(panel + row * F32_STRIDE + c) = r[i];
  }
}

__device__ __forceinline__ void store_bf16(__bf16* hi, __bf16* lo, const f32x4 (&r)[LOADS]) {
  const int t = threadIdx.x;
  const int c = 4 * (t & 7);
#pragma unroll
  for (int i = 0; i < LOADS; ++i) {
    const int row = (t >> 3) + ROWS_PER_LOAD * i;
    bf16x4 h, l;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float a = r[i][e];
      const __bf16 hb = (__bf16)a;               // round to nearest even
      h[e] = hb;
      l[e] = (__bf16)(a - (float)hb);            // a - hi is exact in FP32
    }
    *reinterpret_cast<bf16x4*>(hi + row * BF_STRIDE + c) = h;
    *reinterpret_cast<bf16x4*>(lo + row * BF_STRIDE + c) = l;
  }
}

template <int PREC, bool VEC>
__global__ void __launch_bounds__(NTHR, 1)
gram_kernel(const float* __restrict__ S, int64_t n, int64_t lds, int64_t m, int64_t ntri,
            int64_t nslice, int64_t kslice, float* __restrict__ part) {
  __shared__ Lds<PREC> sm;

  // XCD-aware (slice, tile) assignment; nslice is a multiple of 8.
  const int64_t w = blockIdx.x;
  const int64_t xcd = w & 7;
  const int64_t local = w >> 3;
  const int64_t q = local / ntri;
  const int64_t tile = local - q * ntri;
  const int64_t slice = xcd * (nslice >> 3) + q;

  int64_t ti, tj;
  tri_index(tile, ti, tj);
  const bool diag = (ti == tj);
  const int64_t rowA = ti * T, rowB = tj * T;
  const int64_t k0 = slice * kslice;
  const int64_t kend = min(m, k0 + kslice);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = wave / WN, wc = wave % WN;
  const int half = lane >> 5;
  const int l32 = lane & 31;
  // In a diagonal tile, wave sub-tiles that lie wholly above the diagonal idle.
  const bool active = !(diag && wc * BNW >= (wr + 1) * BMW);

  f32x16 acc[IM][IN];
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < IN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  const int64_t nsteps = (kend > k0) ? (kend - k0 + KS - 1) / KS : 0;
  f32x4 ra[LOADS], rb[LOADS];
  if (nsteps > 0) {
    load_panel<VEC>(S, lds, n, rowA, k0, kend, ra);
    if (!diag) load_panel<VEC>(S, lds, n, rowB, k0, kend, rb);
  }

  for (int64_t s = 0; s < nsteps; ++s) {
    __syncthreads();  // previous step's fragment reads are done
    if constexpr (PREC == 0) {
      store_f32(sm.a, ra);
      if (!diag) store_f32(sm.b, rb);
    } else {
      store_bf16(sm.ahi, sm.alo, ra);
      if (!diag) store_bf16(sm.bhi, sm.blo, rb);
    }
    __syncthreads();
    if (s + 1 < nsteps) {  // prefetch the next step while this one computes
      const int64_t kc = k0 + (s + 1) * KS;
      load_panel<VEC>(S, lds, n, rowA, kc, kend, ra);
      if (!diag) load_panel<VEC>(S, lds, n, rowB, kc, kend, rb);
    }
    if (!active) continue;

    if constexpr (PREC == 0) {
      const float* pa = sm.a;
      const float* pb = diag ? sm.a : sm.b;
#pragma unroll
      for (int kk = 0; kk < 16; kk += 8) {
        f32x4 fa[IM][2], fb[IN][2];
#pragma unroll
        for (int i = 0; i < IM; ++i) {
          const float* ra_ = pa + (wr * BMW + i * 32 + l32) * F32_STRIDE + half * 16 + kk;
          fa[i][0] = *reinterpret_cast<const f32x4*>(ra_);
          fa[i][1] = *reinterpret_cast<const f32x4*>(ra_ + 4);
        }
#pragma unroll
        for (int j = 0; j < IN; ++j) {
          const float* rb_ = pb + (wc * BNW + j * 32 + l32) * F32_STRIDE + half * 16 + kk;
          fb[j][0] = *reinterpret_cast<const f32x4*>(rb_);
          fb[j][1] = *reinterpret_cast<const f32x4*>(rb_ + 4);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
          for (int i = 0; i < IM; ++i)
#pragma unroll
            for (int j = 0; j < IN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[i][e >> 2][e & 3], fb[j][e >> 2][e & 3],
                                                               acc[i][j], 0, 0, 0);
      }
    } else {
      const __bf16* ph = sm.ahi;
      const __bf16* pl = sm.alo;
      const __bf16* qh = diag ? sm.ahi : sm.bhi;
      const __bf16* ql = diag ? sm.alo : sm.blo;
#pragma unroll
      for (int kk = 0; kk < 16; kk += 8) {
        bf16x8 ah[IM], al[IM], bh[IN], bl[IN];
#pragma unroll
        for (int i = 0; i < IM; ++i) {
          const int oa = (wr * BMW + i * 32 + l32) * BF_STRIDE + half * 16 + kk;
          ah[i] = *reinterpret_cast<const bf16x8*>(ph + oa);
          al[i] = *reinterpret_cast<const bf16x8*>(pl + oa);
        }
#pragma unroll
        for (int j = 0; j < IN; ++j) {
          const int ob = (wc * BNW + j * 32 + l32) * BF_STRIDE + half * 16 + kk;
          bh[j] = *reinterpret_cast<const bf16x8*>(qh + ob);
          bl[j] = *reinterpret_cast<const bf16x8*>(ql + ob);
        }
#pragma unroll
        for (int i = 0; i < IM; ++i)
#pragma unroll
          for (int j = 0; j < IN; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
          }
      }
    }
  }

  // Store the FP32 partial tile (row-major T x T). 32x32 accumulator layout: lane l, register
  // r holds row 8 (r / 4) + 4 (l / 32) + (r % 4), column l % 32.
  float* out = part + (slice * ntri + tile) * (int64_t)(T * T);
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < IN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr * BMW + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
        const int col = wc * BNW + j * 32 + l32;
        out[row * T + col] = active ? acc[i][j][r] : 0.f;
      }
}

// W_ij = sum over slices of the partial tiles (FP64, slice order) for i > j; W_ii = d_i + lambda.
// mirror != 0 also writes W_ji. One workgroup covers 256 consecutive columns j of one row i.
__global__ void gram_reduce_kernel(const float* __restrict__ part, int64_t n, int64_t ntri, int64_t nslice,
                                   const double* __restrict__ d, double lambda, double* __restrict__ W,
                                   int mirror) {
  const int64_t nb = (n + 255) / 256;
  const int64_t i = (int64_t)blockIdx.x / nb;
  const int64_t j = ((int64_t)blockIdx.x - i * nb) * 256 + threadIdx.x;
  if (j > i || i >= n) return;
  double s;
  if (i == j) {
    s = d[i] + lambda;
  } else {
    const int64_t ti = i / T, tj = j / T;
    const int64_t tile = ti * (ti + 1) / 2 + tj;
    const int64_t off = (i - ti * T) * T + (j - tj * T);
    s = 0.0;
    for (int64_t sl = 0; sl < nslice; ++sl) s += (double)part[(sl * ntri + tile) * (int64_t)(T * T) + off];
  }
  W[i * n + j] = s;
  if (mirror && i != j) W[j * n + i] = s;
}

}  // namespace

GramPlan gram_plan(int64_t n, int64_t m, int64_t lds, int prec) {
  GramPlan p{};
  p.n = n;
  p.m = m;
  p.lds = lds;
  p.prec = prec;
  p.ntile = (n + T - 1) / T;
  p.ntri = p.ntile * (p.ntile + 1) / 2;
  // Slices per XCD (q): enough workgroups to fill 256 CUs several times with little tail,
  // while keeping at least ~2048 columns per slice.
  const int64_t maxq_cols = std::max<int64_t>(1, m / (8 * 2048));
  int64_t best_q = 1;
  double best_score = -1.0;
  for (int64_t q = 1; q <= 64; ++q) {
    if (q > maxq_cols && q > 1) break;
    const int64_t wgs = 8 * q * p.ntri;
    const int64_t rounds = (wgs + 255) / 256;
    const double eff = (double)wgs / (double)(rounds * 256);
    // prefer >= 4 rounds, then efficiency
    const double score = eff * (rounds >= 4 ? 1.0 : 0.5 + 0.125 * (double)rounds);
    if (score > best_score + 1e-9) {
      best_score = score;
      best_q = q;
    }
  }
  p.nslice = 8 * best_q;
  int64_t ks = (m + p.nslice - 1) / p.nslice;
  ks = (ks + KS - 1) / KS * KS;
  if (ks < KS) ks = KS;
  p.kslice = ks;
  p.part_bytes = (size_t)p.nslice * (size_t)p.ntri * (size_t)(T * T) * sizeof(float);
  return p;
}

hipError_t gram_launch(const GramPlan& p, const float* S, float* part, hipStream_t st) {
  const bool vec = ((p.lds & 3) == 0) && ((reinterpret_cast<uintptr_t>(S) & 15) == 0);
  const dim3 grid((unsigned)(p.nslice * p.ntri));
  const dim3 block(NTHR);
  if (p.prec == 0) {
    if (vec)
      hipLaunchKernelGGL((gram_kernel<0, true>), grid, block, 0, st, S, p.n, p.lds, p.m, p.ntri, p.nslice, p.kslice, part);
    else
      hipLaunchKernelGGL((gram_kernel<0, false>), grid, block, 0, st, S, p.n, p.lds, p.m, p.ntri, p.nslice, p.kslice, part);
  } else {
    if (vec)
      hipLaunchKernelGGL((gram_kernel<1, true>), grid, block, 0, st, S, p.n, p.lds, p.m, p.ntri, p.nslice, p.kslice, part);
    else
      hipLaunchKernelGGL((gram_kernel<1, false>), grid, block, 0, st, S, p.n, p.lds, p.m, p.ntri, p.nslice, p.kslice, part);
  }
  return hipGetLastError();
}

hipError_t gram_reduce(const GramPlan& p, const float* part, const double* d, double lambda, double* W,
                       int mirror, hipStream_t st) {
  const int64_t nb = (p.n + 255) / 256;
  const dim3 grid((unsigned)(nb * p.n));
  hipLaunchKernelGGL(gram_reduce_kernel, grid, dim3(256), 0, st, part, p.n, p.ntri, p.nslice, d, lambda, W, mirror);
  return hipGetLastError();
}

}  // namespace dfi
