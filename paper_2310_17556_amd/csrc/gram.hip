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
#include <type_traits>

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

// A value the whole wave agrees on, moved to scalar registers. 64-bit division and the square
// root in tri_index expand to vector code, and without this everything derived from their
// results (column ranges, step counts, load addresses) would be computed per lane in the loops.
__device__ __forceinline__ int64_t uni64(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
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

// Flip the sign bits of eight bf16 values when mask = 0x80008000 (identity for mask = 0).
__device__ __forceinline__ bf16x8 flip_sign(bf16x8 v, uint32_t mask) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  u32x4 u = __builtin_bit_cast(u32x4, v);
  u ^= mask;
  return __builtin_bit_cast(bf16x8, u);
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
  // odd slices negate A (see the alternating slice sign note of gram_kernel_v2)
  const float sgn = (slice & 1) ? -1.f : 1.f;
  const uint32_t bflip = (slice & 1) ? 0x80008000u : 0u;

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
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(sgn * fa[i][e >> 2][e & 3], fb[j][e >> 2][e & 3],
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
          ah[i] = flip_sign(*reinterpret_cast<const bf16x8*>(ph + oa), bflip);
          al[i] = flip_sign(*reinterpret_cast<const bf16x8*>(pl + oa), bflip);
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
        out[row * T + col] = active ? sgn * acc[i][j][r] : 0.f;
      }
}

// ---------------------------------------------------------------------------------------------
// Gram kernel v2 (16-byte aligned rows): asynchronous direct-to-LDS loads into a two-stage ring.
//
//   * Each k-step stages the FP32 columns [k, k+32) of the two 256-row panels with
//     global_load_lds_dwordx4: every wave instruction moves 8 rows x 128 B straight from global
//     memory to LDS (no register staging). Row r's eight 16-byte chunks are stored XOR-swizzled
//     (LDS chunk p holds column chunk p ^ (r & 7)) so that fragment reads of 8 consecutive rows
//     hit distinct banks.
//   * Two LDS stages: the loads for step s+1 are in flight while step s is multiplied; one
//     barrier per step.
//   * 4 waves in a 2 x 2 layout, each owning a 128 x 128 sub-tile (4 x 4 blocks of 32 x 32
//     accumulators). Split-BF16 fragments are formed when a wave reads its FP32 fragment from
//     LDS: hi = bf16_rne(a), lo = bf16_rne(a - hi).
//   * Rows beyond n load a valid row (their products only reach discarded outputs). The kernel
//     covers columns [0, m4) with m4 = m rounded down to a multiple of 4; chunks past a slice end
//     load zeros, and the FP64 reduction adds the products of the last m - m4 (< 4) columns.
//   * Alternating slice sign: on odd k-slices the A operand is negated and the stored partial
//     tile negated back. The bf16 matrix-core accumulation shows a small sign-independent bias
//     (low-order bits of the aligned addends are dropped toward minus infinity); it is the same
//     for +A and -A, so it cancels between even and odd slices instead of adding up coherently
//     over all entries (which would shift W along directions where many entries add, such as
//     the all-ones direction of a column-centered S).
namespace v2 {

constexpr int NW = 4;
constexpr int NT = 64 * NW;
constexpr int WT = 128;                 // wave sub-tile edge
constexpr int NB = WT / 32;             // 4 blocks per edge
constexpr int PANEL = T * KS;           // floats per panel per stage (32 KB)

typedef __attribute__((address_space(3))) void lds_void;

// Source of the zero chunks loaded past the end of a k-slice.
__device__ __align__(16) float g_zero_chunk[4] = {0.f, 0.f, 0.f, 0.f};

struct Stage {
  float a[PANEL];
  float b[PANEL];
};

// Issue the direct-to-LDS loads of one panel for one k-step. Wave w moves row groups
// g = w, w + 4, ..., each of 8 rows.
__device__ __forceinline__ void issue_panel(const float* __restrict__ S, int64_t lds, int64_t n, int64_t row0,
                                            int64_t kcol, int64_t kend, float* panel) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int rsub = lane >> 3;        // row inside the 8-row group
  const int p = lane & 7;            // LDS chunk position
#pragma unroll
  for (int i = 0; i < T / 8 / NW; ++i) {
    const int g = wave + NW * i;
    const int r = 8 * g + rsub;
    const int c = p ^ (r & 7);       // column chunk this lane fetches
    int64_t R = row0 + r;
    if (R >= n) R = n - 1;
    const int64_t col = kcol + 4 * c;
    // kend is a multiple of 4 here: a chunk is either wholly inside the slice or wholly past it
    const float* src = (col < kend) ? S + R * lds + col : g_zero_chunk;
    __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)(panel + 8 * g * KS), 16, 0, 0);
  }
}

// Read the 8 FP32 values of row r, step columns [c0, c0 + 8) (c0 a multiple of 8) from a
// swizzled panel.
__device__ __forceinline__ void read8(const float* panel, int r, int c0, float (&v)[8]) {
  const int q0 = (c0 >> 2) ^ (r & 7);
  const int q1 = ((c0 >> 2) + 1) ^ (r & 7);
  const f32x4 x0 = *reinterpret_cast<const f32x4*>(panel + r * KS + 4 * q0);
  const f32x4 x1 = *reinterpret_cast<const f32x4*>(panel + r * KS + 4 * q1);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    v[e] = x0[e];
    v[4 + e] = x1[e];
  }
}

__device__ __forceinline__ void split8(const float (&v)[8], float sgn, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float a = v[e] * sgn;
    const __bf16 h = (__bf16)a;
    hi[e] = h;
    lo[e] = (__bf16)(a - (float)h);
  }
}

// One k-step of the wave's 128 x 128 sub-tile from the current LDS stage.
template <int PREC>
__device__ __forceinline__ void step_compute(const float* pa, const float* pb, int ra0, int rb0, int half, float sgn,
                                             f32x16 (&acc)[NB][NB]) {
  if constexpr (PREC == 1) {
#pragma unroll
    for (int kk = 0; kk < 16; kk += 8) {
      // B fragments stay in registers for the substep; A fragments stream through, the next one
      // read while the current one's products issue.
      bf16x8 bh[NB], bl[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        float v[8];
        read8(pb, rb0 + j * 32, half * 16 + kk, v);
        split8(v, 1.f, bh[j], bl[j]);
      }
      float va[8];
      read8(pa, ra0, half * 16 + kk, va);
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        bf16x8 ah, al;
        split8(va, sgn, ah, al);
        if (i + 1 < NB) read8(pa, ra0 + (i + 1) * 32, half * 16 + kk, va);
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
        }
      }
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < 16; kk += 8) {
      float fb[NB][8];
#pragma unroll
      for (int j = 0; j < NB; ++j) read8(pb, rb0 + j * 32, half * 16 + kk, fb[j]);
      float fa[8];
      read8(pa, ra0, half * 16 + kk, fa);
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        float a[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) a[e] = fa[e] * sgn;
        if (i + 1 < NB) read8(pa, ra0 + (i + 1) * 32, half * 16 + kk, fa);
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
          for (int j = 0; j < NB; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[e], fb[j][e], acc[i][j], 0, 0, 0);
      }
    }
  }
}

template <int PREC>
__global__ void __launch_bounds__(NT, 1)
gram_kernel_v2(const float* __restrict__ S, int64_t n, int64_t lds, int64_t m, int64_t ntri, int64_t nslice,
               int64_t kslice, float* __restrict__ part) {
  __shared__ Stage st0;
  __shared__ Stage st1;

  const int64_t w = blockIdx.x;
  const int64_t xcd = w & 7;
  const int64_t local = w >> 3;
  const int64_t q = local / ntri;
  const int64_t tile = local - q * ntri;
  const int64_t slice = xcd * (nslice >> 3) + q;
  const float sgn = (slice & 1) ? -1.f : 1.f;

  int64_t ti, tj;
  tri_index(tile, ti, tj);
  const bool diag = (ti == tj);
  const int64_t rowA = ti * T, rowB = tj * T;
  const int64_t k0 = slice * kslice;
  const int64_t kend = min(m & ~(int64_t)3, k0 + kslice);   // columns [m4, m) go to the reduction
  const int64_t nsteps = (kend > k0) ? (kend - k0 + KS - 1) / KS : 0;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int half = lane >> 5;
  const int l32 = lane & 31;
  const bool active = !(diag && wr == 0 && wc == 1);

  f32x16 acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  if (nsteps > 0) {
    issue_panel(S, lds, n, rowA, k0, kend, st0.a);
    if (!diag) issue_panel(S, lds, n, rowB, k0, kend, st0.b);
  }
  for (int64_t s = 0; s < nsteps; ++s) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads for step s have landed
    __syncthreads();                // ... and every wave's; stage (s+1)&1 is free again
    const int64_t kc = k0 + s * KS;
    if (s + 1 < nsteps) {
      Stage& nx = ((s + 1) & 1) ? st1 : st0;
      issue_panel(S, lds, n, rowA, kc + KS, kend, nx.a);
      if (!diag) issue_panel(S, lds, n, rowB, kc + KS, kend, nx.b);
    }
    // (in diagonal tiles the wave above the diagonal computes too; its result is not stored:
    // a divergent skip here makes the compiler shuffle every accumulator each step)
    const Stage& cu = (s & 1) ? st1 : st0;
    const float* pa = cu.a;
    const float* pb = diag ? cu.a : cu.b;
    step_compute<PREC>(pa, pb, wr * WT + l32, wc * WT + l32, half, sgn, acc);
  }

  float* out = part + (slice * ntri + tile) * (int64_t)(T * T);
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr * WT + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
        const int col = wc * WT + j * 32 + l32;
        out[row * T + col] = active ? sgn * acc[i][j][r] : 0.f;
      }
}

}  // namespace v2

// ---------------------------------------------------------------------------------------------
// Gram kernel v3: scaled FP8. The operands are the block-scaled E4M3 codes written by the row
// pass in its column-blocked layout: 64-column blocks (one k-step), each holding all n rows
// contiguously (code (i, k) at q[((k / 64) n + i) 64 + k % 64]; the four E8M0 scale bytes of row
// i and 128-column block k / 128 form one aligned 4-byte word at sc[((k / 128) n + i) 4]). A
// k-step of a 256-row panel is then 16 KB of dense contiguous memory: whole cache lines, few
// pages, half the memory requests of 64-byte pieces of longer rows.
//   * k-step = 64 columns (two scale blocks). Codes move direct-to-LDS: each wave instruction
//     carries 16 rows x 64 B; row r's four 16-byte chunks are XOR-swizzled by (r >> 2) & 3 so the
//     fragment reads of 16 consecutive rows hit distinct banks. Scale bytes move direct-to-LDS as
//     one 4-byte word per row (four blocks, 128 columns; the step uses two of them), since the LDS
//     side of these loads advances 4 bytes per lane.
//   * Four LDS stages: the direct-to-LDS loads run up to four steps ahead of the matrix cores.
//     Every wave issues the same number of loads per step (diagonal tiles load their B panel as
//     well), so waiting for a stage is a vmcnt wait on the count of loads issued after it, plus
//     one barrier per step. Inside a step each A fragment is read one MFMA group ahead of its use;
//     the step's barrier sits before its last group, so the next step's B fragments and first A
//     fragment are read while that group's products run.
//   * v_mfma_scale_f32_32x32x64_f8f6f4: lane l supplies row (l % 32), 16 codes from scale block 0
//     and 16 from block 1 of the step (bytes [16h, 16h+16) and [32+16h, 32+16h+16) for h = l/32),
//     and the E8M0 scale of block h of its row. A and B use the same byte arrangement, so every
//     product pairs one column with itself.
//   * The slices cover all of [0, ldq): past m the row pass wrote zero codes, so every k-step is
//     whole and nothing is masked; the reduction adds no tail columns for this kernel.
//   * No alternating slice sign: the accumulation bias it cancels for bf16 (about 1e-6 relative)
//     is far below the E4M3 rounding of the operands.
namespace v3 {

constexpr int NW = 4;
constexpr int NT = 64 * NW;
constexpr int WT = 128;
constexpr int NB = WT / 32;
constexpr int KS8 = 64;                  // codes (bytes) per row per step
constexpr int PANEL = T * KS8;           // 16 KB
constexpr int NS = 4;                    // LDS stages
constexpr int LOADS_PER_STEP = 2 * (T / 16 / NW) + 2;   // codes A, B + scales A, B (per wave)

typedef __attribute__((address_space(3))) void lds_void;
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

struct Stage {
  uint8_t a[PANEL];
  uint8_t b[PANEL];
  uint8_t sa[4 * T];   // scale word of row r at [4r, 4r + 4): blocks 4w .. 4w + 3, w = kcol / 128
  uint8_t sb[4 * T];
};

// Loop-invariant per-lane byte offsets, inside one column block, of what this lane moves for a
// 256-row panel: code chunks (wave instruction i carries rows 16 g .. 16 g + 15, g = wave + 4 i;
// lane l fills LDS row 16 g + l / 4, chunk slot l % 4, with column chunk (l % 4) ^ ((row >> 2) & 3))
// and the scale word of row 64 wave + lane. Rows past n are clamped to n - 1 (their products are
// never stored).
struct PanelOffs {
  uint32_t code[T / 16 / NW];
  uint32_t scale;
};

__device__ __forceinline__ void panel_offsets(int64_t n, int64_t row0, PanelOffs& po) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < T / 16 / NW; ++i) {
    const int g = wave + NW * i;
    const int r = 16 * g + (lane >> 2);
    const int c = (lane & 3) ^ ((r >> 2) & 3);
    const int64_t R = min(row0 + r, n - 1);
    po.code[i] = (uint32_t)((R << 6) + 16 * c);
  }
  po.scale = (uint32_t)(min(row0 + 64 * wave + lane, n - 1) << 2);
}

// The step at column kcol (a multiple of 64): 64 code bytes of each of the panel's rows and the
// rows' scale words, direct to LDS. Every step lies inside [0, ldq), where the row pass wrote
// zero codes past m, so there is nothing to mask. issue_codes moves the rows of wave instruction
// i (16 rows x 64 B), issue_scales the scale words; a whole panel is i = 0 .. T / 16 / NW - 1
// plus the scales.
__device__ __forceinline__ void issue_codes(const uint8_t* q, int64_t n, int64_t kcol, const PanelOffs& po,
                                            uint8_t* panel, int i) {
  const int g = (int)(threadIdx.x >> 6) + NW * i;
  const uint8_t* qb = q + ((kcol >> 6) * n << 6);   // row 0 of this step's block, uniform
  __builtin_amdgcn_global_load_lds((const void*)(qb + po.code[i]), (lds_void*)(panel + 16 * g * KS8), 16, 0, 0);
}
__device__ __forceinline__ void issue_scales(const uint8_t* sc, int64_t n, int64_t kcol, const PanelOffs& po,
                                             uint8_t* sdst) {
  const int wave = threadIdx.x >> 6;
  const uint8_t* sb = sc + ((kcol >> 7) * n << 2);
  __builtin_amdgcn_global_load_lds((const void*)(sb + po.scale), (lds_void*)(sdst + 256 * wave), 4, 0, 0);
}

// Fragment of row r: chunks h and 2 + h (swizzled) -> 32 codes.
__device__ __forceinline__ i32x8 read_frag(const uint8_t* panel, int r, int h) {
  const int sw = (r >> 2) & 3;
  const i32x4 x0 = *reinterpret_cast<const i32x4*>(panel + r * KS8 + 16 * (h ^ sw));
  const i32x4 x1 = *reinterpret_cast<const i32x4*>(panel + r * KS8 + 16 * ((2 + h) ^ sw));
  i32x8 v;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    v[e] = x0[e];
    v[4 + e] = x1[e];
  }
  return v;
}

// vmcnt(N) with the other counters left alone (gfx9 encoding: vmcnt bits [3:0] and [15:14]).
#define DFI_WAIT_VM(N) __builtin_amdgcn_s_waitcnt(((N) & 15) | (((N) >> 4) << 14) | (7 << 4) | (15 << 8))
// lgkmcnt(0) with the other counters left alone (lgkmcnt bits [11:8]).
#define DFI_WAIT_LGKM0() __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4))

// The work item of workgroup w (the kernel body; the grouped form below runs it for one problem's
// share of a launch over many problems).
__device__ __forceinline__ void gram_fp8_body(const uint8_t* __restrict__ q, const uint8_t* __restrict__ sc, int64_t n,
                                              int64_t kcap, int64_t ntri, int64_t nslice, int64_t kslice,
                                              float* __restrict__ part, int64_t w) {
  __shared__ Stage stg0, stg1, stg2, stg3;

  const int64_t xcd = w & 7;
  const int64_t local = w >> 3;
  const int64_t qq = uni64(local / ntri);
  const int64_t tile = local - qq * ntri;
  const int64_t slice = xcd * (nslice >> 3) + qq;

  int64_t ti, tj;
  tri_index(tile, ti, tj);
  ti = uni64(ti);
  tj = uni64(tj);
  const bool diag = (ti == tj);
  const int64_t rowA = ti * T, rowB = tj * T;
  const int64_t k0 = uni64(slice * kslice);
  const int64_t kend = min(kcap, k0 + kslice);
  const int64_t nsteps = uni64((kend > k0) ? (kend - k0) / KS8 : 0);   // both multiples of 64

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int half = lane >> 5;
  const int l32 = lane & 31;
  const bool active = !(diag && wr == 0 && wc == 1);

  f32x16 acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  // Stage k of the ring, k a compile-time constant: the step loop is unrolled by NS so that every
  // LDS access names its stage object. The compiler's tracking of direct-to-LDS loads can then
  // tell the stages apart; with a stage picked at run time it cannot, and it inserts a wait for
  // every load in flight (the three steps ahead included) before the first operand read of a step.
  auto stage = [&](auto k) -> Stage& {
    constexpr int K = decltype(k)::value;
    if constexpr (K == 0) return stg0;
    else if constexpr (K == 1) return stg1;
    else if constexpr (K == 2) return stg2;
    else return stg3;
  };
  PanelOffs offA, offB;
  panel_offsets(n, rowA, offA);
  panel_offsets(n, rowB, offB);
  // Refill stage k with `step` (k = step mod NS). Steps past the slice's end load the slice's
  // last step again (never read as operands): every step then issues the same loads and waits
  // for the same count, with no branch in the loop.
  // Piece p (0 .. NB - 1) of the refill: code instruction p of both panels, and with the last
  // piece both panels' scale words. Diagonal tiles load their B panel too: uniform load counts.
  static_assert(T / 16 / NW == NB, "one refill piece per product of a group");
  auto issue_piece = [&](auto k, int64_t step, int p) {
    Stage& sp = stage(k);
    const int64_t kc = k0 + min(step, nsteps - 1) * KS8;
    issue_codes(q, n, kc, offA, sp.a, p);
    issue_codes(q, n, kc, offB, sp.b, p);
    if (p == NB - 1) {
      issue_scales(sc, n, kc, offA, sp.sa);
      issue_scales(sc, n, kc, offB, sp.sb);
    }
  };
  auto issue_step = [&](auto k, int64_t step) {
#pragma unroll
    for (int p = 0; p < NB; ++p) issue_piece(k, step, p);
  };
  // this wave's operands of one step, read from LDS into registers
  // head of a step: the four B fragments with their scales and the first A fragment
  struct Head {
    i32x8 fb[NB];
    int sbv[NB];
    i32x8 fa0;
    int sa0;
  };
  // Per-lane LDS byte offsets inside a stage. Fragment i of the wave's A rows is row
  // wr WT + 32 i + l32; its swizzle (row >> 2) & 3 depends on l32 only, so fragment i sits at the
  // fragment-0 offsets + 32 i KS8 and its scale byte at + 128 i.
  struct LaneOffs {
    int a0, a1, b0, b1, sa, sb;
  };
  LaneOffs lo0;
  {
    const int sw = (l32 >> 2) & 3;
    const int ra = wr * WT + l32, rb = wc * WT + l32;
    lo0.a0 = ra * KS8 + 16 * (half ^ sw);
    lo0.a1 = ra * KS8 + 16 * ((2 + half) ^ sw);
    lo0.b0 = rb * KS8 + 16 * (half ^ sw);
    lo0.b1 = rb * KS8 + 16 * ((2 + half) ^ sw);
    lo0.sa = 4 * ra + half;
    lo0.sb = 4 * rb + half;
  }
  auto frag = [](const uint8_t* p0, const uint8_t* p1) {
    const i32x4 x0 = *reinterpret_cast<const i32x4*>(p0);
    const i32x4 x1 = *reinterpret_cast<const i32x4*>(p1);
    i32x8 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[e] = x0[e];
      v[4 + e] = x1[e];
    }
    return v;
  };
  auto load_head = [&](auto k, int64_t step, Head& h, const LaneOffs& lo) {
    const Stage& cu = stage(k);
    const int sbyte = (int)(((k0 + step * KS8) >> 5) & 3);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      h.fb[j] = frag(cu.b + lo.b0 + 32 * KS8 * j, cu.b + lo.b1 + 32 * KS8 * j);
      h.sbv[j] = cu.sb[lo.sb + 128 * j + sbyte];
    }
    h.fa0 = frag(cu.a + lo.a0, cu.a + lo.a1);
    h.sa0 = cu.sa[lo.sa + sbyte];
  };
  // Step s (in stage k) from head h (already in registers): A fragments 1..3 are read one group
  // ahead; after the third group every LDS read of step s is done, so the wave waits for step
  // s + 1's loads (two steps' loads issued later may stay in flight), meets the others at the
  // barrier, reads step s + 1's head into hn and refills stage k with step s + NS while the last
  // group of matrix-core products runs. The step has no branch: the scheduling fences below only
  // hold inside one basic block, and with branches in the step the compiler sinks its products
  // below the waits and the barrier, leaving the matrix cores idle through them. At the last step
  // the head read is of a stage that holds no later step; it is never used. The lane offsets are
  // made opaque once per step, so that the compiler forms each address next to its read instead
  // of keeping every stage's addresses live (which spills).
  auto body = [&](auto k, int64_t s, Head& h, Head& hn) {
    constexpr int K = decltype(k)::value;
    const Stage& cu = stage(k);
    LaneOffs lo = lo0;
    asm volatile("" : "+v"(lo.a0), "+v"(lo.a1), "+v"(lo.b0), "+v"(lo.b1), "+v"(lo.sa), "+v"(lo.sb));
    const int sbyte = (int)(((k0 + s * KS8) >> 5) & 3);
    i32x8 fa[2];
    int sav[2];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      // Group i's operands were requested a whole group earlier and have arrived; waiting for
      // them here, before fragment i + 1 is requested, keeps the wait off the newer reads.
      DFI_WAIT_LGKM0();
      if (i + 1 < NB) {
        fa[(i + 1) & 1] = frag(cu.a + lo.a0 + 32 * KS8 * (i + 1), cu.a + lo.a1 + 32 * KS8 * (i + 1));
        sav[(i + 1) & 1] = cu.sa[lo.sa + 128 * (i + 1) + sbyte];
      }
      if (i == NB - 1) {
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        DFI_WAIT_VM(2 * LOADS_PER_STEP);
        asm volatile("s_barrier" ::: "memory");
        load_head(std::integral_constant<int, (K + 1) % NS>{}, s + 1, hn, lo);
      }
      __builtin_amdgcn_sched_barrier(0);
      const i32x8 a = (i == 0) ? h.fa0 : fa[i & 1];
      const int sa = (i == 0) ? h.sa0 : sav[i & 1];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, h.fb[j], acc[i][j], 0, 0, 0, sa, 0, h.sbv[j]);
        if (i == NB - 1) {
          // the refill of stage k goes out in pieces between the last group's products, whose
          // execution hides the issue of its loads and their address arithmetic
          __builtin_amdgcn_sched_barrier(0);
          issue_piece(k, s + NS, j);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  using K0 = std::integral_constant<int, 0>;
  using K1 = std::integral_constant<int, 1>;
  using K2 = std::integral_constant<int, 2>;
  using K3 = std::integral_constant<int, 3>;
  static_assert(NS == 4, "the step loop is unrolled by the stage count");
  Head h0, h1;
  if (nsteps > 0) {
    issue_step(K0{}, 0);
    issue_step(K1{}, 1);
    issue_step(K2{}, 2);
    issue_step(K3{}, 3);
    DFI_WAIT_VM(3 * LOADS_PER_STEP);
    asm volatile("s_barrier" ::: "memory");
    load_head(K0{}, 0, h0, lo0);
    int64_t s = 0;
    for (; s + 3 < nsteps; s += 4) {
      body(K0{}, s, h0, h1);
      body(K1{}, s + 1, h1, h0);
      body(K2{}, s + 2, h0, h1);
      body(K3{}, s + 3, h1, h0);
    }
    if (s < nsteps) body(K0{}, s, h0, h1);
    if (s + 1 < nsteps) body(K1{}, s + 1, h1, h0);
    if (s + 2 < nsteps) body(K2{}, s + 2, h0, h1);
    DFI_WAIT_VM(0);   // the trailing refills land in LDS before the workgroup ends
  }

  float* out = part + (slice * ntri + tile) * (int64_t)(T * T);
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr * WT + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
        const int col = wc * WT + j * 32 + l32;
        out[row * T + col] = active ? acc[i][j][r] : 0.f;
      }
}

__global__ void __launch_bounds__(NT, 1)
gram_kernel_fp8(const uint8_t* __restrict__ q, const uint8_t* __restrict__ sc, int64_t n, int64_t kcap,
                int64_t ntri, int64_t nslice, int64_t kslice, float* __restrict__ part) {
  gram_fp8_body(q, sc, n, kcap, ntri, nslice, kslice, part, blockIdx.x);
}

// Many problems' scaled-FP8 Grams in one launch: job j owns workgroups [wg0_j, wg0_j + ntri_j
// nslice_j) and runs its (tile, slice) work items exactly as its own launch would (wg0_j a
// multiple of 8, so each work item keeps its XCD), writing its own partial tiles. The jobs are
// ordered by the work of one item (slice length), largest first, so the dispatcher hands the
// largest items out first and the small ones fill the end of the launch. A workgroup finds its job
// by bisection (uniform, scalar loads).
__global__ void __launch_bounds__(NT, 1)
gram_kernel_fp8_grouped(const GramJob* __restrict__ jobs, int njobs) {
  const int64_t w = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].wg0 <= w) lo = mid;
    else hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  const GramJob& j = jobs[lo];
  const int64_t wl = w - j.wg0;
  if (wl < 0 || wl >= j.ntri * j.nslice) return;
  gram_fp8_body(j.q, j.sc, j.n, j.kcap, j.ntri, j.nslice, j.kslice, j.part, wl);
}

}  // namespace v3

// ---------------------------------------------------------------------------------------------
// Gram kernel v4: split-BF16 from pre-split planes. The row pass writes hi = bf16_rne(S) and
// lo = bf16_rne(S - hi) as two bf16 planes in its column-blocked layout (16-column blocks, one
// k-step, of all n rows: element (i, k) at [((k / 16) n + i) 16 + k % 16], so a step of a panel
// is 8 KB of dense contiguous memory); the tile kernel is then a plain bf16
// matrix-core product with three terms per pair of elements (lo.hi, hi.lo, hi.hi) and no
// conversion work in its loop.
//   * k-step = 16 columns: 32 bytes of each of the 256 rows of a panel, per plane. One wave
//     instruction moves 32 rows straight to LDS (two 16-byte chunks per row); a row's chunks are
//     swapped when (row >> 2) is odd, so the fragment reads of 8 consecutive rows cover all banks.
//   * Four LDS stages of 32 KB (A hi, A lo, B hi, B lo) and two register sets of operands, with
//     the same schedule and vmcnt-counted waits as v3 (every wave issues the same number of loads
//     per step; diagonal tiles load their B panel too).
//   * v_mfma_f32_32x32x16_bf16: lane l supplies row l % 32 and columns 8h .. 8h + 7 of the step
//     (h = l / 32), for A and B alike.
//   * The slices cover all of [0, ldh): past m the planes hold zeros, so every k-step is whole;
//     the reduction adds no tail columns for this kernel.
//   * Alternating slice sign as in v1: odd slices flip the sign bits of A's fragments.
namespace v4 {

constexpr int NW = 4;
constexpr int NT = 64 * NW;
constexpr int WT = 128;
constexpr int NB = WT / 32;
constexpr int KSB = 16;                          // bf16 columns per step
constexpr int ROWB = 2 * KSB;                    // 32 bytes per row and plane
constexpr int PANEL = T * ROWB;                  // 8 KB
constexpr int NS = 4;                            // LDS stages
constexpr int INSTR = T / 32 / NW;               // load instructions per wave, panel and plane (2)
constexpr int LOADS_PER_STEP = 4 * INSTR;        // A hi, A lo, B hi, B lo

typedef __attribute__((address_space(3))) void lds_void;

struct Stage {
  uint8_t ah[PANEL];
  uint8_t al[PANEL];
  uint8_t bh[PANEL];
  uint8_t bl[PANEL];
};

// Loop-invariant per-lane element offsets (inside one 16-column block of a plane) of the chunks
// this lane moves for a 256-row panel: wave instruction i carries rows 32 g .. 32 g + 31
// (g = wave + 4 i); lane l fills LDS row 32 g + l / 2, chunk slot l % 2, with column chunk
// (l % 2) ^ ((row >> 2) & 1). Rows past n are clamped to n - 1 (their products are never stored).
struct PanelOffs {
  uint32_t e[INSTR];
};

__device__ __forceinline__ void panel_offsets(int64_t n, int64_t row0, PanelOffs& po) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < INSTR; ++i) {
    const int g = wave + NW * i;
    const int r = 32 * g + (lane >> 1);
    const int c = (lane & 1) ^ ((r >> 2) & 1);
    const int64_t R = min(row0 + r, n - 1);
    po.e[i] = (uint32_t)((R << 4) + 8 * c);
  }
}

// One plane of one panel for the step at column kcol (a multiple of 16): every step lies inside
// [0, ldh), where the row pass wrote zeros past m, so nothing is masked.
__device__ __forceinline__ void issue_plane(const uint16_t* plane, int64_t n, int64_t kcol, const PanelOffs& po,
                                            uint8_t* panel) {
  const uint16_t* pb = plane + ((kcol >> 4) * n << 4);   // row 0 of this step's block, uniform
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < INSTR; ++i) {
    const int g = wave + NW * i;
    __builtin_amdgcn_global_load_lds((const void*)(pb + po.e[i]), (lds_void*)(panel + 32 * g * ROWB), 16, 0, 0);
  }
}

// One wave's operands of one k-step: hi and lo fragments of its 4 A and 4 B row blocks.
struct Frags {
  bf16x8 ah[NB], al[NB], bh[NB], bl[NB];
};

__global__ void __launch_bounds__(NT, 1)
gram_kernel_split(const uint16_t* __restrict__ hi, const uint16_t* __restrict__ lo, int64_t n,
                  int64_t kcap, int64_t ntri, int64_t nslice, int64_t kslice, float* __restrict__ part) {
  __shared__ Stage stg0, stg1, stg2, stg3;

  const int64_t w = blockIdx.x;
  const int64_t xcd = w & 7;
  const int64_t local = w >> 3;
  const int64_t qq = uni64(local / ntri);
  const int64_t tile = local - qq * ntri;
  const int64_t slice = xcd * (nslice >> 3) + qq;
  const uint32_t bflip = (slice & 1) ? 0x80008000u : 0u;

  int64_t ti, tj;
  tri_index(tile, ti, tj);
  ti = uni64(ti);
  tj = uni64(tj);
  const bool diag = (ti == tj);
  const int64_t rowA = ti * T, rowB = tj * T;
  const int64_t k0 = uni64(slice * kslice);
  const int64_t kend = min(kcap, k0 + kslice);
  const int64_t nsteps = uni64((kend > k0) ? (kend - k0) / KSB : 0);   // both multiples of 16

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int half = lane >> 5;
  const int l32 = lane & 31;
  const bool active = !(diag && wr == 0 && wc == 1);

  f32x16 acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  // Stage k of the ring, k a compile-time constant (see the scaled-FP8 kernel: the loop is unrolled
  // by NS so that every LDS access names its stage object).
  auto stage = [&](auto k) -> Stage& {
    constexpr int K = decltype(k)::value;
    if constexpr (K == 0) return stg0;
    else if constexpr (K == 1) return stg1;
    else if constexpr (K == 2) return stg2;
    else return stg3;
  };
  PanelOffs offA, offB;
  panel_offsets(n, rowA, offA);
  panel_offsets(n, rowB, offB);
  // Piece p of the refill of stage k with `step` (k = step mod NS): plane p of the four (A hi, A lo,
  // B hi, B lo; diagonal tiles load B too: uniform load counts). Steps past the slice's end load
  // the slice's last step again (never read as operands), so every step issues the same loads.
  auto issue_piece = [&](auto k, int64_t step, int p) {
    Stage& sp = stage(k);
    const int64_t kc = k0 + min(step, nsteps - 1) * KSB;
    if (p == 0) issue_plane(hi, n, kc, offA, sp.ah);
    else if (p == 1) issue_plane(lo, n, kc, offA, sp.al);
    else if (p == 2) issue_plane(hi, n, kc, offB, sp.bh);
    else issue_plane(lo, n, kc, offB, sp.bl);
  };
  auto issue_step = [&](auto k, int64_t step) {
#pragma unroll
    for (int p = 0; p < 4; ++p) issue_piece(k, step, p);
  };
  // Per-lane LDS byte offsets of fragment 0 of the wave's A and B rows inside a plane; fragment i
  // is 32 rows further on (+ 32 i ROWB), with the same swizzle ((row >> 2) & 1 depends on l32 only).
  int oA0, oB0;
  {
    const int sw = (l32 >> 2) & 1;
    oA0 = (wr * WT + l32) * ROWB + 16 * (half ^ sw);
    oB0 = (wc * WT + l32) * ROWB + 16 * (half ^ sw);
  }
  auto rd = [](const uint8_t* p) { return *reinterpret_cast<const bf16x8*>(p); };
  auto load_frags = [&](auto k, Frags& f, int oA, int oB) {
    const Stage& cu = stage(k);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      f.bh[j] = rd(cu.bh + oB + 32 * ROWB * j);
      f.bl[j] = rd(cu.bl + oB + 32 * ROWB * j);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      f.ah[i] = rd(cu.ah + oA + 32 * ROWB * i);
      f.al[i] = rd(cu.al + oA + 32 * ROWB * i);
    }
  };
  // term t of the product of A row block i with B row block j: lo.hi, hi.lo, hi.hi in that order
  auto mfma_term = [&](const Frags& f, int i, int j, int t) {
    const bf16x8 a = flip_sign(t == 0 ? f.al[i] : f.ah[i], bflip);
    const bf16x8 b = t == 1 ? f.bl[j] : f.bh[j];
    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[i][j], 0, 0, 0);
  };
  // Step s (stage k) from operands cur (already in registers): the products of A row blocks
  // 0 .. NB - 2 run first; then the wave waits for step s + 1's loads (two later steps' loads may
  // stay in flight), meets the others at the barrier (every wave has read stage k, which it did
  // into cur one step earlier), reads step s + 1's operands into nxt and refills stage k with step
  // s + NS between the last row block's products. The step has no branch, so the
  // scheduling fences hold and the products overlap the waits.
  auto body = [&](auto k, Frags& cur, Frags& nxt, int64_t s) {
    constexpr int K = decltype(k)::value;
    int oA = oA0, oB = oB0;
    asm volatile("" : "+v"(oA), "+v"(oB));
#pragma unroll
    for (int i = 0; i < NB - 1; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int t = 0; t < 3; ++t) mfma_term(cur, i, j, t);
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    DFI_WAIT_VM(2 * LOADS_PER_STEP);
    asm volatile("s_barrier" ::: "memory");
    load_frags(std::integral_constant<int, (K + 1) % NS>{}, nxt, oA, oB);
    __builtin_amdgcn_sched_barrier(0);
    // the last row block term by term (four independent accumulators between fences), with the
    // refill's planes 0 and 1, 2, 3 after the three terms
#pragma unroll
    for (int t = 0; t < 3; ++t) {
#pragma unroll
      for (int j = 0; j < NB; ++j) mfma_term(cur, NB - 1, j, t);
      __builtin_amdgcn_sched_barrier(0);
      if (t == 0) issue_piece(k, s + NS, 0);
      issue_piece(k, s + NS, t + 1);
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  using K0 = std::integral_constant<int, 0>;
  using K1 = std::integral_constant<int, 1>;
  using K2 = std::integral_constant<int, 2>;
  using K3 = std::integral_constant<int, 3>;
  static_assert(NS == 4 && NB == 4, "the step loop is unrolled by the stage count");
  Frags f0, f1;
  if (nsteps > 0) {
    issue_step(K0{}, 0);
    issue_step(K1{}, 1);
    issue_step(K2{}, 2);
    issue_step(K3{}, 3);
    DFI_WAIT_VM(3 * LOADS_PER_STEP);
    asm volatile("s_barrier" ::: "memory");
    load_frags(K0{}, f0, oA0, oB0);
    int64_t s = 0;
    for (; s + 3 < nsteps; s += 4) {
      body(K0{}, f0, f1, s);
      body(K1{}, f1, f0, s + 1);
      body(K2{}, f0, f1, s + 2);
      body(K3{}, f1, f0, s + 3);
    }
    if (s < nsteps) body(K0{}, f0, f1, s);
    if (s + 1 < nsteps) body(K1{}, f1, f0, s + 1);
    if (s + 2 < nsteps) body(K2{}, f0, f1, s + 2);
    DFI_WAIT_VM(0);   // the trailing refills land in LDS before the workgroup ends
  }

  const float sgn = (slice & 1) ? -1.f : 1.f;
  float* out = part + (slice * ntri + tile) * (int64_t)(T * T);
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr * WT + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
        const int col = wc * WT + j * 32 + l32;
        out[row * T + col] = active ? sgn * acc[i][j][r] : 0.f;
      }
}

}  // namespace v4

// W_ij = sum over slices of the partial tiles (FP64, slice order) for i > j, plus the products of
// columns [ktail, m) that the tile kernel left out (FP64); W_ii = d_i + lambda.
// mirror != 0 also writes W_ji. One workgroup covers 256 consecutive columns j of one row i.
__global__ void gram_reduce_kernel(const float* __restrict__ part, int64_t n, int64_t ntri, int64_t nslice,
                                   const double* __restrict__ d, double lambda, double* __restrict__ W,
                                   int mirror, const float* __restrict__ S, int64_t lds, int64_t ktail, int64_t m) {
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
    // slices added in order; unrolled so that several slices' loads are in flight at once
    const float* pp = part + tile * (int64_t)(T * T) + off;
    const int64_t sstride = ntri * (int64_t)(T * T);
    int64_t sl = 0;
    for (; sl + 8 <= nslice; sl += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = pp[(sl + u) * sstride];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += (double)v[u];
    }
    for (; sl < nslice; ++sl) s += (double)pp[sl * sstride];
    for (int64_t k = ktail; k < m; ++k) s += (double)S[i * lds + k] * (double)S[j * lds + k];
  }
  W[i * n + j] = s;
  if (mirror && i != j) W[j * n + i] = s;
}

}  // namespace

GramPlan gram_plan(int64_t n, int64_t m, int64_t lds, int prec, bool aligned16, int q_override, int split_mode) {
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
  if (q_override > 0) best_q = q_override;
  p.nslice = 8 * best_q;
  const int64_t kstep = (prec == 2) ? 64 : KS;
  int64_t ks = (m + p.nslice - 1) / p.nslice;
  ks = (ks + kstep - 1) / kstep * kstep;
  if (ks < kstep) ks = kstep;
  p.kslice = ks;
  p.ldh = (prec == 1 && aligned16 && split_mode != 0) ? split_ldh(m) : 0;
  p.part_bytes = (size_t)p.nslice * (size_t)p.ntri * (size_t)(T * T) * sizeof(float);
  return p;
}

void gram_q_candidates(int64_t n, int64_t m, size_t max_part_bytes, int* out, int* count, int cap) {
  const int64_t ntile = (n + T - 1) / T;
  const int64_t ntri = ntile * (ntile + 1) / 2;
  const int64_t maxq = std::max<int64_t>(1, m / (8 * 2048));
  static const int qs[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};
  int c = 0;
  for (int q : qs) {
    if (q > 1 && q > maxq) break;
    if (q > 1 && (size_t)8 * q * ntri * T * T * sizeof(float) > max_part_bytes) break;
    if (c < cap) out[c++] = q;
  }
  *count = c;
}

hipError_t gram_launch_fp8(const GramPlan& p, const uint8_t* q, const uint8_t* sc, int64_t ldq, float* part,
                           hipStream_t st) {
  const dim3 grid((unsigned)(p.nslice * p.ntri));
  if ((ldq & 127) != 0 || ldq < p.m || p.nslice * p.kslice < ldq || (p.kslice & 63) != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(v3::gram_kernel_fp8, grid, dim3(v3::NT), 0, st, q, sc, p.n, ldq, p.ntri, p.nslice, p.kslice,
                     part);
  return hipGetLastError();
}

hipError_t gram_launch_fp8_grouped(const GramJob* jobs_dev, int njobs, int64_t nwg, hipStream_t st) {
  if (njobs < 1 || nwg < 1 || nwg > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(v3::gram_kernel_fp8_grouped, dim3((unsigned)nwg), dim3(v3::NT), 0, st, jobs_dev, njobs);
  return hipGetLastError();
}

hipError_t gram_launch_split(const GramPlan& p, const uint16_t* hi, const uint16_t* lo, float* part, hipStream_t st) {
  if (p.prec != 1 || p.ldh <= 0 || (p.ldh & 63) != 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(p.nslice * p.ntri));
  if (p.nslice * p.kslice < p.ldh || (p.kslice & 15) != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(v4::gram_kernel_split, grid, dim3(v4::NT), 0, st, hi, lo, p.n, p.ldh, p.ntri, p.nslice,
                     p.kslice, part);
  return hipGetLastError();
}

// Which tile kernel runs for an FP32 input S, and the first column it leaves to the reduction:
//   * FP32 products, 16-byte aligned rows: v2 (direct-to-LDS), columns [0, m rounded down to 4);
//   * split-BF16, or unaligned rows: v1 (register staging, conversion on the LDS store), all columns.
// (For split-BF16 the register-staged kernel converts each element once per workgroup; v2 would
// convert it once per reading wave, which measured slower.)
static bool use_v2(const GramPlan& p, const float* S) {
  const bool vec = ((p.lds & 3) == 0) && ((reinterpret_cast<uintptr_t>(S) & 15) == 0);
  return vec && p.prec == 0;
}

static int64_t tail_start(const GramPlan& p, const float* S) {
  if (p.prec == 2) return p.m;   // the FP8 kernel covers every column (zero codes past m)
  if (p.prec == 1 && p.ldh > 0) return p.m;   // the plane kernel covers every column (zeros past m)
  return use_v2(p, S) ? (p.m & ~(int64_t)3) : p.m;
}

int64_t gram_tail_start(const GramPlan& p, const float* S) { return tail_start(p, S); }

hipError_t gram_launch(const GramPlan& p, const float* S, float* part, hipStream_t st) {
  const bool vec = ((p.lds & 3) == 0) && ((reinterpret_cast<uintptr_t>(S) & 15) == 0);
  const dim3 grid((unsigned)(p.nslice * p.ntri));
  if (use_v2(p, S)) {
    hipLaunchKernelGGL((v2::gram_kernel_v2<0>), grid, dim3(v2::NT), 0, st, S, p.n, p.lds, p.m, p.ntri, p.nslice, p.kslice, part);
  } else if (p.prec == 0) {
    hipLaunchKernelGGL((gram_kernel<0, false>), grid, dim3(NTHR), 0, st, S, p.n, p.lds, p.m, p.ntri, p.nslice, p.kslice, part);
  } else if (vec) {
    hipLaunchKernelGGL((gram_kernel<1, true>), grid, dim3(NTHR), 0, st, S, p.n, p.lds, p.m, p.ntri, p.nslice, p.kslice, part);
  } else {
    hipLaunchKernelGGL((gram_kernel<1, false>), grid, dim3(NTHR), 0, st, S, p.n, p.lds, p.m, p.ntri, p.nslice, p.kslice, part);
  }
  return hipGetLastError();
}

hipError_t gram_reduce(const GramPlan& p, const float* S, const float* part, const double* d, double lambda,
                       double* W, int mirror, hipStream_t st) {
  const int64_t ktail = tail_start(p, S);   // first column the tile kernel left out
  const int64_t nb = (p.n + 255) / 256;
  const dim3 grid((unsigned)(nb * p.n));
  hipLaunchKernelGGL(gram_reduce_kernel, grid, dim3(256), 0, st, part, p.n, p.ntri, p.nslice, d, lambda, W, mirror,
                     S, p.lds, ktail, p.m);
  return hipGetLastError();
}

}  // namespace dfi
