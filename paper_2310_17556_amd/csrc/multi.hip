// Multi-vector streaming passes over S for many right-hand sides and damping values that share
// one S: the batched form of the right-to-left evaluation x = (v - S^T L^-T L^-1 S v) / lambda
// (Section 2), where one HBM pass over S serves up to MV = 16 vectors instead of one.
//
// Row pass  B_c = S V_c for c < nv. A workgroup owns 32 rows (4 per wave) and a group of
//           columns; per 256-column step the vectors' entries are staged once in LDS as FP64 and
//           each lane reuses its 4 columns of every vector for its 4 rows, with one FP64
//           accumulator per (row, vector). Vectors are FP32 (separate arrays, the caller's
//           right-hand sides) or FP64 interleaved T[k * MV + c] (the column pass output).
//           FP64 partials per (column group, vector, row) are added in fixed order by a second
//           kernel, which can also form refinement residuals r = b - lambda y - S t.
// Column pass t_c = S^T y_c for c < nc on the FP64 matrix cores. A wave owns 64 consecutive
//           columns and walks all rows, 4 at a time per product, with the y_c copied out
//           interleaved by row first. Output either T[k * MV + c] (FP64) or
//           x_c = (v_c - t_c) / lambda_c (FP32 or FP64), each column with its own v, x, lambda.
// Products of FP32 and FP64 values are formed and accumulated in FP64.
#include "dfisher_internal.h"

#include <algorithm>

namespace dfi {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int MV = MULTI_VECS;   // 16
constexpr int RM_STEP = 256;     // columns per wave step (4 per lane)

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ void load_s4(const float* __restrict__ p, int64_t col, int64_t c1, bool vec, f32x4& out) {
  if (vec && col + 4 <= c1) {
    out = *reinterpret_cast<const f32x4*>(p);
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e] = (col + e < c1) ? p[e] : 0.f;
  }
}

// Row pass B_c = S V_c for c < nv, the vectors either FP64 interleaved, T[k * MV + c] (the
// refinement's S t_c, from the column pass), or FP32 arrays vs.f[c] (the caller's right-hand
// sides). Grid: x = blocks of RT_ROWS rows, y = column groups of cg columns; part[(g * MV + c) * n
// + i] = sum over group g of S_ik V_c[k]. The workgroup's RT_WAVES waves (32 rows) share each
// 256-column step of the vectors through LDS, widened to FP64 (32 KB, double-buffered), so the
// vectors are read once per 32 rows of S instead of once per wave. In LDS each lane's 4 columns
// x 16 vectors (512 bytes) are padded by 16 bytes, so the 16-byte fragment reads of 16
// consecutive lanes cover all banks. Four rows per wave: the 4 x 16 FP64 accumulators take 128
// registers per lane. The next step's rows of S and share of the vectors are loaded while the
// current step's products run. This form serves the caller's FP32 right-hand sides, and T when
// 16 row strides do not fit a 32-bit buffer offset; otherwise rowpass_multi_tm_kernel takes T.
constexpr int RT_WAVES = 8;
constexpr int RT_RPW = 4;                    // rows per wave
constexpr int RT_ROWS = RT_WAVES * RT_RPW;   // 32 rows per workgroup
constexpr int RT_GROUP = 4 * MV + 2;         // doubles per lane group (4 columns x MV vectors + pad)
constexpr int RT_PIECES = 256 * MV / (2 * 64 * RT_WAVES);   // 16-byte pieces of T per thread and step

template <bool FP32V>
__global__ void __launch_bounds__(64 * RT_WAVES)
rowpass_multi_t_kernel(const float* __restrict__ S, int64_t n, int64_t m, int64_t lds, const double* __restrict__ T,
                       MultiVecs vs, int nv, int64_t cg, double* __restrict__ part, int vec) {
  __shared__ __attribute__((aligned(16))) double tl[2][64 * RT_GROUP];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * RT_ROWS + wave * RT_RPW;
  const int64_t g = blockIdx.y;
  const int64_t c0 = g * cg;
  const int64_t c1 = min(m, c0 + cg);
  // waves whose rows lie past n still load their share of T and meet the barriers
  const int nr = (int)max<int64_t>(0, min<int64_t>(RT_RPW, n - row0));

  double acc[RT_RPW][MV];
#pragma unroll
  for (int r = 0; r < RT_RPW; ++r)
#pragma unroll
    for (int c = 0; c < MV; ++c) acc[r][c] = 0.0;

  // This thread's share of one step of the vectors, loaded into registers: FP32V, vector tid / 32
  // and 8 consecutive columns (two 16-byte loads, zero past c1 and for vectors c >= nv); else
  // RT_PIECES 16-byte pieces of T[cs .. cs + 256) x MV (zero past c1).
  static_assert(!FP32V || 64 * RT_WAVES == 32 * MV, "one vector per 32 threads");
  struct VecShare {
    f32x4 f[2];
    f64x2 t[RT_PIECES];
  };
  auto load_vecs = [&](int64_t cs, VecShare& vsh) {
    if constexpr (FP32V) {
      const int c = tid >> 5;
      const int cl0 = (tid & 31) * 8;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int cl = cl0 + 4 * h;
        vsh.f[h] = (f32x4){0.f, 0.f, 0.f, 0.f};
        if (c < nv) load_s4(vs.f[c] + cs + cl, cs + cl, c1, (vec & 2) != 0, vsh.f[h]);
      }
    } else {
#pragma unroll
      for (int h = 0; h < RT_PIECES; ++h) {
        const int idx = 2 * (h * 64 * RT_WAVES + tid);   // double index in the step: column idx / MV, vector idx % MV
        vsh.t[h] = (f64x2){0.0, 0.0};
        if (cs + idx / MV < c1) vsh.t[h] = *reinterpret_cast<const f64x2*>(T + cs * MV + idx);
      }
    }
  };
  // ... and stored to LDS, widened to FP64, in the layout the products read
  auto store_vecs = [&](const VecShare& vsh, double* tb) {
    if constexpr (FP32V) {
      const int c = tid >> 5;
      const int cl0 = (tid & 31) * 8;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 4; ++e) tb[((cl0 + 4 * h) >> 2) * RT_GROUP + e * MV + c] = (double)vsh.f[h][e];
    } else {
#pragma unroll
      for (int h = 0; h < RT_PIECES; ++h) {
        const int idx = 2 * (h * 64 * RT_WAVES + tid);
        const int cl = idx / MV;
        *reinterpret_cast<f64x2*>(&tb[(cl >> 2) * RT_GROUP + (cl & 3) * MV + (idx % MV)]) = vsh.t[h];
      }
    }
  };
  auto load_rows = [&](int64_t cs, f32x4* sv) {
    const int64_t col = cs + 4 * lane;
#pragma unroll
    for (int r = 0; r < RT_RPW; ++r) {
      sv[r] = (f32x4){0.f, 0.f, 0.f, 0.f};
      if (r < nr) load_s4(S + (row0 + r) * lds + col, col, c1, (vec & 1) != 0, sv[r]);
    }
  };
  // Software pipeline: step cs + 256's rows of S and share of the vectors are loaded into
  // registers while step cs's products run, so each step's loads have a whole step to arrive.
  VecShare vn;
  f32x4 sn[RT_RPW];
  if (c0 < c1) {
    load_vecs(c0, vn);
    load_rows(c0, sn);
  }
  int buf = 0;
  for (int64_t cs = c0; cs < c1; cs += RM_STEP, buf ^= 1) {
    store_vecs(vn, tl[buf]);
    __syncthreads();   // the other buffer is rewritten only after the next step's barrier
    f32x4 sv[RT_RPW];
#pragma unroll
    for (int r = 0; r < RT_RPW; ++r) sv[r] = sn[r];
    if (cs + RM_STEP < c1) {
      load_vecs(cs + RM_STEP, vn);
      load_rows(cs + RM_STEP, sn);
    }
    const double* tg = &tl[buf][lane * RT_GROUP];
    // one column at a time: its MV vector entries are live only while its products are formed
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      double vv[MV];
#pragma unroll
      for (int c = 0; c < MV; c += 2) {
        const f64x2 t2 = *reinterpret_cast<const f64x2*>(tg + e * MV + c);
        vv[c] = t2[0];
        vv[c + 1] = t2[1];
      }
#pragma unroll
      for (int r = 0; r < RT_RPW; ++r) {
        const double sd = (double)sv[r][e];
#pragma unroll
        for (int c = 0; c < MV; ++c) acc[r][c] = fma(sd, vv[c], acc[r][c]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int r = 0; r < RT_RPW; ++r) {
    if (r >= nr) continue;
#pragma unroll
    for (int c = 0; c < MV; ++c) {
      const double t = wave_sum(acc[r][c]);
      if (lane == 0 && c < nv) part[(g * MV + c) * n + row0 + r] = t;
    }
  }
}

// The row pass with the FP64 vectors T on the FP64 matrix cores. A wave owns 16 rows; a
// workgroup of RG_WAVES waves (64 rows) walks its column group 256 columns at a time, with that
// step of T staged in LDS (double-buffered, each group of 4 columns' 64 values padded to 80 so that
// a product's B-operand read touches each bank at most twice). Per step each lane = 16 kr + q loads
// row r0 + q, columns 16 u + 4 kr .. + 3 for u < 16 (16 loads of 16 bytes: the wave reads 1 KB of
// each of its rows), and product (u, j) takes element j of load u as its A operand (row q, column
// 16 u + 4 kr + j) and T[16 u + 4 kr + j][q] from LDS as its B operand: D(16 rows x 16 vectors) +=
// S(16 x 4) T(4 x 16) with v_mfma_f64_16x16x4f64. Lane l then holds D[row kr + 4 r][vector q] in
// register r, the partial this wave stores for the group. Rows past n and columns past c1 read
// as zero.
constexpr int RG_WAVES = 4;
constexpr int RG_ROWS = 16 * RG_WAVES;
constexpr int RG_GSTRIDE = 80;                        // doubles per 4-column group in LDS (64 used)

// NG groups of up to MV vectors (T0, T1) share every load of S: with NG = 2 each 16-byte piece of
// S feeds eight products instead of four, and the step is 128 columns so that the two groups'
// double-buffered LDS stages (80 KB) still let two workgroups share a compute unit.
template <int NG>
__global__ void __launch_bounds__(64 * RG_WAVES, 2)
rowpass_multi_tm_kernel(const float* __restrict__ S, int64_t n, int64_t m, int64_t lds, const double* __restrict__ T0,
                        const double* __restrict__ T1, int nv0, int nv1, int64_t cg, double* __restrict__ part0,
                        double* __restrict__ part1, int vec) {
  constexpr int STEP = NG == 1 ? 256 : 128;             // columns per step
  constexpr int BUF = (STEP / 4) * RG_GSTRIDE;          // doubles per LDS buffer and group
  constexpr int PIECES = STEP * MV / 2 / (64 * RG_WAVES);   // 16-byte pieces of T per thread, step, group
  constexpr int NU = STEP / 16;                         // 16-byte loads of S per lane and step
  __shared__ __attribute__((aligned(16))) double tl[2][NG][BUF];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane & 15, kr = lane >> 4;
  const int64_t rbase = (int64_t)blockIdx.x * RG_ROWS + wave * 16;
  const int64_t g = blockIdx.y;
  const int64_t c0 = g * cg;
  const int64_t c1 = min(m, c0 + cg);
  // waves whose rows lie past n still stage their share of T and meet the barriers
  auto load_t = [&](const double* T, int64_t cs, f64x2* tv) {
#pragma unroll
    for (int h = 0; h < PIECES; ++h) {
      const int idx = 2 * (h * 64 * RG_WAVES + tid);   // double index in the step: column idx / MV, vector idx % MV
      tv[h] = (f64x2){0.0, 0.0};
      if (cs + idx / MV < c1) tv[h] = *reinterpret_cast<const f64x2*>(T + cs * MV + idx);
    }
  };
  auto store_t = [&](const f64x2* tv, double* tb) {
#pragma unroll
    for (int h = 0; h < PIECES; ++h) {
      const int idx = 2 * (h * 64 * RG_WAVES + tid);
      const int cl = idx / MV;
      *reinterpret_cast<f64x2*>(&tb[(cl >> 2) * RG_GSTRIDE + (cl & 3) * MV + (idx % MV)]) = tv[h];
    }
  };
  // The wave's 16 rows of S as one buffer from a wave-uniform base (row rbase, column c0) with a
  // 32-bit lane offset (the launcher checks 16 lds * 4 < 2^31): the records end at row n, so lanes
  // of rows past n read zeros, and a wave with no rows below n has no records and touches no memory.
  const int rin = (int)max<int64_t>(0, min<int64_t>(16, n - rbase));
  const float* sbase = S + (rin > 0 ? rbase : 0) * lds + c0;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(sbase), 0, rin > 0 ? (int)((int64_t)rin * lds * 4) : 0, 0x00020000);
  const uint32_t qoff = (uint32_t)((int64_t)q * lds * 4);
  // NA independent accumulators per group (product j of each load into accumulator j % NA), added
  // in a fixed order at the end: with NG = 2 a single chain of dependent products per group would
  // leave the matrix cores waiting on each product's result
  constexpr int NA = NG == 2 ? 2 : 1;
  f64x4 acc[NG][NA];
  f64x2 tv[NG][PIECES];
#pragma unroll
  for (int gg = 0; gg < NG; ++gg)
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[gg][a] = (f64x4){0.0, 0.0, 0.0, 0.0};
  if (c0 < c1) {
#pragma unroll
    for (int gg = 0; gg < NG; ++gg) {
      load_t(gg ? T1 : T0, c0, tv[gg]);
      store_t(tv[gg], tl[0][gg]);
    }
  }
  __syncthreads();
  // S of the next step is loaded while this step's products run (NG = 2: the products of a step
  // take about as long as the loads' latency, which would otherwise be exposed every step)
  auto load_s = [&](int64_t cs, f32x4* sv) {
    const int kc = (int)(cs - c0);
#pragma unroll
    for (int u = 0; u < NU; ++u)
      sv[u] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                            rs, (int)(qoff + 4u * (uint32_t)(kc + 16 * u + 4 * kr)), 0, 0));
  };
  f32x4 sn[NU];
  if (NG == 2 && c0 < c1) load_s(c0, sn);
  int buf = 0;
  for (int64_t cs = c0; cs < c1; cs += STEP, buf ^= 1) {
    const bool more = cs + STEP < c1;
    if (more) {   // the next step's T, stored after this step's products
#pragma unroll
      for (int gg = 0; gg < NG; ++gg) load_t(gg ? T1 : T0, cs + STEP, tv[gg]);
    }
    f32x4 sv[NU];
    if constexpr (NG == 2) {
#pragma unroll
      for (int u = 0; u < NU; ++u) sv[u] = sn[u];
      if (more) load_s(cs + STEP, sn);
    } else {
      load_s(cs, sv);
    }
    // columns past c1 (in the group's last step only) count as zero: a select, no branch
    const int lim = (int)min<int64_t>(c1 - cs, STEP);
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) sv[u][e] = (16 * u + 4 * kr + e < lim) ? sv[u][e] : 0.f;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double a = (double)sv[u][j];
#pragma unroll
        for (int gg = 0; gg < NG; ++gg) {
          const double b = tl[buf][gg][(4 * u + kr) * RG_GSTRIDE + j * MV + q];
          acc[gg][j % NA] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[gg][j % NA], 0, 0, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);   // widen load u's values only where its products use them
    }
    if (more) {   // the other buffer was last read before the previous barrier
#pragma unroll
      for (int gg = 0; gg < NG; ++gg) store_t(tv[gg], tl[buf ^ 1][gg]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int gg = 0; gg < NG; ++gg) {
    if (q >= (gg ? nv1 : nv0)) continue;
    double* part = gg ? part1 : part0;
    f64x4 tot = acc[gg][0];
#pragma unroll
    for (int a = 1; a < NA; ++a) tot += acc[gg][a];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rr = rbase + kr + 4 * r;
      if (rr < n) part[(g * MV + q) * n + rr] = tot[r];
    }
  }
}

// out.b[c][i] = sum_g part[(g * MV + c) * n + i]; with out.r0[c] set:
// out.b[c][i] = (r0_c[i] - lam_c y_c[i]) - sum_g part[...] (refinement residual).
__global__ void rowpass_multi_reduce_kernel(const double* __restrict__ part, int64_t n, int64_t ngroups, int nv,
                                            MultiOut out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n || c >= nv) return;
  double s = 0.0;
  for (int64_t g = 0; g < ngroups; ++g) s += part[(g * MV + c) * n + i];
  const double* r0 = out.r0[c];
  out.b[c][i] = r0 ? (r0[i] - out.lam[c] * out.y[c][i]) - s : s;
}

// Yi[i * stride + off + c] = mc.y[c][i] for i < n, c < MV: the y vectors interleaved by row.
__global__ void interleave_y_kernel(MultiCols mc, int64_t n, int stride, int off, double* __restrict__ Yi) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * MV) return;
  Yi[(idx / MV) * stride + off + idx % MV] = mc.y[idx % MV][idx / MV];
}

// The column pass on the FP64 matrix cores: per wave 64 consecutive columns, D_j(16 vectors x 16
// columns) += Y(4 rows x 16 vectors)^T S(4 rows x 16 columns) with v_mfma_f64_16x16x4f64. Lane l
// = 16 kr + q loads row i + kr, columns col .. col + 3 (col = c0 + 4 q) of S with one 16-byte load
// and supplies element j to product j (columns col + j: D_j covers columns c0 + 4 n + j); its A
// operand is Yi[(i + kr) MV + q], one 8-byte load. Lane l holds D_j[vector kr + 4 r][n = q] in
// register r. Each product adds 4 rows (its k = 4) in FP64; rows past n and columns past m read
// as zero. The accumulators take 32 registers per lane, so many waves keep loads in flight.
constexpr int CF_WAVES = 4;
constexpr int CF_COLS = 64;    // columns per wave
constexpr int CF_GROUPS = 4;   // 4-row groups per loop step
static_assert(MV == 16, "one MFMA dimension holds the vectors");

template <int MODE, int NG>
__global__ void __launch_bounds__(64 * CF_WAVES)
colpass_multi_mfma_kernel(const float* __restrict__ S, int64_t n, int64_t m, int64_t lds, MultiCols mc0, int nc0,
                          MultiCols mc1, int nc1, const double* __restrict__ Yi, double* __restrict__ T0,
                          double* __restrict__ T1, int vec, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t c0 = ((int64_t)blockIdx.x * CF_WAVES + wave) * CF_COLS;
  if (c0 >= m) return;   // the whole wave
  const int q = lane & 15, kr = lane >> 4;
  const int64_t col = c0 + 4 * q;
  const bool full = vec && (col + 4 <= m);
  auto load_s = [&](int64_t row) {
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (row < n) {
      const float* p = S + row * lds + col;
      if (full) {
        v = *reinterpret_cast<const f32x4*>(p);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (col + e < m) ? p[e] : 0.f;
      }
    }
    return v;
  };
  // Yi holds NG groups of MV vectors per row: Yi[row (NG MV) + g MV + c]
  auto load_y = [&](int64_t row, int gg) { return row < n ? Yi[row * (MV * NG) + gg * MV + q] : 0.0; };
  f64x4 acc[NG][4];
#pragma unroll
  for (int gg = 0; gg < NG; ++gg)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[gg][j] = (f64x4){0.0, 0.0, 0.0, 0.0};
  // NG = 2: the next rows' S and y are loaded while this iteration's products run
  f32x4 sn[CF_GROUPS];
  double yn[NG][CF_GROUPS];
  auto load_rows = [&](int64_t i, f32x4* sv, double (*ya)[CF_GROUPS]) {
#pragma unroll
    for (int g = 0; g < CF_GROUPS; ++g) {
      sv[g] = load_s(i + 4 * g + kr);
#pragma unroll
      for (int gg = 0; gg < NG; ++gg) ya[gg][g] = load_y(i + 4 * g + kr, gg);
    }
  };
  if (NG == 2) load_rows(0, sn, yn);
  for (int64_t i = 0; i < n; i += 4 * CF_GROUPS) {
    f32x4 sv[CF_GROUPS];
    double ya[NG][CF_GROUPS];
    if constexpr (NG == 2) {
#pragma unroll
      for (int g = 0; g < CF_GROUPS; ++g) {
        sv[g] = sn[g];
#pragma unroll
        for (int gg = 0; gg < NG; ++gg) ya[gg][g] = yn[gg][g];
      }
      if (i + 4 * CF_GROUPS < n) load_rows(i + 4 * CF_GROUPS, sn, yn);
    } else {
      load_rows(i, sv, ya);
    }
#pragma unroll
    for (int g = 0; g < CF_GROUPS; ++g)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double b = (double)sv[g][j];
#pragma unroll
        for (int gg = 0; gg < NG; ++gg) acc[gg][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[gg][g], b, acc[gg][j], 0, 0, 0);
      }
  }
#pragma unroll
  for (int gg = 0; gg < NG; ++gg) {
    if constexpr (MODE == 2) {
      double* T = gg ? T1 : T0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (col + j >= m) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) T[(col + j) * MV + kr + 4 * r] = acc[gg][j][r];
      }
    } else {
      const MultiCols& mc = gg ? mc1 : mc0;
      const int nc = gg ? nc1 : nc0;
      // vector by vector with a uniform index into the argument arrays: vector c lives in register
      // c / 4 of the lanes with kr = c % 4
#pragma unroll
      for (int c = 0; c < MV; ++c) {
        if (c < nc && kr == (c & 3)) {
          const float* vc = mc.v[c];
          const double lam = mc.lam[c];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int64_t k = col + j;
            if (k < m) {
              const double x = ((double)vc[k] - acc[gg][j][c >> 2]) / lam;
              if constexpr (MODE == 0) static_cast<float*>(mc.x[c])[k] = (float)x;
              else static_cast<double*>(mc.x[c])[k] = x;
            }
          }
        }
      }
    }
  }
}

__global__ void axpy_many_kernel(double* __restrict__ y, const double* __restrict__ d, int64_t len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) y[i] += d[i];
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

RowMultiPlan rowmulti_plan(int64_t n, int64_t m, int64_t lds) {
  RowMultiPlan p{};
  p.n = n;
  p.m = m;
  p.lds = lds;
  const int64_t rowblocks = (n + RT_ROWS - 1) / RT_ROWS;
  const int64_t target = std::max<int64_t>(1, 2048 / rowblocks);       // ~2048 workgroups
  const int64_t maxg = (m + 2047) / 2048;                                // >= 2048 columns per group
  p.nchunk = std::max<int64_t>(1, std::min(target, maxg));
  int64_t cg = (m + p.nchunk - 1) / p.nchunk;
  cg = (cg + RM_STEP - 1) / RM_STEP * RM_STEP;
  p.chunk = cg;
  p.nchunk = (m + cg - 1) / cg;
  p.part_bytes = (size_t)p.nchunk * MV * (size_t)n * sizeof(double);
  return p;
}

hipError_t rowpass_multi_launch(const RowMultiPlan& p, const float* S, const MultiVecs& vs, const double* T, int nv,
                                double* part, hipStream_t st) {
  if (nv < 1 || nv > MV) return hipErrorInvalidValue;
  const bool vec = ((p.lds & 3) == 0) && aligned16(S);
  bool vecv = true;
  if (!T)
    for (int c = 0; c < nv; ++c) vecv = vecv && aligned16(vs.f[c]);
  const int iv = (vec ? 1 : 0) | (vecv ? 2 : 0);
  const dim3 grid((unsigned)((p.n + RT_ROWS - 1) / RT_ROWS), (unsigned)p.nchunk);
  if (T && 16 * p.lds * 4 < ((int64_t)1 << 31) && p.chunk < ((int64_t)1 << 28))
    hipLaunchKernelGGL(rowpass_multi_tm_kernel<1>, dim3((unsigned)((p.n + RG_ROWS - 1) / RG_ROWS), (unsigned)p.nchunk),
                       dim3(64 * RG_WAVES), 0, st, S, p.n, p.m, p.lds, T, (const double*)nullptr, nv, 0, p.chunk,
                       part, (double*)nullptr, iv);
  else if (T)
    hipLaunchKernelGGL(rowpass_multi_t_kernel<false>, grid, dim3(64 * RT_WAVES), 0, st, S, p.n, p.m, p.lds, T, vs, nv,
                       p.chunk, part, iv);
  else
    hipLaunchKernelGGL(rowpass_multi_t_kernel<true>, grid, dim3(64 * RT_WAVES), 0, st, S, p.n, p.m, p.lds,
                       (const double*)nullptr, vs, nv, p.chunk, part, iv);
  return hipGetLastError();
}

hipError_t rowpass_multi_launch2(const RowMultiPlan& p, const float* S, const double* T0, int nv0, const double* T1,
                                 int nv1, double* part0, double* part1, hipStream_t st) {
  if (nv0 < 1 || nv0 > MV || nv1 < 1 || nv1 > MV || !T0 || !T1) return hipErrorInvalidValue;
  if (16 * p.lds * 4 >= ((int64_t)1 << 31) || p.chunk >= ((int64_t)1 << 28)) {   // two single-group passes
    const MultiVecs none{};
    const hipError_t e = rowpass_multi_launch(p, S, none, T0, nv0, part0, st);
    if (e != hipSuccess) return e;
    return rowpass_multi_launch(p, S, none, T1, nv1, part1, st);
  }
  const bool vec = ((p.lds & 3) == 0) && aligned16(S);
  hipLaunchKernelGGL(rowpass_multi_tm_kernel<2>, dim3((unsigned)((p.n + RG_ROWS - 1) / RG_ROWS), (unsigned)p.nchunk),
                     dim3(64 * RG_WAVES), 0, st, S, p.n, p.m, p.lds, T0, T1, nv0, nv1, p.chunk, part0, part1,
                     vec ? 3 : 2);
  return hipGetLastError();
}

hipError_t rowpass_multi_reduce(const RowMultiPlan& p, const double* part, int nv, const MultiOut& out,
                                hipStream_t st) {
  if (nv < 1 || nv > MV) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((p.n + 255) / 256), (unsigned)nv);
  hipLaunchKernelGGL(rowpass_multi_reduce_kernel, grid, dim3(256), 0, st, part, p.n, p.nchunk, nv, out);
  return hipGetLastError();
}

hipError_t colpass_multi_launch(const float* S, int64_t n, int64_t m, int64_t lds, const MultiCols& mc, int nc,
                                int mode, double* T, double* Yi, hipStream_t st, const int* skip) {
  if (nc < 1 || nc > MV || !Yi) return hipErrorInvalidValue;
  const bool vec = ((lds & 3) == 0) && aligned16(S);
  hipLaunchKernelGGL(interleave_y_kernel, dim3((unsigned)((n * MV + 255) / 256)), dim3(256), 0, st, mc, n, MV, 0, Yi);
  const dim3 grid((unsigned)((m + CF_WAVES * CF_COLS - 1) / (CF_WAVES * CF_COLS)));
  const dim3 block(64 * CF_WAVES);
  const double* yi = Yi;
  const MultiCols none{};
  double* const nul = nullptr;
  switch (mode) {
    case 0:
      hipLaunchKernelGGL((colpass_multi_mfma_kernel<0, 1>), grid, block, 0, st, S, n, m, lds, mc, nc, none, 0, yi, T,
                         nul, vec ? 1 : 0, skip);
      break;
    case 1:
      hipLaunchKernelGGL((colpass_multi_mfma_kernel<1, 1>), grid, block, 0, st, S, n, m, lds, mc, nc, none, 0, yi, T,
                         nul, vec ? 1 : 0, skip);
      break;
    case 2:
      hipLaunchKernelGGL((colpass_multi_mfma_kernel<2, 1>), grid, block, 0, st, S, n, m, lds, mc, nc, none, 0, yi, T,
                         nul, vec ? 1 : 0, skip);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t colpass_multi_launch2(const float* S, int64_t n, int64_t m, int64_t lds, const MultiCols& mc0, int nc0,
                                 const MultiCols& mc1, int nc1, int mode, double* T0, double* T1, double* Yi,
                                 hipStream_t st, const int* skip) {
  if (nc0 < 1 || nc0 > MV || nc1 < 1 || nc1 > MV || !Yi) return hipErrorInvalidValue;
  if (mode == 2 && (!T0 || !T1)) return hipErrorInvalidValue;
  const bool vec = ((lds & 3) == 0) && aligned16(S);
  const unsigned ib = (unsigned)((n * MV + 255) / 256);
  hipLaunchKernelGGL(interleave_y_kernel, dim3(ib), dim3(256), 0, st, mc0, n, 2 * MV, 0, Yi);
  hipLaunchKernelGGL(interleave_y_kernel, dim3(ib), dim3(256), 0, st, mc1, n, 2 * MV, MV, Yi);
  const dim3 grid((unsigned)((m + CF_WAVES * CF_COLS - 1) / (CF_WAVES * CF_COLS)));
  const dim3 block(64 * CF_WAVES);
  const double* yi = Yi;
  switch (mode) {
    case 0:
      hipLaunchKernelGGL((colpass_multi_mfma_kernel<0, 2>), grid, block, 0, st, S, n, m, lds, mc0, nc0, mc1, nc1, yi,
                         T0, T1, vec ? 1 : 0, skip);
      break;
    case 1:
      hipLaunchKernelGGL((colpass_multi_mfma_kernel<1, 2>), grid, block, 0, st, S, n, m, lds, mc0, nc0, mc1, nc1, yi,
                         T0, T1, vec ? 1 : 0, skip);
      break;
    case 2:
      hipLaunchKernelGGL((colpass_multi_mfma_kernel<2, 2>), grid, block, 0, st, S, n, m, lds, mc0, nc0, mc1, nc1, yi,
                         T0, T1, vec ? 1 : 0, skip);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t axpy_many(double* y, const double* d, int64_t len, hipStream_t st) {
  hipLaunchKernelGGL(axpy_many_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, y, d, len);
  return hipGetLastError();
}

}  // namespace dfi
