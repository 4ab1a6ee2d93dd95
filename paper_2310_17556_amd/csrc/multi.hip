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
// Column pass t_c = S^T y_c for c < nc. A workgroup owns 1024 consecutive columns (4 per lane)
//           and walks all rows; y_c[i] is wave-uniform. Output either T[k * MV + c] (FP64) or
//           x_c = (v_c - t_c) / lambda_c (FP32 or FP64), each column with its own v, x, lambda.
// Products of FP32 and FP64 values are formed and accumulated in FP64.
#include "dfisher_internal.h"

#include <algorithm>

namespace dfi {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

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
// registers per lane.
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

constexpr int CM_THREADS = 256;
constexpr int CM_COLS = 4 * CM_THREADS;
constexpr int CM_UNROLL = 4;

// MODE 2: T[k * MV + c] = t_c[k]; MODE 0 / 1: x_c[k] = (v_c[k] - t_c[k]) / lam_c as FP32 / FP64.
// Vectors c >= nc are computed from y_0 and discarded.
template <int MODE>
__global__ void __launch_bounds__(CM_THREADS)
colpass_multi_kernel(const float* __restrict__ S, int64_t n, int64_t m, int64_t lds, MultiCols mc, int nc,
                     double* __restrict__ T, int vec) {
  const int64_t col = (int64_t)blockIdx.x * CM_COLS + 4 * threadIdx.x;
  if (col >= m) return;
  const bool full = vec && (col + 4 <= m);
  double t[4][MV];
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int c = 0; c < MV; ++c) t[e][c] = 0.0;
  int64_t i = 0;
  for (; i < n; i += CM_UNROLL) {
    f32x4 sv[CM_UNROLL];
#pragma unroll
    for (int u = 0; u < CM_UNROLL; ++u) {
      sv[u] = (f32x4){0.f, 0.f, 0.f, 0.f};
      if (i + u < n) {
        const float* p = S + (i + u) * lds + col;
        if (full) {
          sv[u] = *reinterpret_cast<const f32x4*>(p);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) sv[u][e] = (col + e < m) ? p[e] : 0.f;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < CM_UNROLL; ++u) {
      if (i + u >= n) break;
#pragma unroll
      for (int c = 0; c < MV; ++c) {
        const double yc = mc.y[c][i + u];
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e][c] = fma((double)sv[u][e], yc, t[e][c]);
      }
    }
  }
  if constexpr (MODE == 2) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t k = col + e;
      if (k < m) {
#pragma unroll
        for (int c = 0; c < MV; c += 2) *reinterpret_cast<f64x2*>(T + k * MV + c) = (f64x2){t[e][c], t[e][c + 1]};
      }
    }
  } else {
    // vector-major, every index a constant after unrolling (a loop that stops at nc would keep
    // the argument arrays in scratch memory)
#pragma unroll
    for (int c = 0; c < MV; ++c) {
      if (c < nc) {
        const float* vc = mc.v[c];
        const double lam = mc.lam[c];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t k = col + e;
          if (k < m) {
            const double x = ((double)vc[k] - t[e][c]) / lam;
            if constexpr (MODE == 0) static_cast<float*>(mc.x[c])[k] = (float)x;
            else static_cast<double*>(mc.x[c])[k] = x;
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
  if (T)
    hipLaunchKernelGGL(rowpass_multi_t_kernel<false>, grid, dim3(64 * RT_WAVES), 0, st, S, p.n, p.m, p.lds, T, vs, nv,
                       p.chunk, part, iv);
  else
    hipLaunchKernelGGL(rowpass_multi_t_kernel<true>, grid, dim3(64 * RT_WAVES), 0, st, S, p.n, p.m, p.lds,
                       (const double*)nullptr, vs, nv, p.chunk, part, iv);
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
                                int mode, double* T, hipStream_t st) {
  if (nc < 1 || nc > MV) return hipErrorInvalidValue;
  const bool vec = ((lds & 3) == 0) && aligned16(S);
  const dim3 grid((unsigned)((m + CM_COLS - 1) / CM_COLS));
  switch (mode) {
    case 0:
      hipLaunchKernelGGL((colpass_multi_kernel<0>), grid, dim3(CM_THREADS), 0, st, S, n, m, lds, mc, nc, T, vec ? 1 : 0);
      break;
    case 1:
      hipLaunchKernelGGL((colpass_multi_kernel<1>), grid, dim3(CM_THREADS), 0, st, S, n, m, lds, mc, nc, T, vec ? 1 : 0);
      break;
    case 2:
      hipLaunchKernelGGL((colpass_multi_kernel<2>), grid, dim3(CM_THREADS), 0, st, S, n, m, lds, mc, nc, T, vec ? 1 : 0);
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
