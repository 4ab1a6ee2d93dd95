// Internal interfaces between the C ABI (dfisher.cpp) and the HIP kernels. Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace dfi {

// ----------------------------------------------------------------------------- Gram (SYRK)
// Lower-triangle tile SYRK on the matrix cores. A work item is (tile, k-slice); each writes its
// FP32 partial tile to `part`, and gram_reduce sums the slices in FP64 in a fixed order.
constexpr int GRAM_TILE = 256;   // output tile edge (rows and columns of W per workgroup)
constexpr int GRAM_KSTEP = 32;   // columns of S staged through LDS per step

struct GramPlan {
  int64_t n, m, lds;
  int64_t ntile;      // tiles per edge = ceil(n / GRAM_TILE)
  int64_t ntri;       // lower-triangle tiles = ntile (ntile + 1) / 2
  int64_t nslice;     // k-slices (split-K factor)
  int64_t kslice;     // columns per slice (multiple of GRAM_KSTEP)
  int prec;           // dfisher_gram_prec
  size_t part_bytes;  // FP32 partial tiles: nslice * ntri * TILE * TILE * 4
};

GramPlan gram_plan(int64_t n, int64_t m, int64_t lds, int prec);
hipError_t gram_launch(const GramPlan& p, const float* S, float* part, hipStream_t st);
// W = sum of slices (lower triangle; also upper if mirror), diagonal = d + lambda (d = FP64 row norms).
hipError_t gram_reduce(const GramPlan& p, const float* part, const double* d, double lambda,
                       double* W, int mirror, hipStream_t st);

// ----------------------------------------------------------------------------- streaming GEMVs
// Row pass: b = S v (if v != nullptr) and d_i = |s_i|^2 (if d != nullptr), FP64 accumulation.
// `vd` (FP64 vector) may replace `v` (FP32) for the refinement residual; at most one is set.
// Partials per (row, column chunk) go to `part`, then are reduced in fixed order.
struct RowPassPlan {
  int64_t n, m, lds;
  int64_t nchunk;     // column chunks
  int64_t chunk;      // columns per chunk
  size_t part_bytes;  // 2 * nchunk * n * 8
};
RowPassPlan rowpass_plan(int64_t n, int64_t m, int64_t lds);
hipError_t rowpass_launch(const RowPassPlan& p, const float* S, const float* v, const double* vd,
                          bool want_b, bool want_d, double* part, hipStream_t st);
// Reduce: b_i = sum_c part_b[c][i]; when r0 != nullptr: b_i = r0_i - lam * y_i - sum_c part_b[c][i]
hipError_t rowpass_reduce(const RowPassPlan& p, const double* part, bool want_b, bool want_d, double* b,
                          double* d, const double* r0, const double* y, double lam, hipStream_t st);

// Column pass: t_k = sum_i S_ik y_i (FP64). mode 0: x = (v - t)/lambda as FP32,
// mode 1: same as FP64, mode 2: store t itself as FP64 (for the refinement residual).
// When m is small the rows are split over nsplit workgroups; `part` (part_bytes) then holds
// FP64 partial sums.
struct ColPassPlan {
  int64_t nsplit;     // row splits
  int64_t rps;        // rows per split
  size_t part_bytes;  // nsplit * m * 8 when nsplit > 1, else 0
};
ColPassPlan colpass_plan(int64_t n, int64_t m);
hipError_t colpass_launch(const ColPassPlan& p, const float* S, int64_t n, int64_t m, int64_t lds, const double* y,
                          const float* v, double lambda, void* out, int mode, double* part, hipStream_t st);

// ----------------------------------------------------------------------------- Cholesky
// In-place blocked FP64 Cholesky (row-major, lower). info_dev: device int64, 0 or 1-based
// index of the first bad pivot. flag_dev: device int32 scratch (stop flag).
hipError_t potrf_launch(double* A, int64_t n, int64_t* info_dev, int32_t* flag_dev, hipStream_t st);

// ----------------------------------------------------------------------------- triangular solves
hipError_t trsv_launch(const double* L, int64_t n, int trans, const double* b, double* y, hipStream_t st);
size_t trsv_lds_bytes(int64_t n, int trans);
hipError_t trsv_prepare();  // once per device, before the first launch

// ----------------------------------------------------------------------------- small helpers
// dst = src + tau * I (n x n, row-major), copies the full matrix.
hipError_t shift_copy(const double* src, double* dst, int64_t n, double tau, hipStream_t st);
// y += d (length n)
hipError_t axpy_inplace(double* y, const double* d, int64_t n, hipStream_t st);
// max_i W_ii
hipError_t diag_max(const double* W, int64_t n, double* out_dev, hipStream_t st);
// zero the strict upper triangle
hipError_t zero_upper(double* A, int64_t n, hipStream_t st);

}  // namespace dfi
