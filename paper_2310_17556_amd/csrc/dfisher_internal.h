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
  int prec;           // dfisher_gram_prec (0 FP32, 1 split-BF16, 2 scaled FP8)
  int64_t ldh;        // split-BF16 from pre-split planes: their row stride (0: split inside the tile kernel)
  size_t part_bytes;  // FP32 partial tiles: nslice * ntri * TILE * TILE * 4
};

// aligned16: rows of S start on 16-byte boundaries (lds % 4 == 0 and S 16-byte aligned). For
// split-BF16 on aligned rows the plan uses planes hi/lo written by the row pass (ldh > 0).
// q_override > 0 fixes the split-K factor (nslice = 8 q); split_mode 0 keeps split-BF16 inside the
// tile kernel even on aligned rows (-1: planes whenever possible).
GramPlan gram_plan(int64_t n, int64_t m, int64_t lds, int prec, bool aligned16, int q_override = 0,
                   int split_mode = -1);
// The split-K factors q (nslice = 8 q) worth trying for a shape: every q from 1 up to the largest
// that keeps >= 2048 columns per slice and the partial tiles within max_part_bytes.
void gram_q_candidates(int64_t n, int64_t m, size_t max_part_bytes, int* out, int* count, int cap);
hipError_t gram_launch(const GramPlan& p, const float* S, float* part, hipStream_t st);
// The first column the tile kernel of plan p leaves to gram_reduce.
int64_t gram_tail_start(const GramPlan& p, const float* S);
// Row stride (bf16 elements) of the split-BF16 planes for m columns.
inline int64_t split_ldh(int64_t m) { return (m + 63) / 64 * 64; }
// Split-BF16 Gram from the column-blocked planes hi = bf16(S), lo = bf16(S - hi) (p.ldh > 0).
hipError_t gram_launch_split(const GramPlan& p, const uint16_t* hi, const uint16_t* lo, float* part, hipStream_t st);
// Scaled-FP8 Gram from the row pass's column-blocked codes and E8M0 scales (see rowpass_launch).
hipError_t gram_launch_fp8(const GramPlan& p, const uint8_t* q, const uint8_t* sc, int64_t ldq, float* part,
                           hipStream_t st);
// Many problems' scaled-FP8 Grams in one launch: job j (plan-checked like gram_launch_fp8: kcap =
// its ldq) owns workgroups [wg0, wg0 + ntri nslice), wg0 a multiple of 8, jobs sorted by wg0;
// nwg = the last wg0 + ntri nslice.
struct GramJob {
  const uint8_t* q;
  const uint8_t* sc;
  float* part;
  int64_t n, kcap, ntri, nslice, kslice, wg0;
};
hipError_t gram_launch_fp8_grouped(const GramJob* jobs_dev, int njobs, int64_t nwg, hipStream_t st);
// Row stride of the FP8 codes for m columns (a multiple of 64).
inline int64_t fp8_ldq(int64_t m) { return (m + 127) / 128 * 128; }   // scale rows: whole 4-byte words
// W = sum of slices (lower triangle; also upper if mirror), diagonal = d + lambda (d = FP64 row norms).
// S is needed for the products of the last few columns (m mod 4, 8 or 16), which the tile kernels
// that stream whole 16-byte chunks leave out.
hipError_t gram_reduce(const GramPlan& p, const float* S, const float* part, const double* d, double lambda,
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
// With q != nullptr the pass also writes the scaled-FP8 copy of S (codes n x ldq bytes, E8M0
// scale bytes n x ldq/32; ldq a multiple of 64, >= m; needs 16-byte aligned rows and want_d).
// Row-major, or with `blocked` (ldq a multiple of 128) in the column-blocked layout the
// scaled-FP8 Gram reads: codes in 64-column blocks, each holding all n rows contiguously, code
// (i, k) at q[((k / 64) n + i) 64 + k % 64]; scale byte (i, k / 32) at sc[((k / 128) n + i) 4 + (k / 32) % 4].
hipError_t rowpass_launch(const RowPassPlan& p, const float* S, const float* v, const double* vd,
                          bool want_b, bool want_d, double* part, hipStream_t st, uint8_t* q = nullptr,
                          uint8_t* sc = nullptr, int64_t ldq = 0, bool blocked = false);
// Row pass that also writes the split-BF16 planes of S: hi = bf16_rne(S), lo = bf16_rne(S - hi),
// column-blocked in 16-column blocks of all n rows: element (i, k) at [((k / 16) n + i) 16 + k % 16]
// (ldh = m rounded up to 64; entries k >= m are zero). Needs 16-byte aligned rows; always
// computes d, and b when v != nullptr.
hipError_t rowpass_launch_split(const RowPassPlan& p, const float* S, const float* v, double* part, uint16_t* hi,
                                uint16_t* lo, int64_t ldh, hipStream_t st);
// Reduce: b_i = sum_c part_b[c][i]; when r0 != nullptr: b_i = r0_i - lam * y_i - sum_c part_b[c][i]
hipError_t rowpass_reduce(const RowPassPlan& p, const double* part, bool want_b, bool want_d, double* b,
                          double* d, const double* r0, const double* y, double lam, hipStream_t st);

// Column pass: t_k = sum_i S_ik y_i (FP64). mode 0: x = (v - t)/lambda as FP32,
// mode 1: same as FP64, mode 2: store t itself as FP64 (for the refinement residual), mode 3:
// t rounded once to FP32 (v and lambda unused in modes 2 and 3).
// When m is small the rows are split over nsplit workgroups; `part` (part_bytes) then holds
// FP64 partial sums.
struct ColPassPlan {
  int64_t nsplit;     // row splits
  int64_t rps;        // rows per split
  size_t part_bytes;  // nsplit * m * 8 when nsplit > 1, else 0
};
ColPassPlan colpass_plan(int64_t n, int64_t m);
// skip (device int, may be null): when *skip != 0 at run time the kernels return at once.
hipError_t colpass_launch(const ColPassPlan& p, const float* S, int64_t n, int64_t m, int64_t lds, const double* y,
                          const float* v, double lambda, void* out, int mode, double* part, hipStream_t st,
                          const int* skip = nullptr);

// Fused refinement pass: part[g][i] = per-workgroup partials of (S S^T y)_i with one read of S
// (n <= 4096, m >= 16, 16-byte aligned rows; `usable` is false otherwise and
// the caller takes the column pass + row pass). The last m % 16 columns add one more group.
// refine_pass_reduce: r_i = b_i - lam y_i - sum_g part[g][i] in fixed order.
struct RefinePassPlan {
  int64_t n;
  int nch;            // 16-byte loads per lane and block (8, 16 or 32)
  bool usable;
  int64_t ngroups;    // workgroups (one per compute unit, or per compute unit and row half)
  bool tail;          // m % block width != 0: one more partial group for the last columns
  bool line;          // whole-line kernels: 32-column blocks (8 lanes per 128-byte row piece)
  int lnch;           // line, not split: loads per lane (8, 16, 32 for n <= 512, 1024, 2048)
  bool split;         // line, rows split over workgroup pairs (2048 < n <= 4096)
  int64_t R;          // line: blocks per workgroup (per pair when split)
  size_t xch_off;     // split: offset (doubles) of the exchanged column partials in part
  size_t xch_len;     // split: doubles of exchange slots (2 members x 64 values per pair and block)
  size_t part_bytes;  // (ngroups + tail) * n * 8 (+ the split's exchange buffers)
};
// split_ok = false keeps the one-workgroup-per-block kernel (smaller workspace)
RefinePassPlan refine_pass_plan(int64_t n, int64_t m, int64_t lds, const float* S, bool split_ok = true);
// skip (device int, may be null): when *skip != 0 at run time the kernels return at once (a
// problem whose refinement stopped, in a launch sequence fixed in advance). spin: the split
// kernel's bound on polls for its partner's partials (< 0: the default; 0: always compute them).
// tout / csout (whole-line kernels only, may be null): the pass also writes t = S^T y and the
// column sums S^T 1 (FP64, m entries), both from the sums it forms for the product.
hipError_t refine_pass_launch(const RefinePassPlan& p, const float* S, int64_t n, int64_t m, int64_t lds,
                              const double* y, double* part, hipStream_t st, const int* skip = nullptr,
                              int spin = -1, double* tout = nullptr, double* csout = nullptr);
hipError_t refine_pass_reduce(const RefinePassPlan& p, const double* part, double* r, const double* b,
                              const double* y, double lam, hipStream_t st, const int* skip = nullptr);
// Many problems' whole-line passes in one launch (plans with line && !split, all of one lnch):
// job j runs workgroups [wg0, wg0 + ngroups) of its own plan (R blocks each) on its S, writing its
// partials to part (ngroups x n doubles), S^T u to tout and S^T 1 to csout (cs launches) when set;
// skip as for refine_pass_launch. Jobs sorted by wg0, contiguous; nwg = the last wg0 + ngroups.
struct LineJob {
  const float* S;
  const double* u;
  double* part;
  double* tout;
  double* csout;
  const int* skip;
  int64_t n, m, lds, R, wg0, ngroups;
};
hipError_t refine_line_grouped_launch(const LineJob* jobs_dev, int njobs, int nch, bool cs, int64_t nwg,
                                      hipStream_t st);
// Their residuals in one launch: job j owns blocks [blk0, blk0 + ceil(n / 16)) and forms
// out = rhs - lam u - sum of its ngroups partials (refine_pass_reduce's arithmetic). nblk = the last
// blk0 + ceil(n / 16).
struct ReduceJob {
  const double* part;
  const double* rhs;
  const double* u;
  double* out;
  const int* skip;
  double lam;
  int64_t n, ngroups, blk0;
};
hipError_t refine_reduce_grouped(const ReduceJob* jobs_dev, int njobs, int64_t nblk, hipStream_t st);

// ----------------------------------------------------------------------------- multi-vector passes
// One pass over S for up to MULTI_VECS vectors (batched right-hand sides / damping values).
constexpr int MULTI_VECS = 16;
struct MultiVecs {                 // FP32 input vectors of length m (row pass)
  const float* f[MULTI_VECS];
};
struct MultiOut {                  // row-pass results of length n
  double* b[MULTI_VECS];           // output c
  const double* r0[MULTI_VECS];    // if set: b_c = r0_c - lam_c y_c - S t_c (refinement residual)
  const double* y[MULTI_VECS];
  double lam[MULTI_VECS];
};
struct MultiCols {                 // column-pass operands, per vector c
  const double* y[MULTI_VECS];     // length n (every slot must point to valid memory)
  const float* v[MULTI_VECS];      // length m (modes 0, 1)
  void* x[MULTI_VECS];             // length m, FP32 (mode 0) or FP64 (mode 1)
  double lam[MULTI_VECS];
};
struct RowMultiPlan {
  int64_t n, m, lds;
  int64_t nchunk, chunk;
  size_t part_bytes;               // nchunk * MULTI_VECS * n * 8
};
RowMultiPlan rowmulti_plan(int64_t n, int64_t m, int64_t lds);
// part <- per-group partials of S V_c, c < nv. V_c = vs.f[c] (FP32) or, with T != nullptr, the FP64
// interleaved T[k * MULTI_VECS + c] written by colpass_multi_launch mode 2.
hipError_t rowpass_multi_launch(const RowMultiPlan& p, const float* S, const MultiVecs& vs, const double* T, int nv,
                                double* part, hipStream_t st);
hipError_t rowpass_multi_reduce(const RowMultiPlan& p, const double* part, int nv, const MultiOut& out,
                                hipStream_t st);
// t_c = S^T y_c (c < nc). mode 2: T[k * MULTI_VECS + c] = t_c[k] (T: m * MULTI_VECS doubles); mode 0 / 1:
// x_c = (v_c - t_c) / lam_c as FP32 / FP64. Yi: scratch of n * MULTI_VECS doubles (the y_c
// interleaved by row).
hipError_t colpass_multi_launch(const float* S, int64_t n, int64_t m, int64_t lds, const MultiCols& mc, int nc,
                                int mode, double* T, double* Yi, hipStream_t st, const int* skip = nullptr);
// Two groups of vectors (mc0: nc0, mc1: nc1, each 1 .. MULTI_VECS) in one pass over S: every load
// of S feeds both groups' products. mode 2 writes T0 and T1 (each m * MULTI_VECS); Yi: scratch of
// n * 2 * MULTI_VECS doubles.
hipError_t colpass_multi_launch2(const float* S, int64_t n, int64_t m, int64_t lds, const MultiCols& mc0, int nc0,
                                 const MultiCols& mc1, int nc1, int mode, double* T0, double* T1, double* Yi,
                                 hipStream_t st, const int* skip = nullptr);
// The row pass over two groups' T (T0: nv0, T1: nv1 vectors) in one pass over S; partials into
// part0 and part1 (each of the plan's part_bytes), reduced with rowpass_multi_reduce per group.
hipError_t rowpass_multi_launch2(const RowMultiPlan& p, const float* S, const double* T0, int nv0, const double* T1,
                                 int nv1, double* part0, double* part1, hipStream_t st);
// y += d over len entries
hipError_t axpy_many(double* y, const double* d, int64_t len, hipStream_t st);

// ----------------------------------------------------------------------------- Cholesky
// In-place blocked FP64 Cholesky (row-major, lower). info_dev: device int64, 0 or 1-based
// index of the first bad pivot. flag_dev: device int32 scratch (stop flag). dkk: device
// scratch of 64 x 64 doubles (the inverses of the current diagonal block's four 16 x 16
// diagonal sub-blocks, for the panel solve).
constexpr size_t POTRF_DKK_BYTES = 64 * 64 * sizeof(double);
hipError_t potrf_launch(double* A, int64_t n, int64_t* info_dev, int32_t* flag_dev, double* dkk, hipStream_t st);
// nbatch independent factorisations in the same launches: matrix b at A + b sA, info_dev[b],
// flag_dev[b], dkk + b 64 * 64 (nbatch <= 65535).
hipError_t potrf_launch_batched(double* A, int64_t n, int64_t nbatch, int64_t sA, int64_t* info_dev, int32_t* flag_dev,
                                double* dkk, hipStream_t st);
// Matrices of different sizes in the same launches: one job per matrix (device table, njobs <= 65535),
// nmax = the largest n. Each job's info / flag are cleared first.
struct FactorJob {
  double* A;         // n x n, factored in place
  int64_t n;
  int64_t* info;     // 0 or the 1-based index of the first bad pivot
  int32_t* flag;     // stop flag
  double* dkk;       // 64 x 64 scratch
};
hipError_t potrf_launch_grouped(const FactorJob* jobs_dev, int64_t njobs, int64_t nmax, hipStream_t st);

// ----------------------------------------------------------------------------- triangular solves
// Inverses of the 64 x 64 diagonal blocks of L and their transposes (Dinv: trsv_dinv_bytes(n)),
// computed once per factor.
size_t trsv_dinv_bytes(int64_t n);
hipError_t trsv_diag_inv(const double* L, int64_t n, double* Dinv, hipStream_t st);
// y = L^-1 b (trans 0) or L^-T b (trans 1); work: n doubles, not aliasing b or y; b may alias y.
hipError_t trsv_launch(const double* L, const double* Dinv, int64_t n, int trans, const double* b, double* y,
                       double* work, hipStream_t st);
// Batched: nfac factors at L + f sL with their block inverses at Dinv + f trsv_dinv_bytes(n) / 8.
hipError_t trsv_diag_inv_batched(const double* L, int64_t sL, int64_t n, int64_t nfac, double* Dinv, hipStream_t st);
// nvec right-hand sides (vector j at b + j n, result at y + j n, work nvec x n) solved in the same
// launches; vector j uses factor j / nper. nvec <= 65535.
hipError_t trsv_launch_batched(const double* L, int64_t sL, const double* Dinv, int64_t n, int64_t nvec, int64_t nper,
                               int trans, const double* b, double* y, double* work, hipStream_t st);
// Systems of different sizes in the same launches (device job table, njobs <= 65535; nmax = the
// largest n). diag_inv: Dinv of each L. Solve: r holds the right-hand side on entry and is reduced
// in place (it is the work vector); the solution goes to out (not aliasing r).
struct TrsvJob {
  const double* L;
  double* Dinv;
  int64_t n;
  double* r;
  double* out;
};
hipError_t trsv_diag_inv_grouped(const TrsvJob* jobs_dev, int64_t njobs, int64_t nmax, hipStream_t st);
hipError_t trsv_launch_grouped(const TrsvJob* jobs_dev, int64_t njobs, int64_t nmax, int trans, hipStream_t st);

// ----------------------------------------------------------------------------- refinement (PCG)
// n-vector steps of conjugate gradients on W y = b preconditioned by the Gram's factor (pcg.hip).
// Segments of a concatenated vector array: s -> [seg[2 s], seg[2 s] + seg[2 s + 1]) from a device
// table of (offset, length) pairs, or [s n, s n + n) when seg is null; a launch covers s0 .. s1 - 1, per-segment scalars at index s.
// pcg_init: p = z, rz = r.z. pcg_step: with nq = -(W p): alpha = rz / (p.W p), y += alpha p,
// r -= alpha W p, rr = r.r (rr may be null). pcg_dir: rz' = r.z, p = z + (rz' / rz) p, rz = rz'.
// pcg_finish: y += z.
// stop (device, per segment, may be null): segments with stop[s] != 0 are left alone.
hipError_t pcg_init(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, const double* r, const double* z, double* p,
                    double* rz, hipStream_t st, const int* stop = nullptr);
// alpha (may be null): the step length of each segment is also stored there.
hipError_t pcg_step(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, const double* p, const double* nq, double* y,
                    double* r, const double* rz, double* rr, hipStream_t st, const int* stop = nullptr,
                    double* alpha = nullptr);
hipError_t pcg_dir(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, const double* r, const double* z, double* p,
                   double* rz, hipStream_t st, const int* stop = nullptr);
// out[s] = |x_s|^2
hipError_t seg_sumsq(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, const double* x, double* out,
                     hipStream_t st);
// Device-side stop test of refinement sweeps (per segment, no host round trip): after sweep `sweep`
// the segment's residual rho = sqrt(rr / bb) is compared with tol (predicted as in the host test
// when `predict`), and a segment that meets it or reaches cap[s] takes y += zc and stops (with
// `keep`, zc is left for the final step instead: final_decide adds it or takes its image).
struct PcgControl {
  const double* bb;   // |b_s|^2
  const double* rr;   // |r_s|^2 of the current iterate
  double* prev;       // rho of the previous sweep (1 at the start)
  int* stop;          // 1 once the segment has stopped
  const int* cap;     // sweep cap per segment
  int* done;          // sweeps the segment ran
  double* resid;      // its last rho
  int* met;           // 1 if it stopped on tol
  double tol;         // 0: stop at the cap only
  double floor;       // least contraction a prediction assumes
  int predict;
  int keep;           // 1: a stopping segment leaves y alone (zc stays for the final step)
};
hipError_t pcg_decide(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, int sweep, const PcgControl& c,
                      const double* zc, double* y, hipStream_t st);
hipError_t pcg_control_init(int64_t nseg, const PcgControl& c, hipStream_t st);
hipError_t pcg_finish(const int64_t* seg, int64_t n, int64_t s0, int64_t s1, const double* z, double* y,
                      hipStream_t st);

// ----------------------------------------------------------------------------- SR front end, complex variant
// (sr.hip) S_ij = fl32((O_ij - t_j / n) / sqrt(n)) from the FP64 column sums t of O; cplx: O is
// complex (interleaved FP32 pairs, row stride ldo complex elements, t interleaved) and the output is
// the stacked Z = [Re S; Im S] (2n x m, row stride lds). Real O and S may be the same array.
hipError_t center_write(const float* O, int64_t n, int64_t m, int64_t ldo, int cplx, const double* t, float* S,
                        int64_t lds, hipStream_t st);
// Preconditioner of a centered S: W (n x n, FP64, lower triangle; both triangles when full) becomes
// M = P W P + lambda U U^T, U the normalised indicators of nseg (1 or 2) equal segments, unless
// W's Rayleigh quotient along an indicator (less lambda) exceeds 1 % of its mean diagonal (then W
// is left unchanged: S is not centered). work: gram_project_work_bytes(n) bytes (tile partials
// and totals), r: nseg * n doubles.
size_t gram_project_work_bytes(int64_t n);
hipError_t gram_project(double* W, int64_t n, int nseg, double lambda, int full, double* work, double* r,
                        hipStream_t st,
                        int* applied = nullptr);
hipError_t fill_value(double* y, int64_t n, double value, hipStream_t st);
// interleaved complex FP32 v (m) -> out[0..m) real parts, out[m..2m) imaginary parts
hipError_t deinterleave(const float* v, int64_t m, float* out, hipStream_t st);
// Wh = [[Wr, -Wi], [Wi, Wr]] + lambda I (2n x 2n) from G = Z Z^T (2n x 2n, both triangles)
hipError_t complex_embed(const double* G, int64_t n, double lambda, double* Wh, hipStream_t st);
// out = rhs - lambda y + sgn [P_top - Q_bot; P_bot + Q_top] (each 2n; rhs, y may be null)
hipError_t complex_combine(const double* P, const double* Q, int64_t n, double sgn, const double* rhs, const double* y,
                           double lambda, double* out, hipStream_t st);
// u1 = [y_top; y_bot], u2 = [y_bot; -y_top]
hipError_t complex_colvecs(const double* y, int64_t n, double* u1, double* u2, hipStream_t st);
// x_k = (v_k - (T[16 k] + i T[16 k + 1])) / lambda, complex interleaved, FP32 or FP64
hipError_t complex_apply(const float* v, const double* T, int64_t m, double lambda, void* x, int x_fp64,
                         hipStream_t st);

// ----------------------------------------------------------------------------- small helpers
// dst = src + scale * dmax[0] * I (n x n, row-major; dmax a device scalar, unread if scale == 0).
hipError_t shift_copy(const double* src, double* dst, int64_t n, double scale, const double* dmax, hipStream_t st);
// dst = src + lam * I
hipError_t add_diag_copy(const double* src, double* dst, int64_t n, double lam, hipStream_t st);
// dst = src + (lam + scale * dmax[0]) * I (dmax unread if scale == 0)
hipError_t shift_add_copy(const double* src, double* dst, int64_t n, double scale, const double* dmax, double lam,
                          hipStream_t st);
// y += d (length n)
hipError_t axpy_inplace(double* y, const double* d, int64_t n, hipStream_t st);
// y = 0 (length n; a kernel, not a memset, so that it may sit in a captured graph)
hipError_t fill_zero(double* y, int64_t n, hipStream_t st);
// max_i W_ii
hipError_t diag_max(const double* W, int64_t n, double* out_dev, hipStream_t st);
// *out_dev = sum_i x_i^2 (FP64, deterministic)
hipError_t sumsq(const double* x, int64_t n, double* out_dev, hipStream_t st);
// zero the strict upper triangle
hipError_t zero_upper(double* A, int64_t n, hipStream_t st);

// ----------------------------------------------------------------------------- final step through the FP8 codes
// The apply x = (v - S^T y) / lambda after the last refinement correction z (apply8.hip). The passes
// carry T = S^T y_c exactly for the iterate y_c before that correction (the residual pass writes
// S^T y_0, each conjugate-gradient pass S^T p, added with its step length), so
// S^T (y_c + z) = T + S^T z, and only the image of the small correction is left to take: through
// the scaled-FP8 copy Q of S the row pass wrote (one byte per entry instead of four). That costs a
// relative error of about 3 % of |S^T z|, which final_decide estimates and allows only while it is
// far below the solve's target.
// t_axpy: T += alpha[0] U (m entries); nothing when skip (device, may be null) is set.
hipError_t t_axpy(double* T, const double* U, const double* alpha, int64_t m, hipStream_t st,
                  const int* skip = nullptr);
// One workgroup. abar = mean(z) when *centered (device, may be null: not centered; the all-ones component, whose image is the exact
// abar S^T 1 = abar cs), zf = float(z - abar); est = sqrt(sum_i d_i zf_i^2 / (y.b - lambda y.y))
// (d_i = |s_i|^2: the expected size of Q^T zf - S^T zf over the relative rounding error, for rounding
// errors independent between entries, against |S^T y|). use = est <= est_max; otherwise y += z
// (the exact apply then takes the corrected iterate).
hipError_t final_decide(int64_t n, double* y, const double* z, const double* b, const double* d, double lambda,
                        const int* centered, double est_max, float* zf, double* abar, int* use, hipStream_t st);
// When *use: x_j = (v_j - T_j - abar cs_j - sum_i Q_ij zf_i) / lambda (cs may be null: abar is 0
// then), FP32 or FP64 x, codes and scales in the row pass's column-blocked layout (ldq a multiple
// of 128). Otherwise returns at once.
hipError_t fp8_apply(const uint8_t* q, const uint8_t* sc, int64_t ldq, int64_t n, int64_t m, const float* zf,
                     const double* T, const double* cs, const double* abar, const float* v, double lambda, void* x,
                     int x64, const int* use, hipStream_t st);

// Many vectors (the batched call): T in the multi-vector passes' layout, groups of 16 vectors
// interleaved by column, T[(g m + j) 16 + c] for vector 16 g + c. t_axpy_multi: T += alpha_v U per
// vector. put_values: count doubles from the host array vals to device memory through kernel
// arguments (no copy node: safe in a captured sequence). multi_final8: per vector the decision
// (zb = bf16(z - abar), ldz a multiple of 64 >= n, zeros past n; abar; usev), flag[0] = every
// vector may take the codes; unless so Y += Z for every vector (the caller then runs the exact
// passes, skipped by flag[0]); if so X_v = (V_{v mod nrhs} - T_v - abar_v cs - (Z Q)_v) / lamv[v / nrhs]
// through the bf16 matrix cores, T_v = Tacc_v (+ alpha_v Ulast_v when Ulast is given: the last
// direction's S^T p, added there instead of by t_axpy_multi).
hipError_t t_axpy_multi(double* T, const double* U, const double* alpha, int64_t m, int64_t nvec, hipStream_t st);
hipError_t put_values(double* out, const double* vals, int64_t count, hipStream_t st);
hipError_t multi_final8(const uint8_t* q, const uint8_t* sc, int64_t ldq, int64_t n, int64_t m, int64_t nvec,
                        int64_t nrhs, double* Y, const double* Z, const double* B, const double* d,
                        const double* lamv, const int* centered, double est_max, void* zb, int64_t ldz,
                        double* abar, int* usev, int* flag, const double* Tacc, const double* Ulast,
                        const double* alpha, const double* cs, const float* V, int64_t ldv, void* X, int64_t ldx,
                        int x64, hipStream_t st);

}  // namespace dfi
