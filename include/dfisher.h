/*
 * dfisher - damped Fisher solves on AMD Instinct MI355X (gfx950).
 *
 * Solves the damped Fisher system of Eq. 1 of Chen, Xie & Wang, "Efficient Numerical
 * Algorithm for Large-Scale Damped Natural Gradient Descent" (arXiv 2310.17556):
 *
 *     (S^T S + lambda I_m) x = v,     S in R^{n x m} (n samples, m parameters), lambda > 0,
 *
 * with Algorithm 1 (Section 2): W = S S^T + lambda I_n, L = Chol(W), and
 * x = (v - S^T L^-T L^-1 S v) / lambda evaluated right to left with triangular solves
 * (the inlined form recommended after Algorithm 1), so that Q = L^-1 S is never formed.
 *
 * Conventions shared by every entry point
 *   Memory     S, v, x, V, X, W, L, b, y are DEVICE pointers owned by the caller. The library
 *              allocates only its own workspace, held by the context. Sizes are int64.
 *   Layout     S is row-major n x m FP32 with row stride lds >= m elements (row i is sample
 *              i's scaled score vector). n x n matrices (W, L) are row-major FP64 with row
 *              stride n. Vectors are dense.
 *   Streams    `stream` is a hipStream_t passed as void*; NULL is the default stream. All
 *              device work of a call is enqueued on that stream.
 *   Sync       Calls that factor W (dfisher_solve, dfisher_factor_create, dfisher_potrf,
 *              dfisher_solve_batched, dfisher_solve_uneven) synchronise the stream once per
 *              factorisation to read the Cholesky status; dfisher_solve_batched with the
 *              DFISHER_ASYNC flag does not (its statuses stay on the device). The others return
 *              without synchronising.
 *   Errors     Every call returns a dfisher_status and never aborts or throws. Arguments are
 *              validated on the host before any device call: null pointers, n < 1, m < 1,
 *              lds < m, lambda not finite or not > 0, and unknown enum values return
 *              DFISHER_E_INVALID_ARG. A missing device or any HIP runtime error returns
 *              DFISHER_E_DEVICE. dfisher_last_error() gives a per-thread message for the
 *              last failure.
 *   Threads    Calls on one context must not overlap. Different contexts are independent.
 */
#ifndef DFISHER_H
#define DFISHER_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define DFISHER_API __attribute__((visibility("default")))
#else
#define DFISHER_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dfisher_status {
  DFISHER_OK = 0,
  DFISHER_E_INVALID_ARG = 1,   /* rejected on the host; nothing was enqueued            */
  DFISHER_E_NOT_SPD = 2,       /* Cholesky met a pivot that is not > 0 (info says where) */
  DFISHER_E_NO_MEMORY = 3,     /* workspace allocation failed                            */
  DFISHER_E_DEVICE = 4,        /* no usable device, or a HIP runtime error               */
  DFISHER_E_NOT_CONVERGED = 5, /* a tolerance was set and no measured refinement residual
                                  met it within opt->sweeps sweeps; x is still written    */
  DFISHER_E_UNSUPPORTED = 6    /* valid request this build does not implement            */
} dfisher_status;

/* Arithmetic of the Gram S S^T (Algorithm 1 step 1, the O(n^2 m) term of Section 2).
 * All forms multiply on the matrix cores with FP32 accumulation inside a K-chunk and FP64
 * accumulation across chunks; the diagonal is always the exact FP64 squared row norm. */
typedef enum dfisher_gram_prec {
  DFISHER_GRAM_FP32 = 0,    /* FP32 inputs, FP32 matrix-core products                      */
  DFISHER_GRAM_BF16X3 = 1,  /* split-BF16: S = hi + lo, keeps hi.hi + hi.lo + lo.hi        */
  DFISHER_GRAM_MXFP8 = 2    /* scaled FP8: E4M3 codes with one power-of-two scale per row
                               and 32-column block (see dfisher_quantize_mxfp8); needs rows
                               aligned to 16 bytes (lds a multiple of 4)                   */
} dfisher_gram_prec;

/* What to do when the Cholesky of the computed W meets a pivot that is not > 0 (the computed
 * Gram can lose definiteness along directions where W's eigenvalue is close to lambda). */
typedef enum dfisher_shift_policy {
  DFISHER_SHIFT_NONE = 0,        /* fail with DFISHER_E_NOT_SPD                                 */
  DFISHER_SHIFT_ON_FAILURE = 1,  /* refactor W + tau I with growing tau (reported in info);
                                    refinement sweeps then correct against the unshifted W   */
  DFISHER_SHIFT_ALWAYS = 2       /* factor W + tau I from the start, tau = 2 sqrt(n) u max_i W_ii
                                    with u = 2^-24 for the FP32 and split-BF16 Grams and
                                    u = 0.25 / sqrt(m) for the scaled-FP8 Gram (above the
                                    rounding error of the computed Gram), so the factored
                                    matrix dominates the exact W and every refinement sweep
                                    contracts; grows like DFISHER_SHIFT_ON_FAILURE if the
                                    Cholesky still fails. Meant for sweeps >= 1.              */
} dfisher_shift_policy;

typedef struct dfisher_options {
  int32_t gram_prec;     /* dfisher_gram_prec                                               */
  int32_t sweeps;        /* FP64 refinement sweeps on W y = S v (one read of S each; see below),
                            0..16 or DFISHER_SWEEPS_AUTO                                      */
  int32_t shift_policy;  /* dfisher_shift_policy                                            */
  int32_t x_fp64;        /* 0: x (and X) are float*, 1: double*                             */
  double tol;            /* 0: run exactly `sweeps` sweeps. > 0 (dfisher_solve, _rowspace,
                            _complex and _uneven; other entry points return
                            DFISHER_E_UNSUPPORTED): after forming sweep k's
                            residual r_k = S v - lambda y_k - S (S^T y_k), read
                            rho_k = |r_k|_2 / |S v|_2 (one stream synchronisation per sweep),
                            apply that sweep's correction, and stop once rho_k <= tol; with
                            `sweeps` as the cap. Finite and >= 0.                             */
  int32_t final_resid;   /* 1: after the last sweep, measure the relative residual of the
                            returned iterate, w_resid = |S v - lambda y - S (S^T y)|_2 / |S v|_2
                            (FP64 accumulation, one more pass over S, not applied) and report
                            it in info->w_resid. dfisher_solve and dfisher_solve_uneven only
                            (other entry points return DFISHER_E_UNSUPPORTED). 0 or 1.        */
  int32_t flags;         /* bitwise OR of DFISHER_CENTERED, DFISHER_ASYNC and
                            DFISHER_EXACT_APPLY below, or 0; other bits are
                            DFISHER_E_INVALID_ARG                                              */
} dfisher_options;

/* opt->flags: the caller declares that every column of S sums to zero over the samples (1^T S = 0),
 * as the SR score matrix of Section 3 does (dfisher_sr_center writes one). S S^T then has the
 * all-ones vector as a null vector, W maps it to lambda times itself, and a Gram formed from
 * rounded inputs misses that by far more than a small lambda (for the scaled-FP8 Gram about 1e-3
 * of the diagonal), which makes its factor a poor preconditioner along that one direction. With
 * the flag the factored matrix is the computed W with that direction made exact,
 *     M = P W P + lambda 1 1^T / n,   P = I - 1 1^T / n   (FP64, before the Cholesky),
 * and for dfisher_solve_complex the same with the indicators of the A and B halves of Z (the real
 * and imaginary halves of the real embedding). The declaration is checked against the computed
 * Gram on the device: when its Rayleigh quotient along an indicator (less lambda) exceeds 1 % of
 * its mean diagonal, S is plainly not centered and W is factored unchanged (the result is then
 * bitwise that of the call without the flag). The refinement sweeps use the exact W either way,
 * so only their convergence (and the sweeps-0 result, M^-1 rather than the computed W^-1) depends
 * on the flag. Honoured by dfisher_solve, _rowspace, _complex, _batched, _uneven and
 * dfisher_factor_create. */
#define DFISHER_CENTERED 1

/* opt->flags: enqueue without waiting (dfisher_solve_batched only; the other entry points return
 * DFISHER_E_UNSUPPORTED). The call puts all of its device work on `stream` and returns without
 * synchronising or reading anything back, so that the caller can capture it into a HIP graph
 * (stream capture on `stream`, any capture mode) and replay it. With the flag:
 *   - infos is a DEVICE pointer to nlam records (or NULL), written by the call's last kernel;
 *     read them after the stream has finished. A failed factorisation shows there only
 *     (potrf_info != 0, that lambda's x unspecified): the return value reports argument,
 *     workspace and HIP errors, never DFISHER_E_NOT_SPD.
 *   - shift_policy must be DFISHER_SHIFT_NONE or DFISHER_SHIFT_ALWAYS; DFISHER_SHIFT_ON_FAILURE
 *     refactors after a host-side decision and returns DFISHER_E_UNSUPPORTED. DFISHER_SWEEPS_AUTO
 *     is the a-priori count (as without the flag when no factorisation fails).
 *   - no autotuning runs (the context's tuning table, or the default plan, is used).
 *   - the workspace cannot be allocated during a capture: make the same call once outside the
 *     capture first, or the captured call returns DFISHER_E_UNSUPPORTED. A call captured on a
 *     context fixes the context's workspace for the rest of its life, since the graph holds its
 *     addresses: later calls on that context that need more workspace return
 *     DFISHER_E_UNSUPPORTED. A replay uses the workspace as a call does: replays and other calls
 *     on the context must not overlap.
 * Results are bitwise those of the same call without the flag. */
#define DFISHER_ASYNC 2

/* The final step x = (v - S^T y) / lambda (step 6 of Algorithm 1) of dfisher_solve with the
 * scaled-FP8 Gram and at least one refinement sweep: the refinement passes carry S^T y_c exactly
 * for the iterate before the last correction z (y = y_c + z), and the image S^T z of that small
 * correction can be taken through the FP8 copy of S that the Gram already made (a quarter of the
 * bytes of S) instead of a fourth read of S. Its error, about 3 % of |S^T z| for independent
 * rounding errors, is estimated on the device from the row norms and z, and the FP8 image is used
 * only while that estimate is about 1e-7 of |S^T y| or less (otherwise the exact column pass runs;
 * nothing waits for the host either way). For a declared centered S the all-ones component of z is
 * taken exactly, through the column sums S^T 1 the first refinement pass forms. The flag below
 * always takes the exact pass. Needs 16-byte aligned rows and n <= 4096 (the passes that carry
 * S^T y), opt->final_resid = 0. */
#define DFISHER_EXACT_APPLY 4

/* Refinement sweeps. Each sweep reads S once. Sweep 1 forms the FP64 residual r = S v - lambda y
 * - S (S^T y) of y = L^-T L^-1 S v; the sweeps after it are conjugate-gradient iterations on
 * W y = S v preconditioned by the Cholesky factor of the computed Gram (one product W p per sweep,
 * FP64 accumulation); after the last sweep the correction L^-T L^-1 r of the final residual is
 * added. One sweep is thus the classic correction y += L^-T L^-1 (S v - W y).
 *
 * opt->sweeps = DFISHER_SWEEPS_AUTO lets the library choose the sweep count.
 *   dfisher_solve: measured. After each sweep's residual rho_k = |r_k| / |S v| (one stream
 *     synchronisation per sweep) the correction is applied, and the sweeps stop once the
 *     residual expected of the corrected iterate, rho_k * max(f, min(1, rho_k / rho_{k-1}))
 *     with rho_{-1} = 1 and f = 0.1 (0.01 with DFISHER_CENTERED, whose projected factor leaves no
 *     stagnating direction), is <= opt->tol (1e-7 when opt->tol is 0); at most 16 sweeps, else
 *     DFISHER_E_NOT_CONVERGED with x written. info->resid is the last rho_k.
 *   dfisher_solve_uneven: measured on the device, per problem, inside the captured launch
 *     sequence (no host round trip): the same predictive test as dfisher_solve after each sweep,
 *     with at most the a-priori count of dfisher_auto_sweeps + 2 sweeps (16 at most); a problem
 *     that stops skips its later passes over S. DFISHER_E_NOT_CONVERGED (x written) if a problem
 *     reached its cap without meeting the test.
 *   dfisher_factor_create, dfisher_solve_batched (no host round trip per sweep): the a-priori
 *     count of dfisher_auto_sweeps for each shape, raised where the factorisation was shifted
 *     (the batched call uses the largest count of its lambdas). */
#define DFISHER_SWEEPS_AUTO (-1)

/* Defaults: FP32 Gram, 0 sweeps, shift on failure, FP32 output, no tolerance, no final residual,
 * no flags. */
#define DFISHER_OPTIONS_DEFAULT {DFISHER_GRAM_FP32, 0, DFISHER_SHIFT_ON_FAILURE, 0, 0.0, 0, 0}

typedef struct dfisher_info {
  int64_t potrf_info;    /* 0, or the 1-based index of the first pivot that is not > 0 in the
                            last factorisation attempt                                       */
  double shift;          /* tau added to W's diagonal by the successful factorisation (0: none) */
  int32_t attempts;      /* number of factorisations run                                      */
  int32_t sweeps_done;   /* refinement sweeps applied                                         */
  double resid;          /* with opt->tol > 0: rho of the last sweep (the relative residual of
                            the iterate that sweep corrected, measured before the correction;
                            the returned iterate's is smaller by about the contraction factor);
                            -1 when not measured (tol == 0 or no sweep)                         */
  double w_resid;        /* with opt->final_resid = 1: |S v - lambda y - S (S^T y)|_2 / |S v|_2 of the
                            returned y (FP64); -1 when not measured                             */
} dfisher_info;

typedef struct dfisher_ctx dfisher_ctx;        /* device id, workspace, pinned status buffer  */
typedef struct dfisher_factor dfisher_factor;  /* owns L (FP64 n x n); borrows S              */

/* Create a context on HIP device `device` (>= 0). Returns DFISHER_E_DEVICE if the device does
 * not exist. The context owns the workspace of every call made with it. */
DFISHER_API dfisher_status dfisher_ctx_create(int device, dfisher_ctx** out);
/* Release a context and its workspace (NULL is accepted). Waits for the device to be idle. */
DFISHER_API dfisher_status dfisher_ctx_destroy(dfisher_ctx* ctx);

/* Per-stage device timing of the last dfisher_solve / dfisher_factor_create / dfisher_gram call
 * made with this context: HIP events recorded on that call's stream around each stage (only
 * while enabled; recording adds no synchronisation). dfisher_ctx_last_timing waits for the
 * events and returns milliseconds; stages a call did not run read 0. */
typedef struct dfisher_timing {
  double rowpass_ms;      /* b = S v and squared row norms (one pass over S)   */
  double gram_ms;         /* matrix-core Gram kernel (split-K partial tiles)   */
  double gram_reduce_ms;  /* FP64 reduction of the partial tiles into W        */
  double potrf_ms;        /* Cholesky, including any shifted retries           */
  double trsv_ms;         /* first L^-1 / L^-T application                     */
  double refine_ms;       /* all refinement sweeps                              */
  double apply_ms;        /* x = (v - S^T y) / lambda (one pass over S)        */
  double total_ms;        /* first to last event                                */
} dfisher_timing;

DFISHER_API dfisher_status dfisher_ctx_enable_timing(dfisher_ctx* ctx, int32_t enable);
DFISHER_API dfisher_status dfisher_ctx_last_timing(dfisher_ctx* ctx, dfisher_timing* out);

/* Algorithm 1 step 1: W = S S^T + lambda I_n.
 * Writes the full symmetric n x n FP64 matrix W (row-major, both triangles). lambda >= 0 is
 * allowed here (lambda = 0 gives the Gram G = S S^T). Off-diagonal entries use `prec`; the
 * diagonal is the FP64 squared row norm plus lambda. */
DFISHER_API dfisher_status dfisher_gram(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds,
                            int32_t prec, double lambda, double* W, void* stream);

/* The scaled-FP8 form of S used by DFISHER_GRAM_MXFP8 (the precision preparation of the Gram's
 * inputs). Row i is cut into 32-column blocks; block b gets the scale 2^e with the smallest
 * integer e such that max_k |S_ik| <= 448 * 2^e over the block (e in [-127, 127], -127 for an
 * all-zero block), and each element becomes the E4M3 code (OCP FP8, 1-4-3, bias 7, max 448)
 * of S_ik / 2^e rounded to nearest even. Outputs (device): codes[i * ldq + k] for k < m
 * (ldq a multiple of 64, >= m; bytes k >= m of a row are unspecified) and
 * scales[i * (ldq / 32) + b] = e + 127 (E8M0). Needs 16-byte aligned rows (lds % 4 == 0 and
 * S 16-byte aligned), else DFISHER_E_UNSUPPORTED. */
DFISHER_API dfisher_status dfisher_quantize_mxfp8(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m,
                                                  int64_t lds, uint8_t* codes, int64_t ldq, uint8_t* scales,
                                                  void* stream);

/* Algorithm 1 step 2: in-place Cholesky W = L L^T of an n x n FP64 SPD matrix (row-major,
 * row stride n). Reads the lower triangle only; writes L to the lower triangle and zeros the
 * strict upper triangle. *info (host pointer) receives 0 or the 1-based index of the first
 * pivot d with !(d > 0) (NaN fails); the call then returns DFISHER_E_NOT_SPD and the
 * matrix contents are unspecified. Synchronises the stream. */
DFISHER_API dfisher_status dfisher_potrf(dfisher_ctx* ctx, double* W, int64_t n, int64_t* info, void* stream);

/* b = S v (FP32 inputs, FP64 accumulation, FP64 output of length n): the first product of the
 * right-to-left evaluation of S^T L^-T L^-1 S v (Section 2, after Algorithm 1). */
DFISHER_API dfisher_status dfisher_gemv(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds,
                            const float* v, double* b, void* stream);

/* Triangular solves with the Cholesky factor (row-major n x n FP64, lower triangle used), the
 * L^-1 and L^-T of the inlined product S^T L^-T L^-1 S v (Section 2, the remark after
 * Algorithm 1: triangular solves instead of forming Q = L^-1 S):
 * trans = 0: y = L^-1 b (forward substitution); trans = 1: y = L^-T b (back substitution).
 * b and y are FP64 device vectors of length n and may alias. */
DFISHER_API dfisher_status dfisher_trsv(dfisher_ctx* ctx, const double* L, int64_t n, int32_t trans,
                            const double* b, double* y, void* stream);

/* Final step of Algorithm 1 with Q inlined: x = (v - S^T y) / lambda, FP64 accumulation over the
 * n samples. y is FP64 (length n); x is FP32 (x_fp64 = 0) or FP64 (x_fp64 = 1), length m, and
 * may alias v when both are FP32. */
DFISHER_API dfisher_status dfisher_apply(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds,
                             const float* v, const double* y, double lambda, void* x, int32_t x_fp64,
                             void* stream);

/* Algorithm 1 end to end: x solving (S^T S + lambda I) x = v. v is FP32 (length m); x is FP32
 * or FP64 per opt->x_fp64 and may alias v when FP32. opt NULL = defaults; info may be NULL.
 * With opt->tol > 0 the sweeps stop at the tolerance (see dfisher_options) and the call returns
 * DFISHER_E_NOT_CONVERGED, with x and info written, if no measured residual met it. */
DFISHER_API dfisher_status dfisher_solve(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds,
                             const float* v, double lambda, void* x, const dfisher_options* opt,
                             void* stream, dfisher_info* info);

/* Structured right-hand side (Appendix B): when v = S^T f lies in the row space of S, the solution
 * of Eq. 1 is x = S^T (S S^T + lambda I)^-1 f (the push-through identity of Proposition 1). This
 * call takes f (FP64 device vector of length n) instead of v and runs Algorithm 1 with b = f: the
 * pass for S v and the subtraction v - S^T y are skipped, and x = S^T y is written (FP32 rounded
 * once, or FP64 per opt->x_fp64; length m). Refinement sweeps (opt->sweeps, DFISHER_SWEEPS_AUTO,
 * opt->tol, opt->final_resid) act on W y = f exactly as in dfisher_solve, with residuals relative
 * to |f|. Same errors and synchronisation as dfisher_solve; x must not overlap S or f. */
DFISHER_API dfisher_status dfisher_solve_rowspace(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m,
                                                  int64_t lds, const double* f, double lambda, void* x,
                                                  const dfisher_options* opt, void* stream, dfisher_info* info);

/* Stochastic reconfiguration front end (Section 3): the score matrix of SR is the centered, scaled
 * log-derivative matrix S = (O - mean O) / sqrt(n), the mean taken over the n samples (rows) for
 * every parameter (column): S_ij = fl32((O_ij - mu_j) / sqrt(n)), mu_j = (sum_i O_ij) / n with
 * FP64 sums and arithmetic and one rounding to FP32 (the column sums' order is the library's: S
 * matches a sequential-sum evaluation to within one FP32 unit in the last place).
 *   is_complex = 0: O is real, n x m FP32 (row stride ldo >= m); S is n x m FP32 (row stride
 *     lds >= m). S may be O itself (in place: same pointer and ldo == lds), else must not overlap.
 *   is_complex = 1: O is complex, n x m values stored as interleaved (real, imaginary) FP32 pairs,
 *     8-byte aligned, row stride ldo >= m complex values; the real and imaginary parts are centered
 *     separately and written as the stacked real matrix Z = [Re S; Im S] (2n x m FP32, row stride
 *     lds >= m; rows 0..n-1 real parts, n..2n-1 imaginary parts), which must not overlap O. Z is the
 *     score matrix of the real-part variant F = Re[S^H S] = Z^T Z (the concatenation of the real and
 *     imaginary parts in the sample dimension): solve it with dfisher_solve (n -> 2n) and the rest of
 *     the algorithm unchanged. It is also the input of dfisher_solve_complex.
 * Two passes over O (column sums, then the write). Does not synchronise. */
DFISHER_API dfisher_status dfisher_sr_center(dfisher_ctx* ctx, const float* O, int64_t n, int64_t m, int64_t ldo,
                                             int32_t is_complex, float* S, int64_t lds, void* stream);

/* Complex variant (Section 3): with a complex S every transpose of Eq. 1 and Algorithm 1 becomes a
 * Hermitian conjugate, (S^H S + lambda I) x = v with x, v complex of length m. S = A + iB is given
 * in the stacked real form Z = [A; B] (2n x m FP32, row stride lds; what dfisher_sr_center writes for
 * a complex O); v and x are interleaved (real, imaginary) pairs, 8-byte aligned: v FP32, x FP32 or
 * FP64 per opt->x_fp64. Solved as the real system of the 2n x 2m matrix [[A, -B], [B, A]], which
 * is never formed: its Gram [[Wr, -Wi], [Wi, Wr]] + lambda I (Wr = A A^T + B B^T, Wi = B A^T -
 * A B^T) is assembled from one Gram of Z (any opt->gram_prec; the scaled-FP8 Gram needs 16-byte
 * aligned rows), factored in FP64 (2n x 2n), and every product with the matrix or its transpose is
 * a pass over Z with two vectors. Options, refinement, errors and synchronisation as in
 * dfisher_solve (residuals relative to |S v|). n <= 32767. */
DFISHER_API dfisher_status dfisher_solve_complex(dfisher_ctx* ctx, const float* Z, int64_t n, int64_t m, int64_t lds,
                                                 const float* v, double lambda, void* x, const dfisher_options* opt,
                                                 void* stream, dfisher_info* info);

/* Factor reuse: steps 1-2 of Algorithm 1 once (Gram + Cholesky, with the shift policy), then
 * any number of right-hand sides. The factor BORROWS S: S must stay valid and unchanged until
 * dfisher_factor_destroy. The factor keeps a pointer to ctx, which must outlive it. */
DFISHER_API dfisher_status dfisher_factor_create(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds,
                                     double lambda, const dfisher_options* opt, void* stream,
                                     dfisher_factor** out, dfisher_info* info);
/* Solve for nrhs right-hand sides: V is nrhs x m FP32 (row r = v_r, row stride ldv >= m);
 * X is nrhs x m (row stride ldx >= m), FP32 or FP64 per the factor's options. */
DFISHER_API dfisher_status dfisher_factor_solve(dfisher_factor* f, const float* V, int64_t nrhs, int64_t ldv,
                                    void* X, int64_t ldx, void* stream, dfisher_info* info);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): dfisher_factor_solve for one right-hand side v (FP32,
 * length m) into x (FP32 or FP64 per the factor's options, length m; may alias v when FP32),
 * with the factor's sweep count. It calls no hipMalloc, hipFree or allocating routine and does not
 * synchronise: its scratch is a 64 MiB device array built into the library, one per device,
 * looked up when a context is created on that device and held until the process ends. Every call
 * on a device shares that array, so calls that overlap on one device (different streams or
 * threads) race; each call rewrites what it reads. A shape whose scratch would exceed 64 MiB, or
 * refinement (sweeps > 0) without the one-read product (n <= 4096, m >= 16, 16-byte aligned rows
 * of S), returns DFISHER_E_UNSUPPORTED before any device work. info may be NULL. */
DFISHER_API dfisher_status dfisher_factor_solve_noalloc(const dfisher_factor* f, const float* v, void* x,
                                                        void* stream, dfisher_info* info);
/* Copy the factor's L (n x n FP64 row-major, zero strict upper triangle) to device memory. */
DFISHER_API dfisher_status dfisher_factor_copy_L(const dfisher_factor* f, double* L, void* stream);
DFISHER_API dfisher_status dfisher_factor_destroy(dfisher_factor* f);

/* Many damping values and right-hand sides sharing one Gram: for every lambda_l (nlam values,
 * host array) and every row v_r of V (nrhs x m FP32, stride ldv), X[(l * nrhs + r) * ldx + k]
 * holds x_{l,r} solving (S^T S + lambda_l I) x = v_r. infos (host, may be NULL) has nlam
 * entries. Algorithm 1 for every pair, with step 1 shared: the Gram G = S S^T is formed once,
 * the nlam Cholesky factorisations of G + lambda_l I run in the same launches, and S V, the
 * refinement residuals and x = (v - S^T y) / lambda run as passes over S that serve 16 vectors
 * each. Needs nlam * nrhs <= 65535 (else DFISHER_E_UNSUPPORTED). A factorisation that fails
 * under DFISHER_SHIFT_NONE makes the call return DFISHER_E_NOT_SPD; the x of that lambda is then
 * unspecified. Synchronises the stream once to read the factorisation statuses, unless
 * opt->flags has DFISHER_ASYNC (then nothing waits, infos is a device array, and the call can be
 * captured into a HIP graph; see DFISHER_ASYNC). */
DFISHER_API dfisher_status dfisher_solve_batched(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds,
                                     const double* lambdas, int32_t nlam, const float* V, int32_t nrhs,
                                     int64_t ldv, void* X, int64_t ldx, const dfisher_options* opt,
                                     void* stream, dfisher_info* infos);

/* Independent problems of different sizes (for example per-layer Fisher blocks): problem p
 * solves (S_p^T S_p + lambda_p I) x_p = v_p with S_p n[p] x m[p] (stride lds[p]). All arrays
 * of length nprob are HOST arrays of device pointers / sizes. infos (host, may be NULL) has
 * nprob entries. Each problem follows Algorithm 1 as in dfisher_solve; the Cholesky
 * factorisations and the triangular solves of all problems share launches, nothing waits for the
 * host until the end, and the launch sequence is captured into a HIP graph and replayed on later
 * calls with the same arguments (dfisher_ctx_enable_graphs). nprob <= 65535. A problem whose
 * factorisation fails is then solved again on its own with the shift policy's escalation
 * (DFISHER_SHIFT_ON_FAILURE / _ALWAYS; under _NONE the call returns DFISHER_E_NOT_SPD and that x
 * is unspecified). Synchronises the stream once, plus once per problem solved again. */
DFISHER_API dfisher_status dfisher_solve_uneven(dfisher_ctx* ctx, int32_t nprob, const float* const* S, const int64_t* n,
                                    const int64_t* m, const int64_t* lds, const float* const* v,
                                    const double* lambda, void* const* x, const dfisher_options* opt,
                                    void* stream, dfisher_info* infos);

/* dfisher_solve_uneven captures its launch sequence into a HIP graph and replays it while the
 * arguments (pointers, sizes, lambdas, options) and the context's buffers stay the same; enable = 0
 * runs every call eagerly instead (and drops the cached graph). Default: enabled. */
DFISHER_API dfisher_status dfisher_ctx_enable_graphs(dfisher_ctx* ctx, int32_t enable);

/* Gram autotuning. The split-K factor of the Gram kernels (how many k-slices the m columns are
 * cut into, which sets the number of workgroups and the partial-tile traffic) and, for
 * split-BF16 on 16-byte aligned rows, whether the row pass pre-splits S into bf16 planes, are
 * chosen per size class (precision, ceil(n / 256), floor(log2 m), row alignment).
 * dfisher_autotune_gram times every candidate on the given S (Gram stage only: row pass, tile
 * kernel, reduction; one untimed and two timed runs each, HIP events on the stream, synchronous)
 * and stores the fastest in the context; later calls with that size class use it. With
 * dfisher_ctx_enable_autotune(ctx, 1), dfisher_gram / _solve / _factor_create / _solve_batched /
 * _solve_uneven tune every size class they have not seen before on first use. The table can be
 * saved to and loaded from a text file ("prec tiles log2m aligned q mode" per line); loading
 * merges into the context's table and rejects malformed files with DFISHER_E_INVALID_ARG. */
DFISHER_API dfisher_status dfisher_autotune_gram(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds,
                                     int32_t prec, void* stream);
DFISHER_API dfisher_status dfisher_ctx_enable_autotune(dfisher_ctx* ctx, int32_t enable);
DFISHER_API dfisher_status dfisher_ctx_save_tuning(const dfisher_ctx* ctx, const char* path);
DFISHER_API dfisher_status dfisher_ctx_load_tuning(dfisher_ctx* ctx, const char* path);

/* The refinement sweep count that DFISHER_SWEEPS_AUTO picks for one problem of n samples and m
 * parameters with the Gram in `prec` and no factored shift (a shift can only raise it; the
 * solves re-evaluate it once the factorisation's shift is known). One y-level sweep multiplies
 * the error of y = W^-1 S v by about c = |W~^-1 E| (E: error of the computed Gram, whose
 * diagonal is exact); the model c = C / (sqrt(m/n) (1 - sqrt(n/m))^2) with C = 0.1 (scaled FP8),
 * 1e-4 (split-BF16), 1e-5 (FP32) bounds the contraction of a Gram of rows with many independent
 * entries, and the count is the smallest k with c^(k+1) <= 1e-7; for the scaled-FP8 Gram it is
 * then raised by 3 below m/n = 150 and by 2 below m/n = 600 (directions where the Gram's error
 * exceeds W's eigenvalue, such as the all-ones direction of a column-centered S, converge only
 * after the bulk); the solves leave that raise out when opt->flags has DFISHER_CENTERED, which
 * makes that direction exact; at most 16. It is a heuristic: for a measured residual use opt->tol
 * with dfisher_solve. Returns -1 for an unknown prec or n, m < 1. */
DFISHER_API int32_t dfisher_auto_sweeps(int32_t prec, int64_t n, int64_t m);

/* Static text for a status code. */
DFISHER_API const char* dfisher_status_string(dfisher_status s);
/* Message describing the last failure on the calling thread ("" if none). */
DFISHER_API const char* dfisher_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DFISHER_H */
