// C ABI of the dfisher library: argument checks, workspace, and the order of device work for
// Algorithm 1 (Section 2) with the Q-inlined right-to-left apply, the Cholesky shift policy and
// FP64 iterative refinement on W y = S v. All arithmetic runs in the HIP kernels of this
// directory; this file only validates, plans, allocates and launches.
#include "dfisher.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <vector>
#include <map>
#include <tuple>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "dfisher_internal.h"

// Scratch of dfisher_factor_solve_noalloc: one copy per device, held until the process ends. In
// host code `scratch` only names the symbol; the device address comes from hipGetSymbolAddress
// (once per device, in init_kernels) and is the only form passed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

dfisher_status fail(dfisher_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(DFISHER_E_DEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),     \
                  __FILE__, __LINE__);                                                         \
  } while (0)

#define DF_TRY(expr)                   \
  do {                                 \
    dfisher_status s_ = (expr);        \
    if (s_ != DFISHER_OK) return s_;   \
  } while (0)

constexpr int MAX_SWEEPS = 16;
constexpr double AUTO_TOL = 1e-7;   // the residual DFISHER_SWEEPS_AUTO aims for in dfisher_solve
constexpr double AUTO_MIN_CONTRACTION = 0.1;   // least contraction a predictive stop assumes
// ... when S is declared centered: the projected factor has no stagnating direction left, and one
// sweep contracts the residual by 1e-3 .. 1e-2 (measured at m/n 100 .. 1000)
constexpr double AUTO_MIN_CONTRACTION_CENTERED = 0.01;
constexpr int MAX_SHIFT_ATTEMPTS = 10;
// The final step takes the last correction's image through the FP8 codes only while its expected
// error, about 3 % of the estimate sqrt(sum_i |s_i|^2 z_i^2) / |S^T y| the device forms, stays near
// 1e-7 of |S^T y| (ten times below the 1e-6 target; for the scaled-FP8 Gram after two sweeps at
// m/n ~ 1000 the estimate is ~2e-6)
constexpr double FINAL8_EST_MAX = 4e-6;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

constexpr int NEV = 8;  // stage boundaries: rowpass | gram | reduce | potrf | trsv | refine | apply |

struct dfisher_ctx {
  int device = 0;
  bool timing = false;
  bool ev_used[NEV] = {};
  hipEvent_t ev[NEV] = {};
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_frozen = false;       // a call captured into a caller's graph holds ws: never reallocated
  int64_t* h_status = nullptr;  // pinned: [0] potrf info
  double* h_scalar = nullptr;   // pinned: [0] diagonal max
  int64_t* d_info = nullptr;
  int32_t* d_flag = nullptr;
  double* d_scalar = nullptr;
  // uneven batches: job tables (own buffer, never carved from ws) and the captured graph of the
  // last call, replayed when the next call has the same arguments and buffers
  bool graphs = true;
  void* tbuf = nullptr;
  size_t tbuf_bytes = 0;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t uneven_exec = nullptr;
  std::vector<uint64_t> uneven_key;
  // Gram autotuning: (precision, tiles per edge, floor(log2 m), aligned rows) -> (q, split mode)
  bool autotune = false;
  std::map<std::tuple<int, int64_t, int, int>, std::pair<int, int>> tune;
};

struct dfisher_factor {
  dfisher_ctx* ctx = nullptr;
  const float* S = nullptr;
  int64_t n = 0, m = 0, lds = 0;
  double lambda = 0.0;
  dfisher_options opt{};
  double* L = nullptr;     // owned: n x n
  double* Dinv = nullptr;  // owned: inverses of the 64 x 64 diagonal blocks of L
  double shift = 0.0;
};

namespace {

// Records stage-boundary events on the call's stream when timing is enabled.
struct StageClock {
  dfisher_ctx* ctx;
  hipStream_t st;
  StageClock(dfisher_ctx* c, hipStream_t s) : ctx(c), st(s) {
    for (int i = 0; i < NEV; ++i) ctx->ev_used[i] = false;
  }
  void mark(int i) {
    if (ctx->timing && hipEventRecord(ctx->ev[i], st) == hipSuccess) ctx->ev_used[i] = true;
  }
};

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

void drop_graph(dfisher_ctx* ctx);

dfisher_status ensure_ws(dfisher_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return DFISHER_OK;
  if (ctx->ws_frozen)
    return fail(DFISHER_E_UNSUPPORTED,
                "the context's workspace (%zu bytes) is held by a captured call and cannot grow to %zu bytes; "
                "use another context", ctx->ws_bytes, bytes);
  drop_graph(ctx);   // a cached graph points into the old workspace
  if (ctx->ws) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  hipError_t e = hipMalloc(&ctx->ws, bytes);
  if (e != hipSuccess) {
    ctx->ws = nullptr;
    (void)hipGetLastError();
    return fail(DFISHER_E_NO_MEMORY, "workspace allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
  }
  ctx->ws_bytes = bytes;
  return DFISHER_OK;
}

// Carves aligned sub-buffers out of one workspace block.
struct Carver {
  size_t off = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += align_up(count * sizeof(T));
    return p;
  }
};

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Byte ranges [a, a + abytes) and [b, b + bbytes) intersect.
bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + bbytes && pb < pa + abytes;
}

dfisher_status check_ctx(dfisher_ctx* ctx) {
  if (!ctx) return fail(DFISHER_E_INVALID_ARG, "ctx is NULL");
  return DFISHER_OK;
}

dfisher_status check_S(const float* S, int64_t n, int64_t m, int64_t lds) {
  if (!S) return fail(DFISHER_E_INVALID_ARG, "S is NULL");
  if (n < 1) return fail(DFISHER_E_INVALID_ARG, "n = %lld < 1", (long long)n);
  if (m < 1) return fail(DFISHER_E_INVALID_ARG, "m = %lld < 1", (long long)m);
  if (lds < m) return fail(DFISHER_E_INVALID_ARG, "lds = %lld < m = %lld", (long long)lds, (long long)m);
  return DFISHER_OK;
}

// async_ok: the entry point honours DFISHER_ASYNC (others return DFISHER_E_UNSUPPORTED for it).
dfisher_status check_opt(const dfisher_options* opt, dfisher_options* out, bool async_ok = false) {
  dfisher_options d = DFISHER_OPTIONS_DEFAULT;
  if (opt) d = *opt;
  if (d.gram_prec != DFISHER_GRAM_FP32 && d.gram_prec != DFISHER_GRAM_BF16X3 && d.gram_prec != DFISHER_GRAM_MXFP8)
    return fail(DFISHER_E_INVALID_ARG, "unknown gram_prec %d", d.gram_prec);
  if ((d.sweeps < 0 && d.sweeps != DFISHER_SWEEPS_AUTO) || d.sweeps > MAX_SWEEPS)
    return fail(DFISHER_E_INVALID_ARG, "sweeps = %d outside 0..%d (or DFISHER_SWEEPS_AUTO)", d.sweeps, MAX_SWEEPS);
  if (d.shift_policy != DFISHER_SHIFT_NONE && d.shift_policy != DFISHER_SHIFT_ON_FAILURE &&
      d.shift_policy != DFISHER_SHIFT_ALWAYS)
    return fail(DFISHER_E_INVALID_ARG, "unknown shift_policy %d", d.shift_policy);
  if (d.x_fp64 != 0 && d.x_fp64 != 1) return fail(DFISHER_E_INVALID_ARG, "x_fp64 must be 0 or 1");
  if (!std::isfinite(d.tol) || d.tol < 0.0) return fail(DFISHER_E_INVALID_ARG, "tol must be finite and >= 0");
  if (d.final_resid != 0 && d.final_resid != 1) return fail(DFISHER_E_INVALID_ARG, "final_resid must be 0 or 1");
  if ((d.flags & ~(DFISHER_CENTERED | DFISHER_ASYNC | DFISHER_EXACT_APPLY)) != 0)
    return fail(DFISHER_E_INVALID_ARG, "unknown flags 0x%x", d.flags);
  if ((d.flags & DFISHER_ASYNC) != 0 && !async_ok)
    return fail(DFISHER_E_UNSUPPORTED, "DFISHER_ASYNC is honoured by dfisher_solve_batched only");
  *out = d;
  return DFISHER_OK;
}

// Entry points that do not measure the final residual reject the request.
dfisher_status check_no_final(const dfisher_options& o) {
  if (o.final_resid != 0)
    return fail(DFISHER_E_UNSUPPORTED, "final_resid is honoured by dfisher_solve and dfisher_solve_uneven only");
  return DFISHER_OK;
}

// Sweep count of DFISHER_SWEEPS_AUTO. One y-level sweep multiplies the error of y by about
// c = |W~^-1 E|, E the error of the computed Gram (its diagonal is exact). For rows of m
// roughly independent entries, |E| ~ C_prec |s|^2 / sqrt(m/n) (C_prec ~ 2 sqrt(2) times the
// relative rounding error of one product: E4M3 about 3e-2, the split-BF16 dropped term
// 2^-16, FP32 accumulation within a slice) and the smallest bulk eigenvalue of S S^T is
// about |s|^2 (1 - sqrt(n/m))^2, so c ~ C_prec / (sqrt(m/n) (1 - sqrt(n/m))^2). A factored
// shift tau adds tau / (|s|^2 (1 - sqrt(n/m))^2) (tau_rel = tau / max_i W_ii). The count is the
// smallest k with c^(k+1) <= 1e-7, ten times below the 1e-6 error target. The scaled-FP8 Gram's
// error can also exceed W's eigenvalue along a few directions (for a column-centered S, the
// all-ones one, eigenvalue ~ lambda); the conjugate-gradient sweeps remove such directions only
// after the bulk, which took two or three more sweeps in measurements at m/n = 78 .. 256 (none at
// m/n ~ 1000), so the count gets 3 more below m/n = 150 and 2 more below m/n = 600, unless the
// caller declared S centered (DFISHER_CENTERED), which makes that direction exact in the factored
// matrix. Capped at 16.
int auto_sweeps(int prec, int64_t n, int64_t m, double tau_rel, bool centered = false) {
  const double a = (double)m / (double)n;
  const double C = prec == DFISHER_GRAM_MXFP8 ? 0.1 : (prec == DFISHER_GRAM_BF16X3 ? 1e-4 : 1e-5);
  const double gap = a > 4.0 ? (1.0 - 1.0 / std::sqrt(a)) * (1.0 - 1.0 / std::sqrt(a)) : 0.25;
  double c = C / (std::sqrt(std::max(a, 1.0)) * gap);
  if (tau_rel > 0.0) c = std::max(c, tau_rel / gap);
  if (!(c < 0.5)) return MAX_SWEEPS;
  int k = 0;
  double e = c;
  while (e > 1e-7 && k < MAX_SWEEPS) {
    e *= c;
    ++k;
  }
  if (prec == DFISHER_GRAM_MXFP8 && !centered) k += a < 150.0 ? 3 : (a < 600.0 ? 2 : 0);
  return std::min(k, MAX_SWEEPS);
}

bool is_centered(const dfisher_options& o) { return (o.flags & DFISHER_CENTERED) != 0; }
double auto_floor(const dfisher_options& o) {
  return is_centered(o) ? AUTO_MIN_CONTRACTION_CENTERED : AUTO_MIN_CONTRACTION;
}

// Entry points that run a fixed number of sweeps reject a tolerance.
dfisher_status check_no_tol(const dfisher_options& o) {
  if (o.tol != 0.0) return fail(DFISHER_E_UNSUPPORTED, "tol is honoured by dfisher_solve only");
  return DFISHER_OK;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

bool rows_aligned16(const float* S, int64_t lds) {
  return (lds % 4) == 0 && (reinterpret_cast<uintptr_t>(S) & 15) == 0;
}

dfisher_status check_prec_layout(int prec, const float* S, int64_t lds) {
  if (prec == DFISHER_GRAM_MXFP8 && !rows_aligned16(S, lds))
    return fail(DFISHER_E_UNSUPPORTED, "the scaled-FP8 Gram needs 16-byte aligned rows (lds %% 4 == 0)");
  return DFISHER_OK;
}

// Rounding unit of the computed Gram's entries, relative to max_i W_ii, used by the up-front shift.
double gram_unit(int prec, int64_t m) {
  // FP8: E4M3 keeps 3 mantissa bits; the relative error of a sum of m products of block-scaled
  // values shrinks like 1/sqrt(m) (random rounding errors), here with constant 2^-4.
  if (prec == DFISHER_GRAM_MXFP8) return 0.0625 / std::sqrt((double)m);
  return std::ldexp(1.0, -24);
}

std::tuple<int, int64_t, int, int> tune_key(int prec, int64_t n, int64_t m, bool aligned) {
  int lg = 0;
  while (lg < 62 && ((int64_t)1 << (lg + 1)) <= m) ++lg;
  return std::make_tuple(prec, (n + dfi::GRAM_TILE - 1) / dfi::GRAM_TILE, lg, aligned ? 1 : 0);
}

// The Gram plan for a shape: the tuned split-K factor / split mode of its size class if the
// context has one, else the built-in choice.
dfi::GramPlan make_gram_plan(const dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds, int prec) {
  const bool al = rows_aligned16(S, lds);
  auto it = ctx->tune.find(tune_key(prec, n, m, al));
  if (it != ctx->tune.end()) return dfi::gram_plan(n, m, lds, prec, al, it->second.first, it->second.second);
  return dfi::gram_plan(n, m, lds, prec, al);
}

// Everything one factorisation + solve needs, carved from the workspace.
struct SolveBufs {
  double* W;       // n x n, unshifted W (lower triangle)
  double* L;       // n x n factor (unless the caller supplies one)
  float* gpart;    // Gram partial tiles
  double* rpart;   // row-pass partials
  double* cpart;   // column-pass partials
  double* b;       // S v
  double* d;       // squared row norms
  double* z;       // work
  double* y;       // W^-1 S v
  double* r;       // refinement residual
  double* zc;      // M^-1 r (refinement correction)
  double* p;       // refinement search direction
  double* nq;      // -(W p)
  double* zero;    // n zeros (right-hand side of the W p pass)
  double* t;       // S^T y (m, FP64)
  double* Dinv;    // inverses of L's 64 x 64 diagonal blocks
  double* dkk;     // Cholesky scratch: current diagonal block inverse
  double* tw;      // triangular-solve work vector (n)
  uint8_t* q8;     // scaled-FP8 codes of S (n x ldq), when the Gram is MXFP8
  uint8_t* sc8;    // their E8M0 scales (n x ldq/32)
  int64_t ldq;
  uint16_t* hi;    // split-BF16 planes of S (n x gp->ldh each), when the Gram uses them
  uint16_t* lo;
  // the final step through the FP8 codes (apply8.hip), when planned: S^T y carried through the
  // passes, S^T p of the last direction, S^T 1 (centered S only), the correction in FP32, scalars
  double* T8;
  double* U8;
  double* cs8;
  float* zf8;
  double* a8;      // [0] the last step length, [1] the correction's all-ones mean
  int* use8;       // 1: the final step went through the codes
  size_t bytes;
};

SolveBufs carve(char* base, int64_t n, int64_t m, const dfi::GramPlan* gp, const dfi::RowPassPlan& rp,
                const dfi::ColPassPlan& cp, bool need_L, bool need_t, const dfi::RefinePassPlan* fp = nullptr,
                bool final8 = false, bool final8_cs = false) {
  Carver c;
  c.base = base;
  SolveBufs s{};
  s.W = gp ? c.take<double>((size_t)(n * n)) : nullptr;
  s.L = need_L ? c.take<double>((size_t)(n * n)) : nullptr;
  s.gpart = gp ? c.take<float>(gp->part_bytes / sizeof(float)) : nullptr;
  s.rpart = c.take<double>(std::max(rp.part_bytes, fp ? fp->part_bytes : 0) / sizeof(double) + 1);
  s.cpart = c.take<double>(cp.part_bytes / sizeof(double) + 1);
  s.b = c.take<double>((size_t)n);
  s.d = c.take<double>((size_t)n);
  s.z = c.take<double>((size_t)n);
  s.y = c.take<double>((size_t)n);
  s.r = c.take<double>((size_t)n);
  s.zc = c.take<double>((size_t)n);
  s.p = c.take<double>((size_t)n);
  s.nq = c.take<double>((size_t)n);
  s.zero = c.take<double>((size_t)n);
  s.t = need_t ? c.take<double>((size_t)m) : nullptr;
  s.Dinv = c.take<double>(dfi::trsv_dinv_bytes(n) / sizeof(double));
  s.dkk = c.take<double>(dfi::POTRF_DKK_BYTES / sizeof(double));
  s.tw = c.take<double>((size_t)n);
  s.ldq = dfi::fp8_ldq(m);
  const bool fp8 = gp && gp->prec == DFISHER_GRAM_MXFP8;
  s.q8 = fp8 ? c.take<uint8_t>((size_t)(n * s.ldq)) : nullptr;
  s.sc8 = fp8 ? c.take<uint8_t>((size_t)(n * (s.ldq / 32))) : nullptr;
  const bool split = gp && gp->prec == DFISHER_GRAM_BF16X3 && gp->ldh > 0;
  s.hi = split ? c.take<uint16_t>((size_t)(n * gp->ldh)) : nullptr;
  s.lo = split ? c.take<uint16_t>((size_t)(n * gp->ldh)) : nullptr;
  s.T8 = final8 ? c.take<double>((size_t)m) : nullptr;
  s.U8 = final8 ? c.take<double>((size_t)m) : nullptr;
  s.cs8 = final8 && final8_cs ? c.take<double>((size_t)m) : nullptr;
  s.zf8 = final8 ? c.take<float>((size_t)n) : nullptr;
  s.a8 = final8 ? c.take<double>(2) : nullptr;
  s.use8 = final8 ? c.take<int>(2) : nullptr;   // [1]: the centered projection was applied
  s.bytes = c.off;
  return s;
}

// Cholesky of W (+ tau I) into L following the shift policy. Synchronises once per attempt.
// `spec`, if given, is enqueued right after the first attempt's factorisation and before the wait
// for its status (work that depends on L, started speculatively so that the host enqueues it while
// the device is still busy); *spec_ok tells whether that work saw the final factor.
dfisher_status factor_with_policy(dfisher_ctx* ctx, const double* W, double* L, double* dkk, int64_t n, int policy,
                                  double unit, hipStream_t st, double* shift_out, int64_t* info_out,
                                  int32_t* attempts_out, const std::function<dfisher_status()>& spec = {},
                                  bool* spec_ok = nullptr) {
  // base shift: about sqrt(n) times the rounding unit of a computed Gram entry
  const double base_scale = std::sqrt((double)n) * unit;
  double scale = 0.0;  // tau = scale * max_i W_ii, evaluated on the device
  if (policy == DFISHER_SHIFT_ALWAYS) scale = 2.0 * base_scale;
  int attempts = 0;
  int64_t info = 0;
  if (policy != DFISHER_SHIFT_NONE) HIP_TRY(dfi::diag_max(W, n, ctx->d_scalar, st));
  for (;;) {
    HIP_TRY(dfi::shift_copy(W, L, n, scale, ctx->d_scalar, st));
    HIP_TRY(dfi::potrf_launch(L, n, ctx->d_info, ctx->d_flag, dkk, st));
    if (attempts == 0 && spec) DF_TRY(spec());
    HIP_TRY(hipMemcpyAsync(ctx->h_status, ctx->d_info, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    if (policy != DFISHER_SHIFT_NONE)
      HIP_TRY(hipMemcpyAsync(ctx->h_scalar, ctx->d_scalar, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    ++attempts;
    info = ctx->h_status[0];
    if (info == 0 || policy == DFISHER_SHIFT_NONE || attempts >= MAX_SHIFT_ATTEMPTS) break;
    if (!std::isfinite(ctx->h_scalar[0])) break;  // NaN/Inf in W: shifting cannot help
    scale = (scale == 0.0) ? base_scale : 8.0 * scale;
  }
  HIP_TRY(dfi::zero_upper(L, n, st));
  if (spec_ok) *spec_ok = attempts == 1 && info == 0;
  *shift_out = (info == 0 && policy != DFISHER_SHIFT_NONE) ? scale * ctx->h_scalar[0] : 0.0;
  *info_out = info;
  *attempts_out = attempts;
  if (info != 0)
    return fail(DFISHER_E_NOT_SPD, "Cholesky failed at pivot %lld after %d attempt(s)", (long long)info, attempts);
  return DFISHER_OK;
}

// Row pass (b = S v when v != nullptr, the exact row norms, and for the scaled-FP8 Gram its codes),
// then the Gram of `prec` reduced into W (lower triangle; upper too if mirror) with lambda added.
// center: W becomes the centered preconditioner P W P + lambda 1 1^T / n (work: B.gpart, B.zc), unless
// W itself shows that S is far from centered.
dfisher_status gram_stage(const float* S, const float* v, const dfi::GramPlan& gp, const dfi::RowPassPlan& rp,
                          const SolveBufs& B, double lambda, double* W, int mirror, hipStream_t st, StageClock* clk,
                          bool center = false, int* applied = nullptr) {
  if (clk) clk->mark(0);
  if (gp.prec == DFISHER_GRAM_MXFP8) {
    HIP_TRY(dfi::rowpass_launch(rp, S, v, nullptr, v != nullptr, true, B.rpart, st, B.q8, B.sc8, B.ldq, true));
  } else if (B.hi) {
    HIP_TRY(dfi::rowpass_launch_split(rp, S, v, B.rpart, B.hi, B.lo, gp.ldh, st));
  } else {
    HIP_TRY(dfi::rowpass_launch(rp, S, v, nullptr, v != nullptr, true, B.rpart, st));
  }
  HIP_TRY(dfi::rowpass_reduce(rp, B.rpart, v != nullptr, true, B.b, B.d, nullptr, nullptr, 0.0, st));
  if (clk) clk->mark(1);
  if (gp.prec == DFISHER_GRAM_MXFP8) {
    HIP_TRY(dfi::gram_launch_fp8(gp, B.q8, B.sc8, B.ldq, B.gpart, st));
  } else if (B.hi) {
    HIP_TRY(dfi::gram_launch_split(gp, B.hi, B.lo, B.gpart, st));
  } else {
    HIP_TRY(dfi::gram_launch(gp, S, B.gpart, st));
  }
  if (clk) clk->mark(2);
  HIP_TRY(dfi::gram_reduce(gp, S, B.gpart, B.d, lambda, W, mirror, st));
  if (center) {   // the Gram partials are free again: they hold the projection's tile sums
    if (gp.part_bytes < dfi::gram_project_work_bytes(gp.n)) return fail(DFISHER_E_DEVICE, "projection work too small");
    HIP_TRY(dfi::gram_project(W, gp.n, 1, lambda, mirror, reinterpret_cast<double*>(B.gpart), B.zc, st, applied));
  }
  return DFISHER_OK;
}

// out = rhs - lambda u - S (S^T u) for an n-vector u (FP64 accumulation): one read of S through the
// fused pass when `fp` allows it, else a column pass (t = S^T u into B.t) and a row pass. With
// rhs = b and u = y it is the residual of y; with rhs = 0 and u = p it is -(W p).
// tout / csout (the whole-line pass only, may be null): S^T u and S^T 1 from the same read of S.
dfisher_status w_pass(const float* S, int64_t n, int64_t m, int64_t lds, double lambda, const double* u,
                      const double* rhs, double* out, const SolveBufs& B, const dfi::RowPassPlan& rp,
                      const dfi::ColPassPlan& cp, const dfi::RefinePassPlan* fp, hipStream_t st,
                      double* tout = nullptr, double* csout = nullptr) {
  if (fp && fp->usable) {
    HIP_TRY(dfi::refine_pass_launch(*fp, S, n, m, lds, u, B.rpart, st, nullptr, -1, tout, csout));
    HIP_TRY(dfi::refine_pass_reduce(*fp, B.rpart, out, rhs, u, lambda, st));
  } else {
    if (tout || csout) return fail(DFISHER_E_DEVICE, "S^T u requested from a pass that does not form it");
    HIP_TRY(dfi::colpass_launch(cp, S, n, m, lds, u, nullptr, 1.0, B.t, 2, B.cpart, st));
    HIP_TRY(dfi::rowpass_launch(rp, S, nullptr, B.t, true, false, B.rpart, st));
    HIP_TRY(dfi::rowpass_reduce(rp, B.rpart, true, false, out, nullptr, rhs, u, lambda, st));
  }
  return DFISHER_OK;
}

// y = W^-1 b through the factor, then `sweeps` refinement sweeps against the exact operator
// W = S S^T + lambda I. A sweep is one read of S. Sweep 1 forms the residual r = b - W y; the
// sweeps after it are conjugate-gradient iterations preconditioned by M = L L^T (the factor of the
// computed, possibly shifted, Gram): q = W p from one pass, alpha = r.z / p.q, y += alpha p,
// r -= alpha q, z = M^-1 r, p = z + beta p. After the last sweep the correction z = M^-1 r of the
// final residual is added (y += z: with one sweep this is the classic correction
// y += L^-T L^-1 (b - W y)). Unlike the plain correction repeated, the iteration does not stall
// on directions where the computed Gram is far from W relative to W's eigenvalue there (for a
// column-centered S, the all-ones direction has eigenvalue ~ lambda while the Gram's rounding
// error along it can be much larger). With tol > 0 (ctx given): after each sweep read
// rho = |r| / |b| (one synchronisation; from sweep 2 on r is the iteration's recurrence), apply
// the correction and stop once rho <= tol. *done and *resid report the sweeps run and the last
// rho (-1 if none was measured).
// With predict > 0 the stop test is on the residual the corrected iterate is expected to have:
// rho_k times the contraction measured over the last sweep, rho_k / rho_{k-1} (rho_{-1} = 1, the
// residual of y = 0), but never less than predict times rho_k (AUTO_MIN_CONTRACTION, or
// AUTO_MIN_CONTRACTION_CENTERED for a declared centered S), so that the call stops only once a
// measured residual is <= tol / predict: the measured contraction of one sweep can hide a slower
// direction (the all-ones one above, unless the factor was projected).
// The sweeps of solve_y for any operator: wop(u, rhs, out, tout, csout) enqueues out = rhs - W u
// (length n) and, where tout / csout are given, S^T u and S^T 1 from the same pass.
using WOp = std::function<dfisher_status(const double* u, const double* rhs, double* out, double* tout,
                                         double* csout)>;

// The exact part of the final step's S^T y (apply8.hip), carried through the passes: T = S^T y of
// the iterate (the residual pass writes S^T y_0; each conjugate-gradient pass writes S^T p into U,
// added as T += alpha U), and S^T 1 when the all-ones component is split off. The last correction
// is then left in B.zc for the final step, not added to y.
struct Final8 {
  double* T;
  double* U;
  double* cs;      // may be null
  double* alpha;   // device: the last step length
  int64_t m;
};

dfisher_status solve_y_op(int64_t n, const double* L, const double* Dinv, const SolveBufs& B, int sweeps,
                          hipStream_t st, const WOp& wop, StageClock* clk = nullptr, dfisher_ctx* ctx = nullptr,
                          double tol = 0.0, int* done = nullptr, double* resid = nullptr, bool initial = true,
                          double predict = 0.0, bool* met = nullptr, const Final8* f8 = nullptr) {
  if (initial) {   // (else the caller has formed y = L^-T L^-1 b already)
    HIP_TRY(dfi::trsv_launch(L, Dinv, n, 0, B.b, B.z, B.tw, st));
    HIP_TRY(dfi::trsv_launch(L, Dinv, n, 1, B.z, B.y, B.tw, st));
    if (clk) clk->mark(5);
  }
  const bool measure = ctx && tol > 0.0;
  if (done) *done = 0;
  if (resid) *resid = -1.0;
  if (met) *met = false;
  if (sweeps > 0) {
    if (!ctx) return fail(DFISHER_E_DEVICE, "refinement needs the context's scalars");
    double* rz = ctx->d_scalar + 4;
    double* rr = ctx->d_scalar + 3;
    if (measure) HIP_TRY(dfi::sumsq(B.b, n, ctx->d_scalar + 2, st));
    HIP_TRY(dfi::fill_zero(B.zero, n, st));
    DF_TRY(wop(B.y, B.b, B.r, f8 ? f8->T : nullptr, f8 ? f8->cs : nullptr));   // sweep 1: r = b - W y
    if (measure) HIP_TRY(dfi::sumsq(B.r, n, rr, st));
    double prev = 1.0;
    for (int s = 1;; ++s) {
      double rho = -1.0;
      if (measure) {
        HIP_TRY(hipMemcpyAsync(ctx->h_scalar + 2, ctx->d_scalar + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const double bb = ctx->h_scalar[2], rrh = ctx->h_scalar[3];
        rho = bb > 0.0 ? std::sqrt(rrh / bb) : (rrh > 0.0 ? INFINITY : 0.0);
        if (resid) *resid = rho;
      }
      HIP_TRY(dfi::trsv_launch(L, Dinv, n, 0, B.r, B.z, B.tw, st));
      HIP_TRY(dfi::trsv_launch(L, Dinv, n, 1, B.z, B.zc, B.tw, st));
      bool stop = s >= sweeps;
      if (measure) {
        const double expect =
            predict > 0.0 ? rho * std::max(predict, std::min(1.0, prev > 0.0 ? rho / prev : 0.0)) : rho;
        prev = rho;
        if (expect <= tol) {
          if (met) *met = true;
          stop = true;
        }
      }
      if (stop) {
        if (!f8) HIP_TRY(dfi::pcg_finish(nullptr, n, 0, 1, B.zc, B.y, st));   // else the final step takes zc
        if (done) *done = s;
        break;
      }
      if (s == 1) HIP_TRY(dfi::pcg_init(nullptr, n, 0, 1, B.r, B.zc, B.p, rz, st));
      else HIP_TRY(dfi::pcg_dir(nullptr, n, 0, 1, B.r, B.zc, B.p, rz, st));
      DF_TRY(wop(B.p, B.zero, B.nq, f8 ? f8->U : nullptr, nullptr));   // -(W p)
      HIP_TRY(dfi::pcg_step(nullptr, n, 0, 1, B.p, B.nq, B.y, B.r, rz, measure ? rr : nullptr, st, nullptr,
                            f8 ? f8->alpha : nullptr));
      if (f8) HIP_TRY(dfi::t_axpy(f8->T, f8->U, f8->alpha, f8->m, st));
    }
  }
  if (clk) clk->mark(6);
  return DFISHER_OK;
}

dfisher_status solve_y(const float* S, int64_t n, int64_t m, int64_t lds, double lambda, const double* L,
                       const double* Dinv, const SolveBufs& B, const dfi::RowPassPlan& rp, const dfi::ColPassPlan& cp,
                       int sweeps, hipStream_t st, StageClock* clk = nullptr, const dfi::RefinePassPlan* fp = nullptr,
                       dfisher_ctx* ctx = nullptr, double tol = 0.0, int* done = nullptr, double* resid = nullptr,
                       bool initial = true, double predict = 0.0, bool* met = nullptr, const Final8* f8 = nullptr) {
  const WOp wop = [&](const double* u, const double* rhs, double* out, double* tout, double* csout) {
    return w_pass(S, n, m, lds, lambda, u, rhs, out, B, rp, cp, fp, st, tout, csout);
  };
  return solve_y_op(n, L, Dinv, B, sweeps, st, wop, clk, ctx, tol, done, resid, initial, predict, met, f8);
}

// r = b - lambda y - S (S^T y) for the current y (FP64), then w = |r| / |b| read back to the host
// (one synchronisation). The residual is not applied.
dfisher_status final_residual(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds, double lambda,
                              const SolveBufs& B, const dfi::RowPassPlan& rp, const dfi::ColPassPlan& cp,
                              const dfi::RefinePassPlan& fp, hipStream_t st, double* w) {
  if (fp.usable) {
    HIP_TRY(dfi::refine_pass_launch(fp, S, n, m, lds, B.y, B.rpart, st));
    HIP_TRY(dfi::refine_pass_reduce(fp, B.rpart, B.r, B.b, B.y, lambda, st));
  } else {
    HIP_TRY(dfi::colpass_launch(cp, S, n, m, lds, B.y, nullptr, 1.0, B.t, 2, B.cpart, st));
    HIP_TRY(dfi::rowpass_launch(rp, S, nullptr, B.t, true, false, B.rpart, st));
    HIP_TRY(dfi::rowpass_reduce(rp, B.rpart, true, false, B.r, nullptr, B.b, B.y, lambda, st));
  }
  HIP_TRY(dfi::sumsq(B.b, n, ctx->d_scalar + 2, st));
  HIP_TRY(dfi::sumsq(B.r, n, ctx->d_scalar + 3, st));
  HIP_TRY(hipMemcpyAsync(ctx->h_scalar + 2, ctx->d_scalar + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const double bb = ctx->h_scalar[2], rr = ctx->h_scalar[3];
  *w = bb > 0.0 ? std::sqrt(rr / bb) : (rr > 0.0 ? INFINITY : 0.0);
  return DFISHER_OK;
}

// Many right-hand sides against nfac factors in shared launches (multi-vector passes over S, batched
// triangular solves). Vector j = f * nrhs + r pairs factor f (L + f n^2, its block inverses at
// Dinv + f trsv_dinv_bytes(n) / 8, damping lams[f]) with v_r = V + r ldv; x_j goes to X + j ldx.
// Per vector: y = W_f^-1 S v_r, `sweeps` FP64 refinement sweeps against the exact operator, then
// x = (v_r - S^T y) / lambda_f. Needs nfac * nrhs <= 65535.
struct MultiBufs {
  double *Bs, *Bexp, *Y, *R, *D, *W1, *T, *T1, *Yi, *part, *part1;   // T1, part1: a second group
  double *Zc, *P, *NQ, *zero, *rz;   // refinement: M^-1 R, directions, -(W P), n zeros, r.z per vector
  // the final step through the FP8 codes (apply8.hip), when planned: S^T y carried per vector (Tacc)
  // and S^T p of the last directions (Uacc), both in the passes' T layout; step lengths; the
  // decision's bf16 corrections, means and flags; lambda per factor on the device; S^T 1 and the
  // ones it is formed from (centered S); whether the centered projection was applied
  double *Tacc = nullptr, *Uacc = nullptr, *alpha8 = nullptr, *abar8 = nullptr, *lamv = nullptr;
  double *cs = nullptr, *ones = nullptr;
  void* zb = nullptr;
  int64_t ldz = 0;
  int *usev = nullptr, *flag8 = nullptr, *cflag = nullptr;
};

// Where the codes of the batched call's Gram are, for the final step through them.
struct MultiF8 {
  const uint8_t* q;
  const uint8_t* sc;
  int64_t ldq;
  const double* d;   // row norms |s_i|^2
};

MultiBufs carve_multi(Carver& c, int64_t n, int64_t m, int64_t nrhs, int64_t nvec, const dfi::RowMultiPlan& rm,
                      bool need_t, bool final8 = false, bool centered = false, int64_t nfac = 1) {
  MultiBufs b{};
  b.Bs = c.take<double>((size_t)(nrhs * n));
  b.Bexp = c.take<double>((size_t)(nvec * n));
  b.Y = c.take<double>((size_t)(nvec * n));
  b.R = c.take<double>((size_t)(nvec * n));
  b.D = c.take<double>((size_t)(nvec * n));
  b.W1 = c.take<double>((size_t)(nvec * n));
  const bool two = nvec > dfi::MULTI_VECS;   // passes take two groups of vectors at a time
  b.T = need_t ? c.take<double>((size_t)(m * dfi::MULTI_VECS)) : nullptr;
  b.T1 = need_t && two ? c.take<double>((size_t)(m * dfi::MULTI_VECS)) : nullptr;
  b.Yi = c.take<double>((size_t)(n * 2 * dfi::MULTI_VECS));
  b.part = c.take<double>(rm.part_bytes / sizeof(double) + 1);
  b.part1 = need_t && two ? c.take<double>(rm.part_bytes / sizeof(double) + 1) : nullptr;
  b.Zc = c.take<double>((size_t)(nvec * n));
  b.P = c.take<double>((size_t)(nvec * n));
  b.NQ = c.take<double>((size_t)(nvec * n));
  b.zero = c.take<double>((size_t)n);
  b.rz = c.take<double>((size_t)nvec);
  if (final8) {
    const int64_t ng = (nvec + dfi::MULTI_VECS - 1) / dfi::MULTI_VECS;
    b.Tacc = c.take<double>((size_t)(ng * m * dfi::MULTI_VECS));
    b.Uacc = c.take<double>((size_t)(ng * m * dfi::MULTI_VECS));
    b.alpha8 = c.take<double>((size_t)nvec);
    b.abar8 = c.take<double>((size_t)nvec);
    b.lamv = c.take<double>((size_t)nfac);
    b.ldz = (n + 63) / 64 * 64;
    b.zb = c.take<uint16_t>((size_t)(nvec * b.ldz));
    b.usev = c.take<int>((size_t)nvec);
    b.flag8 = c.take<int>(1);
    b.cflag = c.take<int>(1);
    b.cs = centered ? c.take<double>((size_t)m) : nullptr;
    b.ones = centered ? c.take<double>((size_t)n) : nullptr;
  }
  return b;
}

dfisher_status multi_solve(const float* S, int64_t n, int64_t m, int64_t lds, int64_t nfac, const double* L,
                           const double* Dinv, const double* lams, const float* V, int64_t nrhs, int64_t ldv, void* X,
                           int64_t ldx, int x_fp64, int sweeps, const dfi::RowMultiPlan& rm, const MultiBufs& b,
                           hipStream_t st, const MultiF8* mf8 = nullptr) {
  constexpr int MV = dfi::MULTI_VECS;
  const int64_t nvec = nfac * nrhs;
  const bool f8 = mf8 && sweeps > 0 && b.Tacc;   // the final step through the codes (b carved for it)
  if (f8) HIP_TRY(dfi::put_values(b.lamv, lams, nfac, st));
  const int64_t sL = n * n;
  // B_r = S v_r, MV right-hand sides per pass over S
  for (int64_t r0 = 0; r0 < nrhs; r0 += MV) {
    const int nv = (int)std::min<int64_t>(MV, nrhs - r0);
    dfi::MultiVecs vs{};
    dfi::MultiOut mo{};
    for (int c = 0; c < nv; ++c) {
      vs.f[c] = V + (r0 + c) * ldv;
      mo.b[c] = b.Bs + (r0 + c) * n;
    }
    HIP_TRY(dfi::rowpass_multi_launch(rm, S, vs, nullptr, nv, b.part, st));
    HIP_TRY(dfi::rowpass_multi_reduce(rm, b.part, nv, mo, st));
  }
  for (int64_t f = 0; f < nfac; ++f)
    HIP_TRY(hipMemcpyAsync(b.Bexp + f * nrhs * n, b.Bs, (size_t)(nrhs * n) * sizeof(double), hipMemcpyDeviceToDevice, st));
  // Y = L^-T L^-1 B for every vector
  HIP_TRY(dfi::trsv_launch_batched(L, sL, Dinv, n, nvec, nrhs, 0, b.Bexp, b.D, b.W1, st));
  HIP_TRY(dfi::trsv_launch_batched(L, sL, Dinv, n, nvec, nrhs, 1, b.D, b.Y, b.W1, st));
  // refinement: OUT_j = RHS_j - lambda_j U_j - S (S^T U_j), MV vectors per pair of passes (the
  // conjugate-gradient sweeps of solve_y, for every vector at once; RHS = B for the residual of Y,
  // RHS = 0 for -(W P))
  // (two groups of MV vectors share each pass over S while at least MV + 1 vectors remain: every
  // load of S then feeds twice the FP64 products)
  auto group = [&](const double* U, const double* RHS, bool rhs_zero, double* OUT, int64_t j0, int nv,
                   dfi::MultiCols& mc, dfi::MultiOut& mo) {
    for (int c = 0; c < MV; ++c) mc.y[c] = U + (j0 + std::min(c, nv - 1)) * n;
    for (int c = 0; c < nv; ++c) {
      const int64_t j = j0 + c;
      mo.b[c] = OUT + j * n;
      mo.r0[c] = rhs_zero ? RHS : RHS + j * n;
      mo.y[c] = U + j * n;
      mo.lam[c] = lams[j / nrhs];
    }
  };
  // tsave (may be null): the passes' T = S^T U of group g goes to tsave + g m MV and stays there
  auto w_pass = [&](const double* U, const double* RHS, bool rhs_zero, double* OUT, double* tsave) -> dfisher_status {
    for (int64_t j0 = 0; j0 < nvec;) {
      const int nv = (int)std::min<int64_t>(MV, nvec - j0);
      const int nv1 = b.T1 ? (int)std::min<int64_t>(MV, std::max<int64_t>(0, nvec - j0 - MV)) : 0;
      double* T0 = tsave ? tsave + (j0 / MV) * m * MV : b.T;
      double* T1 = tsave ? tsave + (j0 / MV + 1) * m * MV : b.T1;
      dfi::MultiCols mc{}, mc1{};
      dfi::MultiOut mo{}, mo1{};
      group(U, RHS, rhs_zero, OUT, j0, nv, mc, mo);
      if (nv1 > 0) {
        group(U, RHS, rhs_zero, OUT, j0 + MV, nv1, mc1, mo1);
        HIP_TRY(dfi::colpass_multi_launch2(S, n, m, lds, mc, nv, mc1, nv1, 2, T0, T1, b.Yi, st));
        HIP_TRY(dfi::rowpass_multi_launch2(rm, S, T0, nv, T1, nv1, b.part, b.part1, st));
        HIP_TRY(dfi::rowpass_multi_reduce(rm, b.part, nv, mo, st));
        HIP_TRY(dfi::rowpass_multi_reduce(rm, b.part1, nv1, mo1, st));
      } else {
        HIP_TRY(dfi::colpass_multi_launch(S, n, m, lds, mc, nv, 2, T0, b.Yi, st));
        dfi::MultiVecs none{};
        HIP_TRY(dfi::rowpass_multi_launch(rm, S, none, T0, nv, b.part, st));
        HIP_TRY(dfi::rowpass_multi_reduce(rm, b.part, nv, mo, st));
      }
      j0 += nv + nv1;
    }
    return DFISHER_OK;
  };
  if (sweeps > 0) {
    HIP_TRY(dfi::fill_zero(b.zero, n, st));
    DF_TRY(w_pass(b.Y, b.Bexp, false, b.R, f8 ? b.Tacc : nullptr));
    for (int s = 1;; ++s) {
      HIP_TRY(dfi::trsv_launch_batched(L, sL, Dinv, n, nvec, nrhs, 0, b.R, b.D, b.W1, st));
      HIP_TRY(dfi::trsv_launch_batched(L, sL, Dinv, n, nvec, nrhs, 1, b.D, b.Zc, b.W1, st));
      if (s >= sweeps) {
        if (!f8) HIP_TRY(dfi::axpy_many(b.Y, b.Zc, nvec * n, st));   // else the final step takes Zc
        break;
      }
      if (s == 1) HIP_TRY(dfi::pcg_init(nullptr, n, 0, nvec, b.R, b.Zc, b.P, b.rz, st));
      else HIP_TRY(dfi::pcg_dir(nullptr, n, 0, nvec, b.R, b.Zc, b.P, b.rz, st));
      DF_TRY(w_pass(b.P, b.zero, true, b.NQ, f8 ? b.Uacc : nullptr));
      HIP_TRY(dfi::pcg_step(nullptr, n, 0, nvec, b.P, b.NQ, b.Y, b.R, b.rz, nullptr, st, nullptr,
                            f8 ? b.alpha8 : nullptr));
      // the last direction's S^T p is added by the final step itself (one pass over T less)
      if (f8 && s + 1 < sweeps) HIP_TRY(dfi::t_axpy_multi(b.Tacc, b.Uacc, b.alpha8, m, nvec, st));
    }
  }
  // the final step: every vector's last correction through the codes when the device allows it for
  // all of them (then the exact passes below return at once), else Y += Zc and the exact passes
  const int* skip = nullptr;
  if (f8) {
    HIP_TRY(dfi::multi_final8(mf8->q, mf8->sc, mf8->ldq, n, m, nvec, nrhs, b.Y, b.Zc, b.Bexp, mf8->d, b.lamv,
                              b.cs ? b.cflag : nullptr, FINAL8_EST_MAX, b.zb, b.ldz, b.abar8, b.usev, b.flag8, b.Tacc,
                              sweeps >= 2 ? b.Uacc : nullptr, b.alpha8, b.cs, V, ldv, X, ldx, x_fp64, st));
    skip = b.flag8;
  }
  // x = (v - S^T y) / lambda, up to 2 MV vectors per pass
  const size_t xel = x_fp64 ? sizeof(double) : sizeof(float);
  auto apply_group = [&](int64_t j0, int nv, dfi::MultiCols& mc) {
    for (int c = 0; c < MV; ++c) {
      const int64_t j = j0 + std::min(c, nv - 1);
      mc.y[c] = b.Y + j * n;
      mc.v[c] = V + (j % nrhs) * ldv;
      mc.x[c] = static_cast<char*>(X) + (size_t)(j * ldx) * xel;
      mc.lam[c] = lams[j / nrhs];
    }
  };
  for (int64_t j0 = 0; j0 < nvec;) {
    const int nv = (int)std::min<int64_t>(MV, nvec - j0);
    const int nv1 = (int)std::min<int64_t>(MV, std::max<int64_t>(0, nvec - j0 - MV));
    dfi::MultiCols mc{}, mc1{};
    apply_group(j0, nv, mc);
    if (nv1 > 0) {
      apply_group(j0 + MV, nv1, mc1);
      HIP_TRY(dfi::colpass_multi_launch2(S, n, m, lds, mc, nv, mc1, nv1, x_fp64 ? 1 : 0, nullptr, nullptr, b.Yi, st,
                                         skip));
    } else {
      HIP_TRY(dfi::colpass_multi_launch(S, n, m, lds, mc, nv, x_fp64 ? 1 : 0, nullptr, b.Yi, st, skip));
    }
    j0 += nv + nv1;
  }
  return DFISHER_OK;
}

// ----------------------------------------------------------------------------- autotuning
// For one size class, times the Gram stage (row pass + tile kernel + reduction) on the caller's
// S for every split-K factor q from dfi::gram_q_candidates (and, for split-BF16 on aligned rows,
// with and without the pre-split planes), keeps the fastest in ctx->tune. Each candidate runs once
// untimed and twice timed (HIP events on the stream; the minimum counts).
constexpr size_t TUNE_MAX_PART_BYTES = (size_t)4 << 30;

dfisher_status tune_gram(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds, int prec,
                         hipStream_t st) {
  const bool al = rows_aligned16(S, lds);
  int qs[16];
  int nq = 0;
  dfi::gram_q_candidates(n, m, TUNE_MAX_PART_BYTES, qs, &nq, 16);
  std::vector<int> modes = {-1};
  if (prec == DFISHER_GRAM_BF16X3 && al) modes = {1, 0};
  const dfi::RowPassPlan rp = dfi::rowpass_plan(n, m, lds);
  const dfi::ColPassPlan cp = dfi::colpass_plan(n, m);
  size_t need = 0;
  for (int mode : modes)
    for (int i = 0; i < nq; ++i) {
      const dfi::GramPlan gp = dfi::gram_plan(n, m, lds, prec, al, qs[i], mode);
      need = std::max(need, carve(nullptr, n, m, &gp, rp, cp, false, false).bytes);
    }
  DF_TRY(ensure_ws(ctx, need));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    if (e0) (void)hipEventDestroy(e0);
    return fail(DFISHER_E_DEVICE, "event creation failed");
  }
  float best = 0.f;
  int best_q = 0, best_mode = -1;
  dfisher_status rs = DFISHER_OK;
  for (int mode : modes) {
    for (int i = 0; i < nq && rs == DFISHER_OK; ++i) {
      const dfi::GramPlan gp = dfi::gram_plan(n, m, lds, prec, al, qs[i], mode);
      const SolveBufs B = carve(static_cast<char*>(ctx->ws), n, m, &gp, rp, cp, false, false);
      float tmin = 0.f;
      for (int rep = 0; rep < 3 && rs == DFISHER_OK; ++rep) {
        if (hipEventRecord(e0, st) != hipSuccess) rs = fail(DFISHER_E_DEVICE, "event record failed");
        if (rs == DFISHER_OK) rs = gram_stage(S, nullptr, gp, rp, B, 0.0, B.W, 0, st, nullptr);
        if (rs == DFISHER_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
          rs = fail(DFISHER_E_DEVICE, "event wait failed");
        float ms = 0.f;
        if (rs == DFISHER_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rs = fail(DFISHER_E_DEVICE, "timing");
        if (rep > 0 && (tmin == 0.f || ms < tmin)) tmin = ms;
      }
      if (rs == DFISHER_OK && (best_q == 0 || tmin < best)) {
        best = tmin;
        best_q = qs[i];
        best_mode = mode;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rs != DFISHER_OK) return rs;
  ctx->tune[tune_key(prec, n, m, al)] = std::make_pair(best_q, best_mode);
  drop_graph(ctx);   // a captured uneven graph may have been laid out with the old plan
  return DFISHER_OK;
}

dfisher_status tune_if_new(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds, int prec,
                           hipStream_t st) {
  if (ctx->tune.count(tune_key(prec, n, m, rows_aligned16(S, lds)))) return DFISHER_OK;
  return tune_gram(ctx, S, n, m, lds, prec, st);
}

// ----------------------------------------------------------------------------- uneven batches
// Independent problems of different sizes (per-layer Fisher blocks). Every problem runs the same
// steps as dfisher_solve, but the latency-bound steps of all problems share launches: one grouped
// Cholesky over all W_p, one grouped set of triangular solves per application of L^-1 / L^-T, and
// one update of all y_p. The streaming passes and Gram kernels run per problem, largest first,
// back to back on one stream with shared scratch. Nothing in between waits for the host, so the
// whole sequence is captured once into a HIP graph and replayed while the arguments stay the same.
// Factorisations are first tried with the policy's initial shift (none, or the up-front shift);
// after the run, problems whose factorisation failed are solved again on their own by
// dfisher_solve, which escalates the shift.

void drop_graph(dfisher_ctx* ctx) {
  if (ctx->uneven_exec) (void)hipGraphExecDestroy(ctx->uneven_exec);
  ctx->uneven_exec = nullptr;
  ctx->uneven_key.clear();
}

dfisher_status ensure_tbuf(dfisher_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->tbuf_bytes) return DFISHER_OK;
  drop_graph(ctx);   // the cached graph points into the old buffer
  if (ctx->tbuf) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(ctx->tbuf));
    ctx->tbuf = nullptr;
    ctx->tbuf_bytes = 0;
  }
  if (hipMalloc(&ctx->tbuf, bytes) != hipSuccess) {
    (void)hipGetLastError();
    ctx->tbuf = nullptr;
    return fail(DFISHER_E_NO_MEMORY, "job table allocation failed");
  }
  ctx->tbuf_bytes = bytes;
  return DFISHER_OK;
}

struct UnevenLayout {
  std::vector<dfi::GramPlan> gp;
  std::vector<dfi::RowPassPlan> rp;
  std::vector<dfi::ColPassPlan> cp;
  std::vector<dfi::RefinePassPlan> fp;   // fused refinement product, where usable
  std::vector<int64_t> voff, woff, doff;   // offsets of problem p in the concatenated vectors / matrices
  int64_t ntot = 0, nmax = 0, mmax = 0;
  SolveBufs shared{};                      // scratch reused by every problem (largest sizes)
  double *W = nullptr, *Dinv = nullptr, *dkk = nullptr, *dmax = nullptr;
  double *b = nullptr, *d = nullptr, *y = nullptr, *z = nullptr, *r = nullptr, *wk = nullptr;
  double *zc = nullptr, *p = nullptr, *nq = nullptr, *zero = nullptr, *rz = nullptr;   // refinement (PCG)
  double *bb = nullptr, *rr = nullptr, *prev = nullptr, *resid = nullptr;   // per table entry
  int *stop = nullptr, *done = nullptr, *met = nullptr;
  int64_t* info = nullptr;
  int32_t* flag = nullptr;
  double* res = nullptr;                   // final residuals: |b_p|^2, |r_p|^2 per problem
  // the final step through the FP8 codes (apply8.hip), when every problem allows it: each problem's
  // codes kept (not shared scratch), S^T y carried through its passes, S^T p, S^T 1 (centered)
  bool f8 = false;
  std::vector<int64_t> qoff, soff, moff;   // per problem: codes, scales, m-vector offsets
  uint8_t *q8all = nullptr, *sc8all = nullptr;
  double *T8 = nullptr, *U8 = nullptr, *cs8 = nullptr;
  double* a8 = nullptr;                    // [table entry] step length, [np + p] the correction's mean
  float* zf8 = nullptr;                    // ntot
  int* use8 = nullptr;                     // [p] final step through the codes, [np + p] projection applied
  // grouped whole-line passes: the problems whose fused pass is a one-workgroup-per-block line
  // plan run their passes of a sweep in shared launches, each with its own partials
  std::vector<char> gline;                 // per problem
  std::vector<int64_t> loff;               // per problem: offset (doubles) of its partials in lpart
  double* lpart = nullptr;
  // grouped Gram (with f8: every problem's codes are kept): one launch over all problems' work
  // items, each problem with one slice per XCD (the launch, not the problem, fills the device) and
  // its own partial tiles at gall + goff[p]
  std::vector<dfi::GramPlan> gpg;
  std::vector<int64_t> goff;               // floats
  float* gall = nullptr;
  size_t bytes = 0;
};

// The uneven call keeps every problem's codes for the FP8 final step only while they take at most
// this much memory (for the 64-problem bench batch, 34 GB)
constexpr size_t UNEVEN_F8_MAX_CODE_BYTES = (size_t)64 << 30;

void uneven_layout(const dfisher_ctx* ctx, char* base, int32_t np, const float* const* S, const int64_t* n,
                   const int64_t* m, const int64_t* lds, int prec, int sweeps, UnevenLayout& U, bool want_f8 = false,
                   bool centered = false) {
  U.gp.clear();
  U.rp.clear();
  U.cp.clear();
  U.fp.clear();
  U.voff.assign((size_t)np, 0);
  U.woff.assign((size_t)np, 0);
  U.doff.assign((size_t)np, 0);
  U.ntot = U.nmax = U.mmax = 0;
  int64_t wtot = 0, dtot = 0;
  size_t gpart = 0, rpart = 0, cpart = 0, q8 = 0, sc8 = 0, planes = 0;
  for (int32_t p = 0; p < np; ++p) {
    U.gp.push_back(make_gram_plan(ctx, S[p], n[p], m[p], lds[p], prec));
    U.rp.push_back(dfi::rowpass_plan(n[p], m[p], lds[p]));
    U.cp.push_back(dfi::colpass_plan(n[p], m[p]));
    U.fp.push_back(dfi::refine_pass_plan(n[p], m[p], lds[p], S[p]));
    U.voff[(size_t)p] = U.ntot;
    U.woff[(size_t)p] = wtot;
    U.doff[(size_t)p] = dtot;
    U.ntot += n[p];
    wtot += n[p] * n[p];
    dtot += (int64_t)(dfi::trsv_dinv_bytes(n[p]) / sizeof(double));
    U.nmax = std::max(U.nmax, n[p]);
    U.mmax = std::max(U.mmax, m[p]);
    gpart = std::max(gpart, U.gp.back().part_bytes);
    rpart = std::max(rpart, std::max(U.rp.back().part_bytes, U.fp.back().part_bytes));
    cpart = std::max(cpart, U.cp.back().part_bytes);
    const int64_t ldq = dfi::fp8_ldq(m[p]);
    if (prec == DFISHER_GRAM_MXFP8) {
      q8 = std::max(q8, (size_t)(n[p] * ldq));
      sc8 = std::max(sc8, (size_t)(n[p] * (ldq / 32)));
    }
    if (U.gp.back().ldh > 0) planes = std::max(planes, (size_t)(n[p] * U.gp.back().ldh));
  }
  // the FP8 final step: scaled-FP8 Gram, whole-line passes for every problem, codes within the cap
  U.f8 = want_f8 && prec == DFISHER_GRAM_MXFP8;
  size_t qall = 0, sall = 0;
  int64_t mall = 0;
  U.qoff.assign((size_t)np, 0);
  U.soff.assign((size_t)np, 0);
  U.moff.assign((size_t)np, 0);
  for (int32_t p = 0; p < np && U.f8; ++p) {
    if (!U.fp[(size_t)p].usable || !U.fp[(size_t)p].line) U.f8 = false;
    const int64_t ldq = dfi::fp8_ldq(m[p]);
    U.qoff[(size_t)p] = (int64_t)qall;
    U.soff[(size_t)p] = (int64_t)sall;
    U.moff[(size_t)p] = mall;
    qall += align_up((size_t)(n[p] * ldq));
    sall += align_up((size_t)(n[p] * (ldq / 32)));
    mall += (m[p] + 31) / 32 * 32;
  }
  if (qall + sall > UNEVEN_F8_MAX_CODE_BYTES) U.f8 = false;
  U.gpg.clear();
  U.goff.assign((size_t)np, 0);
  size_t gall = 0;
  for (int32_t p = 0; p < np && U.f8; ++p) {
    U.gpg.push_back(dfi::gram_plan(n[p], m[p], lds[p], prec, true, 1));
    U.goff[(size_t)p] = (int64_t)gall;
    gall += std::max(U.gpg.back().part_bytes, dfi::gram_project_work_bytes(n[p])) / sizeof(float);
    gall = (gall + 63) / 64 * 64;   // 256-byte aligned regions
  }
  U.gline.assign((size_t)np, 0);
  U.loff.assign((size_t)np, 0);
  size_t lall = 0;
  for (int32_t p = 0; p < np; ++p) {
    const dfi::RefinePassPlan& f = U.fp[(size_t)p];
    if (!f.usable || !f.line || f.split) continue;
    U.gline[(size_t)p] = 1;
    U.loff[(size_t)p] = (int64_t)lall;
    lall += f.part_bytes / sizeof(double);
  }
  Carver c;
  c.base = base;
  SolveBufs& B = U.shared;
  B = SolveBufs{};
  B.gpart = c.take<float>(gpart / sizeof(float) + 1);
  B.rpart = c.take<double>(rpart / sizeof(double) + 1);
  B.cpart = c.take<double>(cpart / sizeof(double) + 1);
  B.t = sweeps > 0 ? c.take<double>((size_t)U.mmax) : nullptr;
  B.q8 = q8 && !U.f8 ? c.take<uint8_t>(q8) : nullptr;
  B.sc8 = sc8 && !U.f8 ? c.take<uint8_t>(sc8) : nullptr;
  U.q8all = U.f8 ? c.take<uint8_t>(qall) : nullptr;
  U.sc8all = U.f8 ? c.take<uint8_t>(sall) : nullptr;
  U.T8 = U.f8 ? c.take<double>((size_t)mall) : nullptr;
  U.U8 = U.f8 ? c.take<double>((size_t)mall) : nullptr;
  U.cs8 = U.f8 && centered ? c.take<double>((size_t)mall) : nullptr;
  B.hi = planes ? c.take<uint16_t>(planes) : nullptr;
  B.lo = planes ? c.take<uint16_t>(planes) : nullptr;
  U.W = c.take<double>((size_t)wtot);
  U.Dinv = c.take<double>((size_t)dtot);
  U.dkk = c.take<double>((size_t)np * 64 * 64);
  U.dmax = c.take<double>((size_t)np);
  U.b = c.take<double>((size_t)U.ntot);
  U.d = c.take<double>((size_t)U.ntot);
  U.y = c.take<double>((size_t)U.ntot);
  U.z = c.take<double>((size_t)U.ntot);
  U.r = c.take<double>((size_t)U.ntot);
  U.wk = c.take<double>((size_t)U.ntot);
  U.zc = c.take<double>((size_t)U.ntot);
  U.p = c.take<double>((size_t)U.ntot);
  U.nq = c.take<double>((size_t)U.ntot);
  U.zero = c.take<double>((size_t)U.nmax);
  U.rz = c.take<double>((size_t)np);
  U.bb = c.take<double>((size_t)np);
  U.rr = c.take<double>((size_t)np);
  U.prev = c.take<double>((size_t)np);
  U.resid = c.take<double>((size_t)np);
  U.stop = c.take<int>((size_t)np);
  U.done = c.take<int>((size_t)np);
  U.met = c.take<int>((size_t)np);
  U.info = c.take<int64_t>((size_t)np);
  U.flag = c.take<int32_t>((size_t)np);
  U.res = c.take<double>((size_t)(2 * np));
  U.a8 = U.f8 ? c.take<double>((size_t)(2 * np)) : nullptr;
  U.zf8 = U.f8 ? c.take<float>((size_t)U.ntot) : nullptr;
  U.use8 = U.f8 ? c.take<int>((size_t)(2 * np)) : nullptr;
  U.lpart = lall ? c.take<double>(lall) : nullptr;
  U.gall = gall ? c.take<float>(gall) : nullptr;
  U.bytes = c.off;
}

// Device tables of the grouped whole-line passes (uneven_solve builds them): per line class
// (8, 16, 32 loads per lane) the residual pass's jobs and the conjugate-gradient pass's, in table
// order (decreasing sweep cap), so that the problems that may run sweep s are a prefix; the counts
// and workgroup / block totals of that prefix per sweep; and the residuals' jobs likewise.
struct GroupedPasses {
  bool on = false;
  bool cs = false;                            // the residual pass also forms S^T 1
  const dfi::LineJob* res[3] = {nullptr, nullptr, nullptr};
  int nres[3] = {0, 0, 0};
  int64_t wres[3] = {0, 0, 0};
  const dfi::LineJob* cg[3] = {nullptr, nullptr, nullptr};
  std::vector<int> ncg[3];                    // [class][s]: jobs with a cap > s
  std::vector<int64_t> wcg[3];
  const dfi::ReduceJob* rres = nullptr;
  int nrres = 0;
  int64_t brres = 0;
  const dfi::ReduceJob* rcg = nullptr;
  std::vector<int> nrcg;                      // [s]
  std::vector<int64_t> brcg;
  const dfi::GramJob* gram = nullptr;         // the grouped Gram's jobs (largest work item first)
  int ngram = 0;
  int64_t gram_nwg = 0;
};
constexpr int LINE_CLASSES[3] = {8, 16, 32};

// Enqueues the whole uneven solve on st (no host synchronisation). fjobs / tjobs: device tables.
// sw[p]: problem p's sweep count. The job tables list the problems by decreasing sweep count, so
// the problems still refining in sweep s are the first nactive[s] entries of each table.
dfisher_status uneven_enqueue(dfisher_ctx* ctx, int32_t np, const float* const* S, const int64_t* n, const int64_t* m,
                              const int64_t* lds, const float* const* v, const double* lambda, void* const* x,
                              const dfisher_options& o, const UnevenLayout& U, const std::vector<int32_t>& order,
                              const std::vector<int>& sw, const std::vector<int64_t>& nactive,
                              const dfi::FactorJob* fjobs, const dfi::TrsvJob* tj_fwd, const dfi::TrsvJob* tj_bwd,
                              const dfi::TrsvJob* tj_bwd_c, const int64_t* seg, const int* cap, double tol,
                              bool predict, const std::vector<int32_t>& jpos, const GroupedPasses& G,
                              hipStream_t st) {
  (void)ctx;
  // Gram stage, largest first: b_p = S_p v_p, d_p, W_p = S_p S_p^T + lambda_p I. With every
  // problem's codes kept (f8): the row passes per problem, then one Gram launch over all problems'
  // work items, then each problem's reduction, projection and shift; else the whole stage per
  // problem.
  if (G.ngram > 0) {
    for (int32_t p : order) {
      const size_t q = (size_t)p;
      double* rpart = U.shared.rpart;
      HIP_TRY(dfi::rowpass_launch(U.rp[q], S[p], v[p], nullptr, true, true, rpart, st, U.q8all + U.qoff[q],
                                  U.sc8all + U.soff[q], dfi::fp8_ldq(m[p]), true));
      HIP_TRY(dfi::rowpass_reduce(U.rp[q], rpart, true, true, U.b + U.voff[q], U.d + U.voff[q], nullptr, nullptr, 0.0,
                                  st));
    }
    HIP_TRY(dfi::gram_launch_fp8_grouped(G.gram, G.ngram, G.gram_nwg, st));
  }
  for (int32_t p : order) {
    if (G.ngram > 0) {
      const size_t q = (size_t)p;
      double* Wp = U.W + U.woff[q];
      float* gp = U.gall + U.goff[q];
      HIP_TRY(dfi::gram_reduce(U.gpg[q], S[p], gp, U.d + U.voff[q], lambda[p], Wp, 0, st));
      if (is_centered(o))   // the partial tiles are free again: they hold the projection's tile sums
        HIP_TRY(dfi::gram_project(Wp, n[p], 1, lambda[p], 0, reinterpret_cast<double*>(gp), U.zc + U.voff[q], st,
                                  U.cs8 ? U.use8 + np + p : nullptr));
      if (o.shift_policy == DFISHER_SHIFT_ALWAYS) {
        const double scale = 2.0 * std::sqrt((double)n[p]) * gram_unit(o.gram_prec, m[p]);
        HIP_TRY(dfi::diag_max(Wp, n[p], U.dmax + p, st));
        HIP_TRY(dfi::shift_add_copy(Wp, Wp, n[p], scale, U.dmax + p, 0.0, st));
      }
      continue;
    }
    SolveBufs B = U.shared;
    B.b = U.b + U.voff[(size_t)p];
    B.d = U.d + U.voff[(size_t)p];
    B.ldq = dfi::fp8_ldq(m[p]);
    if (U.gp[(size_t)p].ldh == 0) B.hi = B.lo = nullptr;   // this problem splits inside the tile kernel
    B.zc = U.zc + U.voff[(size_t)p];   // projection work (free until the refinement)
    if (U.f8) {   // this problem's own codes, kept for its final step
      B.q8 = U.q8all + U.qoff[(size_t)p];
      B.sc8 = U.sc8all + U.soff[(size_t)p];
    }
    DF_TRY(gram_stage(S[p], v[p], U.gp[(size_t)p], U.rp[(size_t)p], B, lambda[p], U.W + U.woff[(size_t)p], 0, st,
                      nullptr, is_centered(o), U.cs8 ? U.use8 + np + p : nullptr));
    if (o.shift_policy == DFISHER_SHIFT_ALWAYS) {
      double* Wp = U.W + U.woff[(size_t)p];
      const double scale = 2.0 * std::sqrt((double)n[p]) * gram_unit(o.gram_prec, m[p]);
      HIP_TRY(dfi::diag_max(Wp, n[p], U.dmax + p, st));
      HIP_TRY(dfi::shift_add_copy(Wp, Wp, n[p], scale, U.dmax + p, 0.0, st));
    }
  }
  // all Cholesky factorisations in the same launches (in place), then the diagonal-block inverses
  HIP_TRY(dfi::potrf_launch_grouped(fjobs, np, U.nmax, st));
  HIP_TRY(dfi::trsv_diag_inv_grouped(tj_fwd, np, U.nmax, st));
  const size_t vb = (size_t)U.ntot * sizeof(double);
  // y = L^-T L^-1 b for every problem (wk is each solve's reduced right-hand side)
  HIP_TRY(hipMemcpyAsync(U.wk, U.b, vb, hipMemcpyDeviceToDevice, st));
  HIP_TRY(dfi::trsv_launch_grouped(tj_fwd, np, U.nmax, 0, st));    // wk -> z
  HIP_TRY(hipMemcpyAsync(U.wk, U.z, vb, hipMemcpyDeviceToDevice, st));
  HIP_TRY(dfi::trsv_launch_grouped(tj_bwd, np, U.nmax, 1, st));    // wk -> y
  // out_p = rhs_p - lambda_p u_p - S_p (S_p^T u_p) (FP64 accumulation): the residual of y_p
  // (rhs = b, u = y) or -(W_p p_p) (rhs = 0, u = p)
  // (skip: the problem's stop flag; its fused pass then reads nothing. The column pass + row pass
  // fallback runs regardless: its result is then unused.)
  auto w_pass = [&](int32_t p, const double* u, const double* rhs, bool rhs_zero, double* out,
                    const int* skip = nullptr, double* tout = nullptr, double* csout = nullptr) -> dfisher_status {
    const int64_t off = U.voff[(size_t)p];
    const double* rh = rhs_zero ? rhs : rhs + off;
    if (U.fp[(size_t)p].usable) {   // one read of S_p
      HIP_TRY(dfi::refine_pass_launch(U.fp[(size_t)p], S[p], n[p], m[p], lds[p], u + off, U.shared.rpart, st, skip, -1,
                                      tout, csout));
      HIP_TRY(dfi::refine_pass_reduce(U.fp[(size_t)p], U.shared.rpart, out + off, rh, u + off, lambda[p], st, skip));
      return DFISHER_OK;
    }
    HIP_TRY(dfi::colpass_launch(U.cp[(size_t)p], S[p], n[p], m[p], lds[p], u + off, nullptr, 1.0, U.shared.t, 2,
                                U.shared.cpart, st));
    HIP_TRY(dfi::rowpass_launch(U.rp[(size_t)p], S[p], nullptr, U.shared.t, true, false, U.shared.rpart, st));
    HIP_TRY(dfi::rowpass_reduce(U.rp[(size_t)p], U.shared.rpart, true, false, out + off, nullptr, rh, u + off,
                                lambda[p], st));
    return DFISHER_OK;
  };
  auto residual = [&](int32_t p) -> dfisher_status { return w_pass(p, U.y, U.b, false, U.r); };
  // the first residual also carries S^T y_0 (and S^T 1) for the FP8 final step
  auto residual0 = [&](int32_t p) -> dfisher_status {
    if (!U.f8) return residual(p);
    const int64_t mo = U.moff[(size_t)p];
    return w_pass(p, U.y, U.b, false, U.r, nullptr, U.T8 + mo, U.cs8 ? U.cs8 + mo : nullptr);
  };
  // the conjugate-gradient sweeps of solve_y, per problem, with the stop test on the device: the job
  // tables and the segment table list the problems by decreasing sweep cap, so the problems that
  // may still run sweep s (cap >= s) are the first nactive[s - 1] entries; a problem that has
  // stopped (tolerance met or cap reached) skips its passes and vector steps from then on
  const int max_sw = nactive.empty() ? 0 : (int)nactive.size();
  if (max_sw > 0) {
    dfi::PcgControl c{};
    c.bb = U.bb;
    c.rr = U.rr;
    c.prev = U.prev;
    c.stop = U.stop;
    c.cap = cap;
    c.done = U.done;
    c.resid = U.resid;
    c.met = U.met;
    c.tol = tol;
    c.floor = auto_floor(o);
    c.predict = predict ? 1 : 0;
    c.keep = U.f8 ? 1 : 0;
    HIP_TRY(dfi::pcg_control_init(np, c, st));
    HIP_TRY(dfi::fill_zero(U.zero, U.nmax, st));
    // the residual passes: the grouped line problems in one launch per class, the rest alone
    if (G.on) {
      for (int c = 0; c < 3; ++c)
        if (G.nres[c] > 0)
          HIP_TRY(dfi::refine_line_grouped_launch(G.res[c], G.nres[c], LINE_CLASSES[c], G.cs, G.wres[c], st));
      if (G.nrres > 0) HIP_TRY(dfi::refine_reduce_grouped(G.rres, G.nrres, G.brres, st));
    }
    for (int32_t p : order)
      if (sw[(size_t)p] > 0 && !(G.on && U.gline[(size_t)p])) DF_TRY(residual0(p));
    HIP_TRY(dfi::seg_sumsq(seg, 0, 0, nactive[0], U.b, U.bb, st));
    HIP_TRY(dfi::seg_sumsq(seg, 0, 0, nactive[0], U.r, U.rr, st));
    for (int s = 1;; ++s) {
      const int64_t act = nactive[(size_t)(s - 1)];
      const int64_t cont = s < max_sw ? nactive[(size_t)s] : 0;
      // zc = L^-T L^-1 r for the problems that may run this sweep
      HIP_TRY(hipMemcpyAsync(U.wk, U.r, vb, hipMemcpyDeviceToDevice, st));
      HIP_TRY(dfi::trsv_launch_grouped(tj_fwd, act, U.nmax, 0, st));     // wk -> z
      HIP_TRY(hipMemcpyAsync(U.wk, U.z, vb, hipMemcpyDeviceToDevice, st));
      HIP_TRY(dfi::trsv_launch_grouped(tj_bwd_c, act, U.nmax, 1, st));   // wk -> zc
      HIP_TRY(dfi::pcg_decide(seg, 0, 0, act, s, c, U.zc, U.y, st));      // stop: y += zc
      if (cont == 0) break;
      if (s == 1) HIP_TRY(dfi::pcg_init(seg, 0, 0, cont, U.r, U.zc, U.p, U.rz, st, U.stop));
      else HIP_TRY(dfi::pcg_dir(seg, 0, 0, cont, U.r, U.zc, U.p, U.rz, st, U.stop));
      if (G.on) {   // -(W_p p_p) for the grouped line problems with a cap > s
        for (int c = 0; c < 3; ++c)
          if (G.ncg[c][(size_t)s] > 0)
            HIP_TRY(dfi::refine_line_grouped_launch(G.cg[c], G.ncg[c][(size_t)s], LINE_CLASSES[c], false,
                                                    G.wcg[c][(size_t)s], st));
        if (G.nrcg[(size_t)s] > 0) HIP_TRY(dfi::refine_reduce_grouped(G.rcg, G.nrcg[(size_t)s], G.brcg[(size_t)s], st));
      }
      for (int32_t p : order)
        if (sw[(size_t)p] > s && !(G.on && U.gline[(size_t)p]))
          DF_TRY(w_pass(p, U.p, U.zero, true, U.nq, U.stop + jpos[(size_t)p],
                        U.f8 ? U.U8 + U.moff[(size_t)p] : nullptr));   // -(W_p p_p)
      HIP_TRY(dfi::pcg_step(seg, 0, 0, cont, U.p, U.nq, U.y, U.r, U.rz, U.rr, st, U.stop, U.a8));
      if (U.f8)   // T_p += alpha_p S^T p_p for the problems that took this step
        for (int32_t p : order)
          if (sw[(size_t)p] > s) {
            const int64_t mo = U.moff[(size_t)p];
            HIP_TRY(dfi::t_axpy(U.T8 + mo, U.U8 + mo, U.a8 + jpos[(size_t)p], m[p], st, U.stop + jpos[(size_t)p]));
          }
    }
  }
  if (o.final_resid) {   // the returned iterate's residual, per problem (not applied)
    for (int32_t p : order) {
      DF_TRY(residual(p));
      HIP_TRY(dfi::sumsq(U.b + U.voff[(size_t)p], n[p], U.res + 2 * p, st));
      HIP_TRY(dfi::sumsq(U.r + U.voff[(size_t)p], n[p], U.res + 2 * p + 1, st));
    }
  }
  // x_p = (v_p - S_p^T y_p) / lambda_p: with the FP8 final step, the last correction (left in zc)
  // through the problem's codes when the device finds that accurate enough, else y_p += zc_p and
  // the exact column pass (one of the two returns at once)
  for (int32_t p : order) {
    const int64_t off = U.voff[(size_t)p];
    const int* use = nullptr;
    if (U.f8 && sw[(size_t)p] > 0) {
      const int64_t mo = U.moff[(size_t)p];
      use = U.use8 + p;
      HIP_TRY(dfi::final_decide(n[p], U.y + off, U.zc + off, U.b + off, U.d + off, lambda[p],
                                U.cs8 ? U.use8 + np + p : nullptr, FINAL8_EST_MAX, U.zf8 + off, U.a8 + np + p, U.use8 + p,
                                st));
      HIP_TRY(dfi::fp8_apply(U.q8all + U.qoff[(size_t)p], U.sc8all + U.soff[(size_t)p], dfi::fp8_ldq(m[p]), n[p], m[p],
                             U.zf8 + off, U.T8 + mo, U.cs8 ? U.cs8 + mo : nullptr, U.a8 + np + p, v[p], lambda[p], x[p],
                             o.x_fp64, U.use8 + p, st));
    }
    HIP_TRY(dfi::colpass_launch(U.cp[(size_t)p], S[p], n[p], m[p], lds[p], U.y + off, v[p], lambda[p], x[p], o.x_fp64,
                                U.shared.cpart, st, use));
  }
  return DFISHER_OK;
}

dfisher_status uneven_solve(dfisher_ctx* ctx, int32_t np, const float* const* S, const int64_t* n, const int64_t* m,
                            const int64_t* lds, const float* const* v, const double* lambda, void* const* x,
                            const dfisher_options& o, hipStream_t st, dfisher_info* infos) {
  if (ctx->autotune)
    for (int32_t p = 0; p < np; ++p) DF_TRY(tune_if_new(ctx, S[p], n[p], m[p], lds[p], o.gram_prec, st));
  // sweep cap per problem. DFISHER_SWEEPS_AUTO: the a-priori count for its precision, shape and
  // up-front shift plus two, with the stop test measured on the device (predictive, aim tol or 1e-7);
  // fixed sweeps: that count, stopping early on a measured tol when one is given.
  const bool autos = o.sweeps == DFISHER_SWEEPS_AUTO;
  const double tol = autos && !(o.tol > 0.0) ? AUTO_TOL : o.tol;
  std::vector<int> sw((size_t)np, o.sweeps);
  int max_sw = 0;
  for (int32_t p = 0; p < np; ++p) {
    if (autos) {
      const double tau_rel = o.shift_policy == DFISHER_SHIFT_ALWAYS
                                 ? 2.0 * std::sqrt((double)n[p]) * gram_unit(o.gram_prec, m[p]) : 0.0;
      sw[(size_t)p] = std::min(MAX_SWEEPS, auto_sweeps(o.gram_prec, n[p], m[p], tau_rel, is_centered(o)) + 2);
    }
    max_sw = std::max(max_sw, sw[(size_t)p]);
  }
  UnevenLayout U;
  const int need_t = (max_sw > 0 || o.final_resid) ? 1 : 0;
  const bool want_f8 = o.sweeps != 0 && !o.final_resid && (o.flags & DFISHER_EXACT_APPLY) == 0;
  uneven_layout(ctx, nullptr, np, S, n, m, lds, o.gram_prec, need_t, U, want_f8, is_centered(o));
  DF_TRY(ensure_ws(ctx, U.bytes));
  uneven_layout(ctx, static_cast<char*>(ctx->ws), np, S, n, m, lds, o.gram_prec, need_t, U, want_f8, is_centered(o));
  // largest problems first (their Gram kernels fill the device; small ones follow)
  std::vector<int32_t> order((size_t)np);
  for (int32_t p = 0; p < np; ++p) order[(size_t)p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return (double)n[a] * (double)n[a] * (double)m[a] > (double)n[b] * (double)n[b] * (double)m[b];
  });
  // job tables: factor jobs, forward solves (wk -> z, the first entry set also drives diag_inv)
  // and backward solves (wk -> y for the first solve, wk -> zc inside sweeps: two tables)
  // table entry j holds problem jord[j]: decreasing sweep count, so that the problems still
  // refining in sweep s are a prefix of the tables (nactive[s] entries)
  std::vector<int32_t> jord((size_t)np);
  for (int32_t p = 0; p < np; ++p) jord[(size_t)p] = p;
  std::stable_sort(jord.begin(), jord.end(), [&](int32_t a, int32_t b) { return sw[(size_t)a] > sw[(size_t)b]; });
  std::vector<int64_t> nactive((size_t)max_sw, 0);
  for (int s = 0; s < max_sw; ++s)
    for (int32_t p = 0; p < np; ++p) nactive[(size_t)s] += sw[(size_t)p] > s ? 1 : 0;
  std::vector<dfi::FactorJob> fj((size_t)np);
  std::vector<dfi::TrsvJob> tf((size_t)np), tb((size_t)np), tr((size_t)np);
  std::vector<int64_t> seg((size_t)(2 * np));   // refinement vectors in table order: (offset, length)
  std::vector<int> capj((size_t)np);               // sweep cap in table order
  std::vector<int32_t> jpos((size_t)np);           // table entry of each problem
  for (int32_t j = 0; j < np; ++j) {
    const int32_t p = jord[(size_t)j];
    const size_t q = (size_t)p;
    double* Wp = U.W + U.woff[q];
    fj[(size_t)j] = dfi::FactorJob{Wp, n[p], U.info + p, U.flag + p, U.dkk + (int64_t)p * 64 * 64};
    tf[(size_t)j] = dfi::TrsvJob{Wp, U.Dinv + U.doff[q], n[p], U.wk + U.voff[q], U.z + U.voff[q]};
    tb[(size_t)j] = dfi::TrsvJob{Wp, U.Dinv + U.doff[q], n[p], U.wk + U.voff[q], U.y + U.voff[q]};
    tr[(size_t)j] = dfi::TrsvJob{Wp, U.Dinv + U.doff[q], n[p], U.wk + U.voff[q], U.zc + U.voff[q]};
    seg[(size_t)(2 * j)] = U.voff[q];
    seg[(size_t)(2 * j + 1)] = n[p];
    capj[(size_t)j] = sw[q];
    jpos[q] = j;
  }
  // grouped whole-line passes, in table order: per class the residual jobs (cap > 0) and the
  // conjugate-gradient jobs (cap > 1), and the matching residual-reduction jobs
  GroupedPasses G;
  std::vector<dfi::LineJob> lres[3], lcg[3];
  std::vector<dfi::ReduceJob> rres, rcg;
  std::vector<int> capcg[3], caprcg;   // each cg job's cap, for the per-sweep prefixes
  for (int32_t j = 0; j < np; ++j) {
    const int32_t p = jord[(size_t)j];
    const size_t q = (size_t)p;
    if (!U.gline[q] || sw[q] == 0) continue;
    const dfi::RefinePassPlan& f = U.fp[q];
    const int c = f.lnch == 8 ? 0 : (f.lnch == 16 ? 1 : 2);
    const int64_t off = U.voff[q];
    const int64_t mo = U.f8 ? U.moff[q] : 0;
    double* part = U.lpart + U.loff[q];
    const int64_t nb16 = (n[p] + 15) / 16;
    lres[c].push_back(dfi::LineJob{S[p], U.y + off, part, U.f8 ? U.T8 + mo : nullptr, U.cs8 ? U.cs8 + mo : nullptr,
                                   nullptr, n[p], m[p], lds[p], f.R, G.wres[c], f.ngroups});
    G.wres[c] += f.ngroups;
    rres.push_back(dfi::ReduceJob{part, U.b + off, U.y + off, U.r + off, nullptr, lambda[p], n[p], f.ngroups, G.brres});
    G.brres += nb16;
    if (sw[q] > 1) {
      const int64_t w0 = lcg[c].empty() ? 0 : lcg[c].back().wg0 + lcg[c].back().ngroups;
      lcg[c].push_back(dfi::LineJob{S[p], U.p + off, part, U.f8 ? U.U8 + mo : nullptr, nullptr, U.stop + j, n[p], m[p],
                                    lds[p], f.R, w0, f.ngroups});
      capcg[c].push_back(sw[q]);
      const int64_t b0 = rcg.empty() ? 0 : rcg.back().blk0 + (rcg.back().n + 15) / 16;
      rcg.push_back(dfi::ReduceJob{part, U.zero, U.p + off, U.nq + off, U.stop + j, lambda[p], n[p], f.ngroups, b0});
      caprcg.push_back(sw[q]);
    }
  }
  G.on = !rres.empty();
  G.cs = U.cs8 != nullptr;
  for (int c = 0; c < 3; ++c) {
    G.nres[c] = (int)lres[c].size();
    G.ncg[c].assign((size_t)std::max(max_sw, 1), 0);
    G.wcg[c].assign((size_t)std::max(max_sw, 1), 0);
    for (int s = 0; s < max_sw; ++s)
      for (size_t k = 0; k < lcg[c].size(); ++k)
        if (capcg[c][k] > s) {   // a prefix: the caps decrease along the table
          G.ncg[c][(size_t)s] = (int)k + 1;
          G.wcg[c][(size_t)s] = lcg[c][k].wg0 + lcg[c][k].ngroups;
        }
  }
  // the grouped Gram's jobs: largest work item (slice length) first, then more tiles first
  std::vector<dfi::GramJob> gjobs;
  if (U.f8) {
    std::vector<int32_t> gord((size_t)np);
    for (int32_t p = 0; p < np; ++p) gord[(size_t)p] = p;
    std::stable_sort(gord.begin(), gord.end(), [&](int32_t a, int32_t b) {
      const dfi::GramPlan &ga = U.gpg[(size_t)a], &gb = U.gpg[(size_t)b];
      return ga.kslice != gb.kslice ? ga.kslice > gb.kslice : ga.ntri > gb.ntri;
    });
    int64_t w0 = 0;
    for (int32_t p : gord) {
      const size_t q = (size_t)p;
      const dfi::GramPlan& g = U.gpg[q];
      const int64_t ldq = dfi::fp8_ldq(m[p]);
      if (g.nslice * g.kslice < ldq || (g.kslice & 63) != 0 || (g.nslice & 7) != 0)
        return fail(DFISHER_E_DEVICE, "grouped Gram plan of problem %d does not cover its codes", (int)p);
      gjobs.push_back(dfi::GramJob{U.q8all + U.qoff[q], U.sc8all + U.soff[q], U.gall + U.goff[q], n[p], ldq, g.ntri,
                                   g.nslice, g.kslice, w0});
      w0 += g.ntri * g.nslice;
    }
    G.ngram = (int)gjobs.size();
    G.gram_nwg = w0;
  }
  G.nrres = (int)rres.size();
  G.nrcg.assign((size_t)std::max(max_sw, 1), 0);
  G.brcg.assign((size_t)std::max(max_sw, 1), 0);
  for (int s = 0; s < max_sw; ++s)
    for (size_t k = 0; k < rcg.size(); ++k)
      if (caprcg[k] > s) {
        G.nrcg[(size_t)s] = (int)k + 1;
        G.brcg[(size_t)s] = rcg[k].blk0 + (rcg[k].n + 15) / 16;
      }
  size_t lbytes[3], lcgbytes[3];
  size_t gbytes = 0;
  for (int c = 0; c < 3; ++c) {
    lbytes[c] = align_up(lres[c].size() * sizeof(dfi::LineJob));
    lcgbytes[c] = align_up(lcg[c].size() * sizeof(dfi::LineJob));
    gbytes += lbytes[c] + lcgbytes[c];
  }
  const size_t rrbytes = align_up(rres.size() * sizeof(dfi::ReduceJob));
  const size_t rcbytes = align_up(rcg.size() * sizeof(dfi::ReduceJob));
  const size_t gjbytes = align_up(gjobs.size() * sizeof(dfi::GramJob));
  gbytes += rrbytes + rcbytes + gjbytes;
  const size_t fbytes = align_up(fj.size() * sizeof(dfi::FactorJob));
  const size_t tbytes = align_up(tf.size() * sizeof(dfi::TrsvJob));
  const size_t sbytes = align_up(seg.size() * sizeof(int64_t));
  const size_t cbytes = align_up(capj.size() * sizeof(int));
  DF_TRY(ensure_tbuf(ctx, fbytes + 3 * tbytes + sbytes + cbytes + gbytes));
  char* tb0 = static_cast<char*>(ctx->tbuf);
  auto* d_fj = reinterpret_cast<dfi::FactorJob*>(tb0);
  auto* d_tf = reinterpret_cast<dfi::TrsvJob*>(tb0 + fbytes);
  auto* d_tb = reinterpret_cast<dfi::TrsvJob*>(tb0 + fbytes + tbytes);
  auto* d_tr = reinterpret_cast<dfi::TrsvJob*>(tb0 + fbytes + 2 * tbytes);
  auto* d_seg = reinterpret_cast<int64_t*>(tb0 + fbytes + 3 * tbytes);
  auto* d_cap = reinterpret_cast<int*>(tb0 + fbytes + 3 * tbytes + sbytes);
  HIP_TRY(hipMemcpyAsync(d_fj, fj.data(), fj.size() * sizeof(dfi::FactorJob), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_tf, tf.data(), tf.size() * sizeof(dfi::TrsvJob), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_tb, tb.data(), tb.size() * sizeof(dfi::TrsvJob), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_tr, tr.data(), tr.size() * sizeof(dfi::TrsvJob), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_seg, seg.data(), seg.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_cap, capj.data(), capj.size() * sizeof(int), hipMemcpyHostToDevice, st));
  {
    char* gp = tb0 + fbytes + 3 * tbytes + sbytes + cbytes;
    for (int c = 0; c < 3; ++c) {
      auto* dres = reinterpret_cast<dfi::LineJob*>(gp);
      auto* dcg = reinterpret_cast<dfi::LineJob*>(gp + lbytes[c]);
      if (!lres[c].empty())
        HIP_TRY(hipMemcpyAsync(dres, lres[c].data(), lres[c].size() * sizeof(dfi::LineJob), hipMemcpyHostToDevice, st));
      if (!lcg[c].empty())
        HIP_TRY(hipMemcpyAsync(dcg, lcg[c].data(), lcg[c].size() * sizeof(dfi::LineJob), hipMemcpyHostToDevice, st));
      G.res[c] = dres;
      G.cg[c] = dcg;
      gp += lbytes[c] + lcgbytes[c];
    }
    auto* drr = reinterpret_cast<dfi::ReduceJob*>(gp);
    auto* drc = reinterpret_cast<dfi::ReduceJob*>(gp + rrbytes);
    if (!rres.empty())
      HIP_TRY(hipMemcpyAsync(drr, rres.data(), rres.size() * sizeof(dfi::ReduceJob), hipMemcpyHostToDevice, st));
    if (!rcg.empty())
      HIP_TRY(hipMemcpyAsync(drc, rcg.data(), rcg.size() * sizeof(dfi::ReduceJob), hipMemcpyHostToDevice, st));
    G.rres = drr;
    G.rcg = drc;
    auto* dgj = reinterpret_cast<dfi::GramJob*>(gp + rrbytes + rcbytes);
    if (!gjobs.empty())
      HIP_TRY(hipMemcpyAsync(dgj, gjobs.data(), gjobs.size() * sizeof(dfi::GramJob), hipMemcpyHostToDevice, st));
    G.gram = dgj;
  }
  HIP_TRY(hipStreamSynchronize(st));   // the host tables go out of scope; the graph reads the device copies

  // the run: replay the captured graph if every argument and buffer is unchanged
  std::vector<uint64_t> key;
  auto put = [&](const void* pp, size_t nbytes) {
    const auto* c = static_cast<const unsigned char*>(pp);
    for (size_t i = 0; i < nbytes; i += 8) {
      uint64_t w = 0;
      std::memcpy(&w, c + i, std::min<size_t>(8, nbytes - i));
      key.push_back(w);
    }
  };
  put(&np, sizeof(np));
  put(S, sizeof(void*) * (size_t)np);
  put(n, sizeof(int64_t) * (size_t)np);
  put(m, sizeof(int64_t) * (size_t)np);
  put(lds, sizeof(int64_t) * (size_t)np);
  put(v, sizeof(void*) * (size_t)np);
  put(lambda, sizeof(double) * (size_t)np);
  put(x, sizeof(void*) * (size_t)np);
  put(&o, sizeof(o));
  put(&ctx->ws, sizeof(void*));
  put(&ctx->tbuf, sizeof(void*));
  // the layout moves with the Gram plans (a tuning change alters a problem's partial-tile bytes
  // and with them every later offset), so the plans and the layout size are part of the key
  put(&U.bytes, sizeof(U.bytes));
  for (int32_t p = 0; p < np; ++p) {
    const dfi::GramPlan& g = U.gp[(size_t)p];
    const int64_t pk[4] = {g.nslice, g.kslice, g.ldh, (int64_t)g.part_bytes};
    put(pk, sizeof(pk));
  }
  bool ran = false;
  if (ctx->graphs) {
    if (!ctx->uneven_exec || ctx->uneven_key != key) {
      drop_graph(ctx);
      if (!ctx->cap_stream && hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        ctx->cap_stream = nullptr;
      }
      if (ctx->cap_stream) {
        hipGraph_t graph = nullptr;
        bool ok = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        dfisher_status se = DFISHER_OK;
        if (ok)
          se = uneven_enqueue(ctx, np, S, n, m, lds, v, lambda, x, o, U, order, sw, nactive, d_fj, d_tf, d_tb, d_tr,
                              d_seg, d_cap, tol, autos, jpos, G, ctx->cap_stream);
        if (ok) ok = hipStreamEndCapture(ctx->cap_stream, &graph) == hipSuccess && graph != nullptr;
        if (ok && se == DFISHER_OK) {
          hipGraphExec_t ex = nullptr;
          if (hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0) == hipSuccess) {
            ctx->uneven_exec = ex;
            ctx->uneven_key = key;
          }
        }
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();   // a failed capture leaves the eager path below
      }
    }
    if (ctx->uneven_exec) {
      HIP_TRY(hipGraphLaunch(ctx->uneven_exec, st));
      ran = true;
    }
  }
  if (!ran)
    DF_TRY(uneven_enqueue(ctx, np, S, n, m, lds, v, lambda, x, o, U, order, sw, nactive, d_fj, d_tf, d_tb, d_tr, d_seg,
                          d_cap, tol, autos, jpos, G, st));
  std::vector<int64_t> hinfo((size_t)np);
  std::vector<double> hmax((size_t)np, 0.0), hres((size_t)(2 * np), -1.0), hrho((size_t)np, -1.0);
  std::vector<int> hdone((size_t)np, 0), hmet((size_t)np, 0);
  HIP_TRY(hipMemcpyAsync(hinfo.data(), U.info, (size_t)np * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  if (max_sw > 0) {
    HIP_TRY(hipMemcpyAsync(hrho.data(), U.resid, (size_t)np * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hdone.data(), U.done, (size_t)np * sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hmet.data(), U.met, (size_t)np * sizeof(int), hipMemcpyDeviceToHost, st));
  }
  if (o.shift_policy == DFISHER_SHIFT_ALWAYS)
    HIP_TRY(hipMemcpyAsync(hmax.data(), U.dmax, (size_t)np * sizeof(double), hipMemcpyDeviceToHost, st));
  if (o.final_resid)
    HIP_TRY(hipMemcpyAsync(hres.data(), U.res, (size_t)(2 * np) * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  dfisher_status worst = DFISHER_OK;
  bool unmet = false;
  for (int32_t p = 0; p < np; ++p) {
    dfisher_info inf{};
    const size_t j = (size_t)jpos[(size_t)p];
    inf.resid = tol > 0.0 && sw[(size_t)p] > 0 ? hrho[j] : -1.0;
    inf.potrf_info = hinfo[(size_t)p];
    inf.attempts = 1;
    inf.sweeps_done = sw[(size_t)p] > 0 ? hdone[j] : 0;
    if (tol > 0.0 && sw[(size_t)p] > 0 && !hmet[j] && inf.potrf_info == 0) unmet = true;
    inf.w_resid = -1.0;
    if (o.final_resid) {
      const double bb = hres[(size_t)(2 * p)], rr = hres[(size_t)(2 * p + 1)];
      inf.w_resid = bb > 0.0 ? std::sqrt(rr / bb) : (rr > 0.0 ? INFINITY : 0.0);
    }
    if (o.shift_policy == DFISHER_SHIFT_ALWAYS)
      inf.shift = 2.0 * std::sqrt((double)n[p]) * gram_unit(o.gram_prec, m[p]) * hmax[(size_t)p];
    if (inf.potrf_info != 0 && o.shift_policy != DFISHER_SHIFT_NONE) {
      // solve this problem again on its own with the escalating shift (uses the workspace anew)
      dfisher_info again{};
      const dfisher_status s2 = dfisher_solve(ctx, S[p], n[p], m[p], lds[p], v[p], lambda[p], x[p], &o, st, &again);
      again.attempts += 1;
      inf = again;
      if (s2 != DFISHER_OK && s2 != DFISHER_E_NOT_SPD) return s2;
    }
    if (inf.potrf_info != 0) worst = DFISHER_E_NOT_SPD;
    if (infos) infos[p] = inf;
  }
  if (worst != DFISHER_OK) return fail(worst, "at least one problem failed to factor (its x is not meaningful)");
  if (unmet)
    return fail(DFISHER_E_NOT_CONVERGED, "at least one problem's measured residual missed tol %.3g at its sweep cap", tol);
  return DFISHER_OK;
}

// The per-lambda records of an asynchronous batched call, written on the device after its
// factorisations: status, the up-front shift scale0 * max_i G_ii (dmax from diag_max, read only
// when scale0 != 0), one attempt, the fixed sweep count, nothing measured.
__global__ void batch_infos_kernel(dfisher_info* __restrict__ out, int64_t nlam, const int64_t* __restrict__ info,
                                   double scale0, const double* __restrict__ dmax, int32_t sweeps) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nlam) return;
  dfisher_info r;
  r.potrf_info = info[l];
  r.shift = scale0 != 0.0 ? scale0 * dmax[0] : 0.0;
  r.attempts = 1;
  r.sweeps_done = sweeps;
  r.resid = -1.0;
  r.w_resid = -1.0;
  out[l] = r;
}

hipError_t write_batch_infos(dfisher_info* out, int64_t nlam, const int64_t* info, double scale0, const double* dmax,
                             int32_t sweeps, hipStream_t st) {
  hipLaunchKernelGGL(batch_infos_kernel, dim3((unsigned)((nlam + 255) / 256)), dim3(256), 0, st, out, nlam, info,
                     scale0, dmax, sweeps);
  return hipGetLastError();
}

// Per-device set-up, called with the device current: the device address of the no-alloc scratch.
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // per device; null until looked up

dfisher_status init_kernels() {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (g_scratch_ptr[(size_t)dev]) return DFISHER_OK;
  void* ptr = nullptr;
  HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return fail(DFISHER_E_DEVICE, "no device address for the no-alloc scratch on device %d", dev);
  g_scratch_ptr[(size_t)dev] = ptr;
  return DFISHER_OK;
}

void* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return dev >= 0 && (size_t)dev < g_scratch_ptr.size() ? g_scratch_ptr[(size_t)dev] : nullptr;
}

}  // namespace

extern "C" {

const char* dfisher_status_string(dfisher_status s) {
  switch (s) {
    case DFISHER_OK: return "ok";
    case DFISHER_E_INVALID_ARG: return "invalid argument";
    case DFISHER_E_NOT_SPD: return "matrix not positive definite";
    case DFISHER_E_NO_MEMORY: return "out of device memory";
    case DFISHER_E_DEVICE: return "device or HIP runtime error";
    case DFISHER_E_UNSUPPORTED: return "unsupported request";
    case DFISHER_E_NOT_CONVERGED: return "refinement tolerance not met";
  }
  return "unknown status";
}

const char* dfisher_last_error(void) { return g_last_error.c_str(); }

dfisher_status dfisher_ctx_create(int device, dfisher_ctx** out) {
  if (!out) return fail(DFISHER_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (device < 0) return fail(DFISHER_E_INVALID_ARG, "device = %d < 0", device);
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0) {
    (void)hipGetLastError();
    return fail(DFISHER_E_DEVICE, "no HIP device available (%s)", hipGetErrorString(e));
  }
  if (device >= count) return fail(DFISHER_E_DEVICE, "device %d does not exist (%d present)", device, count);
  DeviceGuard g(device);
  dfisher_ctx* c = new dfisher_ctx();
  c->device = device;
  void* dstat = nullptr;
  if (hipMalloc(&dstat, 256) != hipSuccess || hipHostMalloc((void**)&c->h_status, 64, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->h_scalar, 64, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    if (dstat) (void)hipFree(dstat);
    if (c->h_status) (void)hipHostFree(c->h_status);
    if (c->h_scalar) (void)hipHostFree(c->h_scalar);
    delete c;
    return fail(DFISHER_E_NO_MEMORY, "context allocation failed");
  }
  c->d_info = reinterpret_cast<int64_t*>(dstat);
  c->d_flag = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(dstat) + 64);
  c->d_scalar = reinterpret_cast<double*>(reinterpret_cast<char*>(dstat) + 128);
  for (int i = 0; i < NEV; ++i) {
    if (hipEventCreate(&c->ev[i]) != hipSuccess) {
      (void)hipGetLastError();
      c->ev[i] = nullptr;
    }
  }
  dfisher_status si = init_kernels();
  if (si != DFISHER_OK) {
    (void)hipFree(dstat);
    (void)hipHostFree(c->h_status);
    (void)hipHostFree(c->h_scalar);
    delete c;
    return si;
  }
  *out = c;
  return DFISHER_OK;
}

dfisher_status dfisher_ctx_destroy(dfisher_ctx* ctx) {
  if (!ctx) return DFISHER_OK;
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  drop_graph(ctx);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->tbuf) (void)hipFree(ctx->tbuf);
  if (ctx->ws) (void)hipFree(ctx->ws);
  for (int i = 0; i < NEV; ++i)
    if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
  if (ctx->d_info) (void)hipFree(ctx->d_info);
  if (ctx->h_status) (void)hipHostFree(ctx->h_status);
  if (ctx->h_scalar) (void)hipHostFree(ctx->h_scalar);
  delete ctx;
  return DFISHER_OK;
}

dfisher_status dfisher_ctx_enable_timing(dfisher_ctx* ctx, int32_t enable) {
  DF_TRY(check_ctx(ctx));
  for (int i = 0; i < NEV; ++i)
    if (!ctx->ev[i]) return fail(DFISHER_E_DEVICE, "timing events unavailable");
  ctx->timing = enable != 0;
  return DFISHER_OK;
}

dfisher_status dfisher_ctx_last_timing(dfisher_ctx* ctx, dfisher_timing* out) {
  DF_TRY(check_ctx(ctx));
  if (!out) return fail(DFISHER_E_INVALID_ARG, "out is NULL");
  DeviceGuard g(ctx->device);
  double ms[NEV - 1] = {};
  int first = -1, last = -1;
  for (int i = 0; i < NEV; ++i) {
    if (!ctx->ev_used[i]) continue;
    HIP_TRY(hipEventSynchronize(ctx->ev[i]));
    if (first < 0) first = i;
    last = i;
  }
  // a stage's time runs from its start event to the next recorded event
  for (int i = 0; i + 1 < NEV; ++i) {
    if (!ctx->ev_used[i]) continue;
    int j = i + 1;
    while (j < NEV && !ctx->ev_used[j]) ++j;
    if (j >= NEV) break;
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev[i], ctx->ev[j]));
    ms[i] = t;
  }
  out->rowpass_ms = ms[0];
  out->gram_ms = ms[1];
  out->gram_reduce_ms = ms[2];
  out->potrf_ms = ms[3];
  out->trsv_ms = ms[4];
  out->refine_ms = ms[5];
  out->apply_ms = ms[6];
  out->total_ms = 0.0;
  if (first >= 0 && last > first) {
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev[first], ctx->ev[last]));
    out->total_ms = t;
  }
  return DFISHER_OK;
}

dfisher_status dfisher_gram(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds, int32_t prec,
                            double lambda, double* W, void* stream) {
  DF_TRY(check_ctx(ctx));
  DF_TRY(check_S(S, n, m, lds));
  if (!W) return fail(DFISHER_E_INVALID_ARG, "W is NULL");
  if (prec != DFISHER_GRAM_FP32 && prec != DFISHER_GRAM_BF16X3 && prec != DFISHER_GRAM_MXFP8)
    return fail(DFISHER_E_INVALID_ARG, "unknown gram precision %d", prec);
  if (!(std::isfinite(lambda) && lambda >= 0.0)) return fail(DFISHER_E_INVALID_ARG, "lambda must be finite and >= 0");
  DF_TRY(check_prec_layout(prec, S, lds));
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  if (ctx->autotune) DF_TRY(tune_if_new(ctx, S, n, m, lds, prec, st));
  const dfi::GramPlan gp = make_gram_plan(ctx, S, n, m, lds, prec);
  const dfi::RowPassPlan rp = dfi::rowpass_plan(n, m, lds);
  const dfi::ColPassPlan cp = dfi::colpass_plan(n, m);
  SolveBufs B = carve(nullptr, n, m, &gp, rp, cp, false, false);
  DF_TRY(ensure_ws(ctx, B.bytes));
  B = carve(static_cast<char*>(ctx->ws), n, m, &gp, rp, cp, false, false);
  StageClock clk(ctx, st);
  DF_TRY(gram_stage(S, nullptr, gp, rp, B, lambda, W, 1, st, &clk));
  clk.mark(3);
  return DFISHER_OK;
}

dfisher_status dfisher_quantize_mxfp8(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds,
                                      uint8_t* codes, int64_t ldq, uint8_t* scales, void* stream) {
  DF_TRY(check_ctx(ctx));
  DF_TRY(check_S(S, n, m, lds));
  if (!codes || !scales) return fail(DFISHER_E_INVALID_ARG, "codes or scales is NULL");
  if (ldq < m || ldq % 64 != 0) return fail(DFISHER_E_INVALID_ARG, "ldq must be a multiple of 64 and >= m");
  DF_TRY(check_prec_layout(DFISHER_GRAM_MXFP8, S, lds));
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  const dfi::RowPassPlan rp = dfi::rowpass_plan(n, m, lds);
  DF_TRY(ensure_ws(ctx, align_up(rp.part_bytes)));
  HIP_TRY(dfi::rowpass_launch(rp, S, nullptr, nullptr, false, true, static_cast<double*>(ctx->ws), st, codes, scales,
                              ldq));
  return DFISHER_OK;
}

dfisher_status dfisher_potrf(dfisher_ctx* ctx, double* W, int64_t n, int64_t* info, void* stream) {
  DF_TRY(check_ctx(ctx));
  if (!W) return fail(DFISHER_E_INVALID_ARG, "W is NULL");
  if (!info) return fail(DFISHER_E_INVALID_ARG, "info is NULL");
  if (n < 1) return fail(DFISHER_E_INVALID_ARG, "n = %lld < 1", (long long)n);
  *info = 0;
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  DF_TRY(ensure_ws(ctx, dfi::POTRF_DKK_BYTES));
  HIP_TRY(dfi::potrf_launch(W, n, ctx->d_info, ctx->d_flag, static_cast<double*>(ctx->ws), st));
  HIP_TRY(hipMemcpyAsync(ctx->h_status, ctx->d_info, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *info = ctx->h_status[0];
  if (*info != 0) return fail(DFISHER_E_NOT_SPD, "Cholesky failed at pivot %lld", (long long)*info);
  HIP_TRY(dfi::zero_upper(W, n, st));
  return DFISHER_OK;
}

dfisher_status dfisher_gemv(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds, const float* v,
                            double* b, void* stream) {
  DF_TRY(check_ctx(ctx));
  DF_TRY(check_S(S, n, m, lds));
  if (!v || !b) return fail(DFISHER_E_INVALID_ARG, "v or b is NULL");
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  const dfi::RowPassPlan rp = dfi::rowpass_plan(n, m, lds);
  DF_TRY(ensure_ws(ctx, align_up(rp.part_bytes)));
  double* rpart = static_cast<double*>(ctx->ws);
  HIP_TRY(dfi::rowpass_launch(rp, S, v, nullptr, true, false, rpart, st));
  HIP_TRY(dfi::rowpass_reduce(rp, rpart, true, false, b, nullptr, nullptr, nullptr, 0.0, st));
  return DFISHER_OK;
}

dfisher_status dfisher_trsv(dfisher_ctx* ctx, const double* L, int64_t n, int32_t trans, const double* b, double* y,
                            void* stream) {
  DF_TRY(check_ctx(ctx));
  if (!L || !b || !y) return fail(DFISHER_E_INVALID_ARG, "L, b or y is NULL");
  if (n < 1) return fail(DFISHER_E_INVALID_ARG, "n = %lld < 1", (long long)n);
  if (trans != 0 && trans != 1) return fail(DFISHER_E_INVALID_ARG, "trans must be 0 or 1");
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  Carver c;
  double* Dinv = c.take<double>(dfi::trsv_dinv_bytes(n) / sizeof(double));
  double* work = c.take<double>((size_t)n);
  DF_TRY(ensure_ws(ctx, c.off));
  c = Carver{};
  c.base = static_cast<char*>(ctx->ws);
  Dinv = c.take<double>(dfi::trsv_dinv_bytes(n) / sizeof(double));
  work = c.take<double>((size_t)n);
  HIP_TRY(dfi::trsv_diag_inv(L, n, Dinv, st));
  HIP_TRY(dfi::trsv_launch(L, Dinv, n, trans, b, y, work, st));
  return DFISHER_OK;
}

dfisher_status dfisher_apply(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds, const float* v,
                             const double* y, double lambda, void* x, int32_t x_fp64, void* stream) {
  DF_TRY(check_ctx(ctx));
  DF_TRY(check_S(S, n, m, lds));
  if (!v || !y || !x) return fail(DFISHER_E_INVALID_ARG, "v, y or x is NULL");
  if (!finite_pos(lambda)) return fail(DFISHER_E_INVALID_ARG, "lambda must be finite and > 0");
  if (x_fp64 != 0 && x_fp64 != 1) return fail(DFISHER_E_INVALID_ARG, "x_fp64 must be 0 or 1");
  DeviceGuard g(ctx->device);
  const dfi::ColPassPlan cp = dfi::colpass_plan(n, m);
  DF_TRY(ensure_ws(ctx, align_up(cp.part_bytes + 8)));
  HIP_TRY(dfi::colpass_launch(cp, S, n, m, lds, y, v, lambda, x, x_fp64 ? 1 : 0, static_cast<double*>(ctx->ws),
                              as_stream(stream)));
  return DFISHER_OK;
}

dfisher_status dfisher_factor_create(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds,
                                     double lambda, const dfisher_options* opt, void* stream, dfisher_factor** out,
                                     dfisher_info* info) {
  DF_TRY(check_ctx(ctx));
  if (!out) return fail(DFISHER_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  DF_TRY(check_S(S, n, m, lds));
  if (!finite_pos(lambda)) return fail(DFISHER_E_INVALID_ARG, "lambda must be finite and > 0");
  dfisher_options o;
  DF_TRY(check_opt(opt, &o));
  DF_TRY(check_no_tol(o));
  DF_TRY(check_no_final(o));
  DF_TRY(check_prec_layout(o.gram_prec, S, lds));
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  if (ctx->autotune) DF_TRY(tune_if_new(ctx, S, n, m, lds, o.gram_prec, st));
  const dfi::GramPlan gp = make_gram_plan(ctx, S, n, m, lds, o.gram_prec);
  const dfi::RowPassPlan rp = dfi::rowpass_plan(n, m, lds);
  const dfi::ColPassPlan cp = dfi::colpass_plan(n, m);
  SolveBufs B = carve(nullptr, n, m, &gp, rp, cp, false, false);
  DF_TRY(ensure_ws(ctx, B.bytes));
  B = carve(static_cast<char*>(ctx->ws), n, m, &gp, rp, cp, false, false);
  dfisher_factor* f = new dfisher_factor();
  f->ctx = ctx;
  f->S = S;
  f->n = n;
  f->m = m;
  f->lds = lds;
  f->lambda = lambda;
  f->opt = o;
  if (hipMalloc(&f->L, (size_t)(n * n) * sizeof(double)) != hipSuccess ||
      hipMalloc(&f->Dinv, dfi::trsv_dinv_bytes(n)) != hipSuccess) {
    (void)hipGetLastError();
    if (f->L) (void)hipFree(f->L);
    delete f;
    return fail(DFISHER_E_NO_MEMORY, "factor allocation failed");
  }
  auto cleanup = [&](dfisher_status s) {
    (void)hipFree(f->L);
    (void)hipFree(f->Dinv);
    delete f;
    return s;
  };
  {
    const dfisher_status sg = gram_stage(S, nullptr, gp, rp, B, lambda, B.W, 0, st, nullptr, is_centered(o));
    if (sg != DFISHER_OK) return cleanup(sg);
  }
  dfisher_info inf{};
  inf.resid = -1.0;
  inf.w_resid = -1.0;
  dfisher_status s = factor_with_policy(ctx, B.W, f->L, B.dkk, n, o.shift_policy, gram_unit(o.gram_prec, m), st, &inf.shift, &inf.potrf_info,
                                       &inf.attempts);
  if (o.sweeps == DFISHER_SWEEPS_AUTO) {   // resolved once, with the factored shift known
    const double wmax = (o.shift_policy != DFISHER_SHIFT_NONE) ? ctx->h_scalar[0] : 0.0;
    f->opt.sweeps = auto_sweeps(o.gram_prec, n, m, (inf.shift > 0.0 && wmax > 0.0) ? inf.shift / wmax : 0.0,
                                is_centered(o));
  }
  inf.sweeps_done = f->opt.sweeps;
  if (info) *info = inf;
  if (s != DFISHER_OK) return cleanup(s);
  if (dfi::trsv_diag_inv(f->L, n, f->Dinv, st) != hipSuccess)
    return cleanup(fail(DFISHER_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(hipGetLastError())));
  f->shift = inf.shift;
  *out = f;
  return DFISHER_OK;
}

dfisher_status dfisher_factor_solve(dfisher_factor* f, const float* V, int64_t nrhs, int64_t ldv, void* X, int64_t ldx,
                                    void* stream, dfisher_info* info) {
  if (!f) return fail(DFISHER_E_INVALID_ARG, "factor is NULL");
  if (!V || !X) return fail(DFISHER_E_INVALID_ARG, "V or X is NULL");
  if (nrhs < 1) return fail(DFISHER_E_INVALID_ARG, "nrhs = %lld < 1", (long long)nrhs);
  if (ldv < f->m || ldx < f->m) return fail(DFISHER_E_INVALID_ARG, "ldv/ldx < m");
  dfisher_ctx* ctx = f->ctx;
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  const int64_t n = f->n, m = f->m;
  if (nrhs > 65535) return fail(DFISHER_E_UNSUPPORTED, "nrhs = %lld > 65535", (long long)nrhs);
  const dfi::RowMultiPlan rm = dfi::rowmulti_plan(n, m, f->lds);
  Carver c;
  MultiBufs mb = carve_multi(c, n, m, nrhs, nrhs, rm, f->opt.sweeps > 0);
  DF_TRY(ensure_ws(ctx, c.off));
  c = Carver{};
  c.base = static_cast<char*>(ctx->ws);
  mb = carve_multi(c, n, m, nrhs, nrhs, rm, f->opt.sweeps > 0);
  const double lam = f->lambda;
  DF_TRY(multi_solve(f->S, n, m, f->lds, 1, f->L, f->Dinv, &lam, V, nrhs, ldv, X, ldx, f->opt.x_fp64, f->opt.sweeps, rm,
                     mb, st));
  if (info) {
    info->potrf_info = 0;
    info->shift = f->shift;
    info->attempts = 0;
    info->sweeps_done = f->opt.sweeps;
    info->resid = -1.0;
    info->w_resid = -1.0;
  }
  return DFISHER_OK;
}

dfisher_status dfisher_factor_solve_noalloc(const dfisher_factor* f, const float* v, void* x, void* stream,
                                            dfisher_info* info) {
  if (!f) return fail(DFISHER_E_INVALID_ARG, "factor is NULL");
  if (!v || !x) return fail(DFISHER_E_INVALID_ARG, "v or x is NULL");
  dfisher_ctx* ctx = f->ctx;
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  const int64_t n = f->n, m = f->m, lds = f->lds;
  const int sweeps = f->opt.sweeps;
  const dfi::RowPassPlan rp = dfi::rowpass_plan(n, m, lds);
  const dfi::ColPassPlan cp = dfi::colpass_plan(n, m);
  const dfi::RefinePassPlan fp = dfi::refine_pass_plan(n, m, lds, f->S, false);   // small workspace
  if (sweeps > 0 && !fp.usable)
    return fail(DFISHER_E_UNSUPPORTED, "the no-alloc solve refines with the one-read product only: it needs "
                "n <= 4096, m >= 16 and 16-byte aligned rows of S (n = %lld, lds = %lld)", (long long)n,
                (long long)lds);
  // everything solve_y and the two passes touch, carved from the device's scratch
  auto lay = [&](char* base, SolveBufs& B) -> size_t {
    Carver c;
    c.base = base;
    B = SolveBufs{};
    B.rpart = c.take<double>(std::max(rp.part_bytes, fp.part_bytes) / sizeof(double) + 1);
    B.cpart = c.take<double>(cp.part_bytes / sizeof(double) + 1);
    B.b = c.take<double>((size_t)n);
    B.z = c.take<double>((size_t)n);
    B.y = c.take<double>((size_t)n);
    B.r = c.take<double>((size_t)n);
    B.zc = c.take<double>((size_t)n);
    B.p = c.take<double>((size_t)n);
    B.nq = c.take<double>((size_t)n);
    B.zero = c.take<double>((size_t)n);
    B.tw = c.take<double>((size_t)n);
    return c.off;
  };
  SolveBufs B;
  const size_t need = lay(nullptr, B);
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(DFISHER_E_UNSUPPORTED, "n = %lld, m = %lld needs %zu bytes of scratch; the no-alloc solve holds %zu",
                (long long)n, (long long)m, need, NOALLOC_SCRATCH_BYTES);
  char* base = static_cast<char*>(scratch_ptr(ctx->device));
  if (!base) return fail(DFISHER_E_DEVICE, "no-alloc scratch of device %d was not set up", ctx->device);
  lay(base, B);
  // b = S v, y = W^-1 b through the factor (+ sweeps), x = (v - S^T y) / lambda
  HIP_TRY(dfi::rowpass_launch(rp, f->S, v, nullptr, true, false, B.rpart, st));
  HIP_TRY(dfi::rowpass_reduce(rp, B.rpart, true, false, B.b, nullptr, nullptr, nullptr, 0.0, st));
  int done = 0;
  DF_TRY(solve_y(f->S, n, m, lds, f->lambda, f->L, f->Dinv, B, rp, cp, sweeps, st, nullptr, &fp, ctx, 0.0, &done));
  HIP_TRY(dfi::colpass_launch(cp, f->S, n, m, lds, B.y, v, f->lambda, x, f->opt.x_fp64, B.cpart, st));
  if (info) {
    info->potrf_info = 0;
    info->shift = f->shift;
    info->attempts = 0;
    info->sweeps_done = done;
    info->resid = -1.0;
    info->w_resid = -1.0;
  }
  return DFISHER_OK;
}

dfisher_status dfisher_factor_copy_L(const dfisher_factor* f, double* L, void* stream) {
  if (!f || !L) return fail(DFISHER_E_INVALID_ARG, "factor or L is NULL");
  DeviceGuard g(f->ctx->device);
  HIP_TRY(hipMemcpyAsync(L, f->L, (size_t)(f->n * f->n) * sizeof(double), hipMemcpyDeviceToDevice,
                         as_stream(stream)));
  return DFISHER_OK;
}

dfisher_status dfisher_factor_destroy(dfisher_factor* f) {
  if (!f) return DFISHER_OK;
  DeviceGuard g(f->ctx->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(f->L);
  (void)hipFree(f->Dinv);
  delete f;
  return DFISHER_OK;
}

dfisher_status dfisher_solve(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds, const float* v,
                             double lambda, void* x, const dfisher_options* opt, void* stream, dfisher_info* info) {
  DF_TRY(check_ctx(ctx));
  DF_TRY(check_S(S, n, m, lds));
  if (!v || !x) return fail(DFISHER_E_INVALID_ARG, "v or x is NULL");
  if (!finite_pos(lambda)) return fail(DFISHER_E_INVALID_ARG, "lambda must be finite and > 0");
  dfisher_options o;
  DF_TRY(check_opt(opt, &o));
  DF_TRY(check_prec_layout(o.gram_prec, S, lds));
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  if (ctx->autotune) DF_TRY(tune_if_new(ctx, S, n, m, lds, o.gram_prec, st));
  const dfi::GramPlan gp = make_gram_plan(ctx, S, n, m, lds, o.gram_prec);
  const dfi::RowPassPlan rp = dfi::rowpass_plan(n, m, lds);
  const dfi::ColPassPlan cp = dfi::colpass_plan(n, m);
  const dfi::RefinePassPlan fp = dfi::refine_pass_plan(n, m, lds, S);
  const bool need_t = (o.sweeps != 0 || o.final_resid) && !fp.usable;
  // the final step may take the last correction's image through the FP8 codes (apply8.hip): the
  // codes exist, the passes can carry S^T y, there is a correction, and the caller allows it
  const bool final8 = o.gram_prec == DFISHER_GRAM_MXFP8 && fp.usable && fp.line && o.sweeps != 0 &&
                      !o.final_resid && (o.flags & DFISHER_EXACT_APPLY) == 0;
  SolveBufs B = carve(nullptr, n, m, &gp, rp, cp, true, need_t, &fp, final8, is_centered(o));
  DF_TRY(ensure_ws(ctx, B.bytes));
  B = carve(static_cast<char*>(ctx->ws), n, m, &gp, rp, cp, true, need_t, &fp, final8, is_centered(o));
  StageClock clk(ctx, st);
  // one pass over S (b = S v, the exact diagonal |s_i|^2, the FP8 codes if used), then step 1
  DF_TRY(gram_stage(S, v, gp, rp, B, lambda, B.W, 0, st, &clk, is_centered(o), B.cs8 ? B.use8 + 1 : nullptr));
  // step 2 (with the shift policy)
  clk.mark(3);
  dfisher_info inf{};
  inf.resid = -1.0;
  // steps 3-4 inlined: y = W^-1 S v (+ refinement), x = (v - S^T y) / lambda. The first
  // application of L^-1 and L^-T is enqueued right behind the first factorisation attempt, before
  // the host waits for its status, and repeated only if that attempt was not the final one.
  auto first_solve = [&]() -> dfisher_status {
    clk.mark(4);
    HIP_TRY(dfi::trsv_diag_inv(B.L, n, B.Dinv, st));
    HIP_TRY(dfi::trsv_launch(B.L, B.Dinv, n, 0, B.b, B.z, B.tw, st));
    HIP_TRY(dfi::trsv_launch(B.L, B.Dinv, n, 1, B.z, B.y, B.tw, st));
    clk.mark(5);
    return DFISHER_OK;
  };
  bool spec_ok = false;
  DF_TRY(factor_with_policy(ctx, B.W, B.L, B.dkk, n, o.shift_policy, gram_unit(o.gram_prec, m), st, &inf.shift,
                            &inf.potrf_info, &inf.attempts, first_solve, &spec_ok));
  if (!spec_ok) DF_TRY(first_solve());
  // DFISHER_SWEEPS_AUTO: measured, predictive stop at tol (default 1e-7), at most MAX_SWEEPS
  const bool autos = o.sweeps == DFISHER_SWEEPS_AUTO;
  const int sweeps = autos ? MAX_SWEEPS : o.sweeps;
  const double tol = autos && !(o.tol > 0.0) ? AUTO_TOL : o.tol;
  int done = 0;
  double resid = -1.0;
  bool met = false;
  const Final8 f8{B.T8, B.U8, B.cs8, B.a8, m};
  DF_TRY(solve_y(S, n, m, lds, lambda, B.L, B.Dinv, B, rp, cp, sweeps, st, &clk, &fp, ctx, tol, &done, &resid,
                 false, autos ? auto_floor(o) : 0.0, &met, final8 ? &f8 : nullptr));
  inf.w_resid = -1.0;
  if (o.final_resid) DF_TRY(final_residual(ctx, S, n, m, lds, lambda, B, rp, cp, fp, st, &inf.w_resid));
  if (final8) {
    // x = (v - T - S^T zc) / lambda with S^T zc through the codes when the device finds that
    // accurate enough; otherwise y += zc there and the exact column pass runs (one of the two
    // kernels returns at once)
    // (the all-ones component is split off only where the projection was applied: a declaration
    // the device rejected leaves the call bitwise that of the call without it)
    HIP_TRY(dfi::final_decide(n, B.y, B.zc, B.b, B.d, lambda, B.cs8 ? B.use8 + 1 : nullptr, FINAL8_EST_MAX, B.zf8,
                              B.a8 + 1, B.use8, st));
    HIP_TRY(dfi::fp8_apply(B.q8, B.sc8, B.ldq, n, m, B.zf8, B.T8, B.cs8, B.a8 + 1, v, lambda, x, o.x_fp64, B.use8, st));
    HIP_TRY(dfi::colpass_launch(cp, S, n, m, lds, B.y, v, lambda, x, o.x_fp64, B.cpart, st, B.use8));
  } else {
    HIP_TRY(dfi::colpass_launch(cp, S, n, m, lds, B.y, v, lambda, x, o.x_fp64, B.cpart, st));
  }
  clk.mark(7);
  inf.sweeps_done = done;
  inf.resid = resid;
  if (info) *info = inf;
  if (tol > 0.0 && !met)
    return fail(DFISHER_E_NOT_CONVERGED, "relative residual %.3g above tol %.3g after %d sweep(s)", resid, tol, done);
  return DFISHER_OK;
}

// Appendix B: v = S^T f. By the push-through identity x = S^T (S S^T + lambda I)^-1 f, so the solve
// runs Algorithm 1 with b = f: no pass for S v and no subtraction v - S^T y (whose cancellation
// costs accuracy when v lies in the row space of S). Refinement sweeps correct y against
// W y = f with the exact operator, as in dfisher_solve.
dfisher_status dfisher_solve_rowspace(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds,
                                      const double* f, double lambda, void* x, const dfisher_options* opt,
                                      void* stream, dfisher_info* info) {
  DF_TRY(check_ctx(ctx));
  DF_TRY(check_S(S, n, m, lds));
  if (!f || !x) return fail(DFISHER_E_INVALID_ARG, "f or x is NULL");
  if (!finite_pos(lambda)) return fail(DFISHER_E_INVALID_ARG, "lambda must be finite and > 0");
  dfisher_options o;
  DF_TRY(check_opt(opt, &o));
  DF_TRY(check_prec_layout(o.gram_prec, S, lds));
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  if (ctx->autotune) DF_TRY(tune_if_new(ctx, S, n, m, lds, o.gram_prec, st));
  const dfi::GramPlan gp = make_gram_plan(ctx, S, n, m, lds, o.gram_prec);
  const dfi::RowPassPlan rp = dfi::rowpass_plan(n, m, lds);
  const dfi::ColPassPlan cp = dfi::colpass_plan(n, m);
  const dfi::RefinePassPlan fp = dfi::refine_pass_plan(n, m, lds, S);
  const bool need_t = (o.sweeps != 0 || o.final_resid) && !fp.usable;
  SolveBufs B = carve(nullptr, n, m, &gp, rp, cp, true, need_t, &fp);
  DF_TRY(ensure_ws(ctx, B.bytes));
  B = carve(static_cast<char*>(ctx->ws), n, m, &gp, rp, cp, true, need_t, &fp);
  StageClock clk(ctx, st);
  // one pass over S for the exact diagonal (and the FP8 codes), then step 1; b = f
  DF_TRY(gram_stage(S, nullptr, gp, rp, B, lambda, B.W, 0, st, &clk, is_centered(o)));
  HIP_TRY(hipMemcpyAsync(B.b, f, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
  clk.mark(3);
  dfisher_info inf{};
  inf.resid = -1.0;
  auto first_solve = [&]() -> dfisher_status {
    clk.mark(4);
    HIP_TRY(dfi::trsv_diag_inv(B.L, n, B.Dinv, st));
    HIP_TRY(dfi::trsv_launch(B.L, B.Dinv, n, 0, B.b, B.z, B.tw, st));
    HIP_TRY(dfi::trsv_launch(B.L, B.Dinv, n, 1, B.z, B.y, B.tw, st));
    clk.mark(5);
    return DFISHER_OK;
  };
  bool spec_ok = false;
  DF_TRY(factor_with_policy(ctx, B.W, B.L, B.dkk, n, o.shift_policy, gram_unit(o.gram_prec, m), st, &inf.shift,
                            &inf.potrf_info, &inf.attempts, first_solve, &spec_ok));
  if (!spec_ok) DF_TRY(first_solve());
  const bool autos = o.sweeps == DFISHER_SWEEPS_AUTO;
  const int sweeps = autos ? MAX_SWEEPS : o.sweeps;
  const double tol = autos && !(o.tol > 0.0) ? AUTO_TOL : o.tol;
  int done = 0;
  double resid = -1.0;
  bool met = false;
  DF_TRY(solve_y(S, n, m, lds, lambda, B.L, B.Dinv, B, rp, cp, sweeps, st, &clk, &fp, ctx, tol, &done, &resid,
                 false, autos ? auto_floor(o) : 0.0, &met));
  inf.w_resid = -1.0;
  if (o.final_resid) DF_TRY(final_residual(ctx, S, n, m, lds, lambda, B, rp, cp, fp, st, &inf.w_resid));
  // x = S^T y, rounded once (FP32) or kept in FP64
  HIP_TRY(dfi::colpass_launch(cp, S, n, m, lds, B.y, nullptr, 1.0, x, o.x_fp64 ? 2 : 3, B.cpart, st));
  clk.mark(7);
  inf.sweeps_done = done;
  inf.resid = resid;
  if (info) *info = inf;
  if (tol > 0.0 && !met)
    return fail(DFISHER_E_NOT_CONVERGED, "relative residual %.3g above tol %.3g after %d sweep(s)", resid, tol, done);
  return DFISHER_OK;
}

// Section 3: S = (O - mean over the samples of O) / sqrt(n). Column sums by the column pass (FP64,
// y = 1), then one pass that writes S (or, for a complex O, the stacked Z = [Re S; Im S]).
dfisher_status dfisher_sr_center(dfisher_ctx* ctx, const float* O, int64_t n, int64_t m, int64_t ldo,
                                 int32_t is_complex, float* S, int64_t lds, void* stream) {
  DF_TRY(check_ctx(ctx));
  if (!O || !S) return fail(DFISHER_E_INVALID_ARG, "O or S is NULL");
  if (n < 1 || m < 1) return fail(DFISHER_E_INVALID_ARG, "n = %lld, m = %lld must be >= 1", (long long)n, (long long)m);
  if (ldo < m || lds < m) return fail(DFISHER_E_INVALID_ARG, "ldo or lds < m");
  if (is_complex != 0 && is_complex != 1) return fail(DFISHER_E_INVALID_ARG, "is_complex = %d not 0 or 1", is_complex);
  const size_t obytes = (size_t)((n - 1) * ldo + m) * sizeof(float) * (is_complex ? 2 : 1);
  const int64_t srows = is_complex ? 2 * n : n;
  const size_t sbytes = (size_t)((srows - 1) * lds + m) * sizeof(float);
  if (is_complex) {
    if (reinterpret_cast<uintptr_t>(O) % 8 != 0) return fail(DFISHER_E_INVALID_ARG, "complex O must be 8-byte aligned");
    if (overlaps(O, obytes, S, sbytes)) return fail(DFISHER_E_INVALID_ARG, "Z overlaps O (no in-place complex form)");
  } else if (overlaps(O, obytes, S, sbytes) && !(O == S && ldo == lds)) {
    return fail(DFISHER_E_INVALID_ARG, "S overlaps O other than in place (same pointer and stride)");
  }
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  const int64_t mc = is_complex ? 2 * m : m;       // FP32 columns of O as the column pass sees them
  const int64_t ldc = is_complex ? 2 * ldo : ldo;
  const dfi::ColPassPlan cp = dfi::colpass_plan(n, mc);
  auto lay = [&](char* base, double** ones, double** t, double** cpart) -> size_t {
    Carver c;
    c.base = base;
    *ones = c.take<double>((size_t)n);
    *t = c.take<double>((size_t)mc);
    *cpart = c.take<double>(cp.part_bytes / sizeof(double) + 1);
    return c.off;
  };
  double *ones, *t, *cpart;
  DF_TRY(ensure_ws(ctx, lay(nullptr, &ones, &t, &cpart)));
  lay(static_cast<char*>(ctx->ws), &ones, &t, &cpart);
  HIP_TRY(dfi::fill_value(ones, n, 1.0, st));
  HIP_TRY(dfi::colpass_launch(cp, O, n, mc, ldc, ones, nullptr, 1.0, t, 2, cpart, st));
  HIP_TRY(dfi::center_write(O, n, m, ldo, is_complex, t, S, lds, st));
  return DFISHER_OK;
}

// Section 3, complex variant: (S^H S + lambda I) x = v with S = A + iB given in the stacked real form
// Z = [A; B]. It is the real system of E = [[A, -B], [B, A]] (2n x 2m) with v = [Re v; Im v], solved
// by Algorithm 1 on E: the Gram E E^T = [[Wr, -Wi], [Wi, Wr]] + lambda I assembled from Z Z^T,
// its FP64 Cholesky, b = E v, refinement sweeps with the matrix-free E (E^T y) (two vectors per
// pass over Z), x = (v - E^T y) / lambda. E is never formed.
dfisher_status dfisher_solve_complex(dfisher_ctx* ctx, const float* Z, int64_t n, int64_t m, int64_t lds, const float* v,
                                     double lambda, void* x, const dfisher_options* opt, void* stream,
                                     dfisher_info* info) {
  DF_TRY(check_ctx(ctx));
  if (n > 32767) return fail(DFISHER_E_UNSUPPORTED, "n = %lld > 32767 (the real Gram is 2n x 2n)", (long long)n);
  DF_TRY(check_S(Z, n >= 1 ? 2 * n : n, m, lds));
  if (!v || !x) return fail(DFISHER_E_INVALID_ARG, "v or x is NULL");
  if (reinterpret_cast<uintptr_t>(v) % 8 != 0) return fail(DFISHER_E_INVALID_ARG, "complex v must be 8-byte aligned");
  if (!finite_pos(lambda)) return fail(DFISHER_E_INVALID_ARG, "lambda must be finite and > 0");
  dfisher_options o;
  DF_TRY(check_opt(opt, &o));
  DF_TRY(check_prec_layout(o.gram_prec, Z, lds));
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  const int64_t N = 2 * n;
  if (ctx->autotune) DF_TRY(tune_if_new(ctx, Z, N, m, lds, o.gram_prec, st));
  const dfi::GramPlan gp = make_gram_plan(ctx, Z, N, m, lds, o.gram_prec);
  const dfi::RowPassPlan rp = dfi::rowpass_plan(N, m, lds);
  const dfi::ColPassPlan cp = dfi::colpass_plan(N, m);
  const dfi::RowMultiPlan rm = dfi::rowmulti_plan(N, m, lds);
  constexpr int MV = dfi::MULTI_VECS;
  struct Extra {
    double *G, *P, *Q, *U1, *U2, *T, *Yi, *mpart;
    float* vp;
  };
  auto lay = [&](char* base, SolveBufs& B, Extra& X) -> size_t {
    B = carve(base, N, m, &gp, rp, cp, true, false, nullptr);
    Carver c;
    c.base = base;
    c.off = B.bytes;
    X.G = c.take<double>((size_t)(N * N));
    X.P = c.take<double>((size_t)N);
    X.Q = c.take<double>((size_t)N);
    X.U1 = c.take<double>((size_t)N);
    X.U2 = c.take<double>((size_t)N);
    X.T = c.take<double>((size_t)m * MV);
    X.Yi = c.take<double>((size_t)N * MV);
    X.mpart = c.take<double>(rm.part_bytes / sizeof(double) + 1);
    X.vp = c.take<float>((size_t)(2 * m));
    return c.off;
  };
  SolveBufs B;
  Extra X;
  DF_TRY(ensure_ws(ctx, lay(nullptr, B, X)));
  lay(static_cast<char*>(ctx->ws), B, X);
  StageClock clk(ctx, st);
  // Z Z^T (both triangles, exact FP64 diagonal) and the embedded W
  DF_TRY(gram_stage(Z, nullptr, gp, rp, B, 0.0, X.G, 1, st, &clk));
  // centered: the indicators of the A and B halves of Z are null vectors of Z Z^T, and those of
  // the real and imaginary halves of E E^T; projecting Z Z^T makes both exact
  if (is_centered(o)) {
    if (gp.part_bytes < dfi::gram_project_work_bytes(N)) return fail(DFISHER_E_DEVICE, "projection work too small");
    HIP_TRY(dfi::gram_project(X.G, N, 2, 0.0, 1, reinterpret_cast<double*>(B.gpart), X.Yi, st));
  }
  HIP_TRY(dfi::complex_embed(X.G, n, lambda, B.W, st));
  // b = E v = [A vr - B vi; B vr + A vi] from Z vr and Z vi (one pass over Z)
  HIP_TRY(dfi::deinterleave(v, m, X.vp, st));
  {
    dfi::MultiVecs vs{};
    vs.f[0] = X.vp;
    vs.f[1] = X.vp + m;
    dfi::MultiOut mo{};
    mo.b[0] = X.P;
    mo.b[1] = X.Q;
    HIP_TRY(dfi::rowpass_multi_launch(rm, Z, vs, nullptr, 2, X.mpart, st));
    HIP_TRY(dfi::rowpass_multi_reduce(rm, X.mpart, 2, mo, st));
    HIP_TRY(dfi::complex_combine(X.P, X.Q, n, 1.0, nullptr, nullptr, 0.0, B.b, st));
  }
  // E^T u for u = [u1; u2]: t1 = Z^T [u1; u2], t2 = Z^T [u2; -u1], into T columns 0 and 1
  auto et = [&](const double* u) -> dfisher_status {
    HIP_TRY(dfi::complex_colvecs(u, n, X.U1, X.U2, st));
    dfi::MultiCols mc{};
    for (int c = 0; c < MV; ++c) mc.y[c] = c == 1 ? X.U2 : X.U1;
    HIP_TRY(dfi::colpass_multi_launch(Z, N, m, lds, mc, 2, 2, X.T, X.Yi, st));
    return DFISHER_OK;
  };
  // out = rhs - lambda u - E (E^T u)
  const WOp wop = [&](const double* u, const double* rhs, double* out, double*, double*) -> dfisher_status {
    DF_TRY(et(u));
    dfi::MultiVecs none{};
    dfi::MultiOut mo{};
    mo.b[0] = X.P;
    mo.b[1] = X.Q;
    HIP_TRY(dfi::rowpass_multi_launch(rm, Z, none, X.T, 2, X.mpart, st));
    HIP_TRY(dfi::rowpass_multi_reduce(rm, X.mpart, 2, mo, st));
    HIP_TRY(dfi::complex_combine(X.P, X.Q, n, -1.0, rhs, u, lambda, out, st));
    return DFISHER_OK;
  };
  clk.mark(3);
  dfisher_info inf{};
  inf.resid = -1.0;
  DF_TRY(factor_with_policy(ctx, B.W, B.L, B.dkk, N, o.shift_policy, gram_unit(o.gram_prec, m), st, &inf.shift,
                            &inf.potrf_info, &inf.attempts));
  clk.mark(4);
  HIP_TRY(dfi::trsv_diag_inv(B.L, N, B.Dinv, st));
  const bool autos = o.sweeps == DFISHER_SWEEPS_AUTO;
  const int sweeps = autos ? MAX_SWEEPS : o.sweeps;
  const double tol = autos && !(o.tol > 0.0) ? AUTO_TOL : o.tol;
  int done = 0;
  double resid = -1.0;
  bool met = false;
  DF_TRY(solve_y_op(N, B.L, B.Dinv, B, sweeps, st, wop, &clk, ctx, tol, &done, &resid, true,
                    autos ? auto_floor(o) : 0.0, &met));
  inf.w_resid = -1.0;
  if (o.final_resid) {
    DF_TRY(wop(B.y, B.b, B.r, nullptr, nullptr));
    HIP_TRY(dfi::sumsq(B.b, N, ctx->d_scalar + 2, st));
    HIP_TRY(dfi::sumsq(B.r, N, ctx->d_scalar + 3, st));
    HIP_TRY(hipMemcpyAsync(ctx->h_scalar + 2, ctx->d_scalar + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double bb = ctx->h_scalar[2], rr = ctx->h_scalar[3];
    inf.w_resid = bb > 0.0 ? std::sqrt(rr / bb) : (rr > 0.0 ? INFINITY : 0.0);
  }
  // x = (v - E^T y) / lambda, complex interleaved
  DF_TRY(et(B.y));
  HIP_TRY(dfi::complex_apply(v, X.T, m, lambda, x, o.x_fp64, st));
  clk.mark(7);
  inf.sweeps_done = done;
  inf.resid = resid;
  if (info) *info = inf;
  if (tol > 0.0 && !met)
    return fail(DFISHER_E_NOT_CONVERGED, "relative residual %.3g above tol %.3g after %d sweep(s)", resid, tol, done);
  return DFISHER_OK;
}

dfisher_status dfisher_solve_batched(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds,
                                     const double* lambdas, int32_t nlam, const float* V, int32_t nrhs, int64_t ldv,
                                     void* X, int64_t ldx, const dfisher_options* opt, void* stream,
                                     dfisher_info* infos) {
  DF_TRY(check_ctx(ctx));
  DF_TRY(check_S(S, n, m, lds));
  if (!lambdas || !V || !X) return fail(DFISHER_E_INVALID_ARG, "lambdas, V or X is NULL");
  if (nlam < 1 || nrhs < 1) return fail(DFISHER_E_INVALID_ARG, "nlam and nrhs must be >= 1");
  if (ldv < m || ldx < m) return fail(DFISHER_E_INVALID_ARG, "ldv/ldx < m");
  for (int32_t l = 0; l < nlam; ++l)
    if (!finite_pos(lambdas[l])) return fail(DFISHER_E_INVALID_ARG, "lambdas[%d] must be finite and > 0", l);
  if ((int64_t)nlam * nrhs > 65535) return fail(DFISHER_E_UNSUPPORTED, "nlam * nrhs > 65535");
  dfisher_options o;
  DF_TRY(check_opt(opt, &o, true));
  DF_TRY(check_no_tol(o));
  DF_TRY(check_no_final(o));
  DF_TRY(check_prec_layout(o.gram_prec, S, lds));
  const bool async = (o.flags & DFISHER_ASYNC) != 0;
  if (async && o.shift_policy == DFISHER_SHIFT_ON_FAILURE)
    return fail(DFISHER_E_UNSUPPORTED, "DFISHER_ASYNC needs shift_policy NONE or ALWAYS (ON_FAILURE decides on the host)");
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  bool capturing = false;
  if (async) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(st, &cs));
    capturing = cs == hipStreamCaptureStatusActive;
  }
  if (ctx->autotune && !async) DF_TRY(tune_if_new(ctx, S, n, m, lds, o.gram_prec, st));
  const dfi::GramPlan gp = make_gram_plan(ctx, S, n, m, lds, o.gram_prec);
  const dfi::RowPassPlan rp = dfi::rowpass_plan(n, m, lds);
  const dfi::ColPassPlan cp = dfi::colpass_plan(n, m);
  const dfi::RowMultiPlan rm = dfi::rowmulti_plan(n, m, lds);
  const int64_t nvec = (int64_t)nlam * nrhs;
  const size_t dinv_el = dfi::trsv_dinv_bytes(n) / sizeof(double);
  // the final step through the codes of the Gram (apply8.hip) for every (lambda, rhs) pair
  const bool final8 = o.gram_prec == DFISHER_GRAM_MXFP8 && o.sweeps != 0 && (o.flags & DFISHER_EXACT_APPLY) == 0;
  // workspace: the single-solve buffers (Gram stage, retry scratch), nlam factors, their block
  // inverses and statuses, and the multi-vector buffers
  auto layout = [&](char* base, SolveBufs& B, double*& Lall, double*& Dall, double*& dkk, int64_t*& dinfo,
                    int32_t*& dflag, MultiBufs& mb) {
    B = carve(base, n, m, &gp, rp, cp, true, false);
    Carver c;
    c.base = base;
    c.off = B.bytes;
    Lall = c.take<double>((size_t)(nlam * n * n));
    Dall = c.take<double>((size_t)nlam * dinv_el);
    dkk = c.take<double>((size_t)nlam * 64 * 64);
    dinfo = c.take<int64_t>((size_t)nlam);
    dflag = c.take<int32_t>((size_t)nlam);
    mb = carve_multi(c, n, m, nrhs, nvec, rm, o.sweeps != 0, final8, is_centered(o), nlam);
    return c.off;
  };
  SolveBufs B;
  double *Lall, *Dall, *dkk;
  int64_t* dinfo;
  int32_t* dflag;
  MultiBufs mb;
  const size_t need = layout(nullptr, B, Lall, Dall, dkk, dinfo, dflag, mb);
  if (capturing) {   // no allocation inside a capture; the graph will hold the workspace's addresses
    if (need > ctx->ws_bytes)
      return fail(DFISHER_E_UNSUPPORTED,
                  "the workspace must grow to %zu bytes, which cannot happen during a capture: make the same call "
                  "once outside the capture first", need);
    ctx->ws_frozen = true;
  }
  DF_TRY(ensure_ws(ctx, need));
  layout(static_cast<char*>(ctx->ws), B, Lall, Dall, dkk, dinfo, dflag, mb);

  // the shared Gram G = S S^T (exact diagonal, no lambda), formed once
  DF_TRY(gram_stage(S, nullptr, gp, rp, B, 0.0, B.W, 0, st, nullptr, is_centered(o), mb.cs ? mb.cflag : nullptr));
  if (mb.cs) {   // S^T 1 for the final step (one column pass with y = 1, FP64 sums)
    HIP_TRY(dfi::fill_value(mb.ones, n, 1.0, st));
    HIP_TRY(dfi::colpass_launch(cp, S, n, m, lds, mb.ones, nullptr, 1.0, mb.cs, 2, B.cpart, st));
  }
  const MultiF8 mf8{B.q8, B.sc8, B.ldq, B.d};
  // every W_l = G + lambda_l I (+ the up-front shift) factored in the same launches
  const double unit = gram_unit(o.gram_prec, m);
  const double scale0 = (o.shift_policy == DFISHER_SHIFT_ALWAYS) ? 2.0 * std::sqrt((double)n) * unit : 0.0;
  if (scale0 != 0.0) HIP_TRY(dfi::diag_max(B.W, n, ctx->d_scalar, st));
  for (int32_t l = 0; l < nlam; ++l)
    HIP_TRY(dfi::shift_add_copy(B.W, Lall + (int64_t)l * n * n, n, scale0, ctx->d_scalar, lambdas[l], st));
  HIP_TRY(dfi::potrf_launch_batched(Lall, n, nlam, n * n, dinfo, dflag, dkk, st));
  if (async) {   // nothing read back: the sweep count is fixed a priori, the statuses go to infos on the device
    const int sweeps = o.sweeps == DFISHER_SWEEPS_AUTO ? auto_sweeps(o.gram_prec, n, m, scale0, is_centered(o))
                                                       : o.sweeps;
    HIP_TRY(dfi::trsv_diag_inv_batched(Lall, n * n, n, nlam, Dall, st));
    DF_TRY(multi_solve(S, n, m, lds, nlam, Lall, Dall, lambdas, V, nrhs, ldv, X, ldx, o.x_fp64, sweeps, rm, mb, st,
                           final8 ? &mf8 : nullptr));
    if (infos) HIP_TRY(write_batch_infos(infos, nlam, dinfo, scale0, ctx->d_scalar, sweeps, st));
    return DFISHER_OK;
  }
  std::vector<int64_t> hinfo((size_t)nlam);
  double dmax = 0.0;
  HIP_TRY(hipMemcpyAsync(hinfo.data(), dinfo, (size_t)nlam * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  if (scale0 != 0.0) HIP_TRY(hipMemcpyAsync(&dmax, ctx->d_scalar, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  dfisher_status worst = DFISHER_OK;
  std::vector<dfisher_info> linf((size_t)nlam);
  int sweeps = o.sweeps == DFISHER_SWEEPS_AUTO ? 0 : o.sweeps;   // AUTO: the largest count any lambda needs
  for (int32_t l = 0; l < nlam; ++l) {
    dfisher_info inf{};
    inf.resid = -1.0;
    inf.w_resid = -1.0;
    inf.attempts = 1;
    inf.potrf_info = hinfo[(size_t)l];
    inf.shift = scale0 * dmax;
    double tau_rel = scale0;
    if (inf.potrf_info != 0 && o.shift_policy != DFISHER_SHIFT_NONE) {
      // rare: refactor this lambda alone with escalating shifts (B.L holds G + lambda_l I)
      HIP_TRY(dfi::add_diag_copy(B.W, B.L, n, lambdas[l], st));
      int32_t att = 0;
      const dfisher_status s = factor_with_policy(ctx, B.L, Lall + (int64_t)l * n * n, B.dkk, n, o.shift_policy, unit,
                                                  st, &inf.shift, &inf.potrf_info, &att);
      inf.attempts += att;
      if (s != DFISHER_OK && s != DFISHER_E_NOT_SPD) return s;
      tau_rel = ctx->h_scalar[0] > 0.0 ? inf.shift / ctx->h_scalar[0] : 0.0;
    }
    if (inf.potrf_info != 0) worst = DFISHER_E_NOT_SPD;
    if (o.sweeps == DFISHER_SWEEPS_AUTO)
      sweeps = std::max(sweeps, auto_sweeps(o.gram_prec, n, m, tau_rel, is_centered(o)));
    linf[(size_t)l] = inf;
  }
  for (int32_t l = 0; l < nlam; ++l) {
    linf[(size_t)l].sweeps_done = sweeps;
    if (infos) infos[l] = linf[(size_t)l];
  }
  HIP_TRY(dfi::trsv_diag_inv_batched(Lall, n * n, n, nlam, Dall, st));
  DF_TRY(multi_solve(S, n, m, lds, nlam, Lall, Dall, lambdas, V, nrhs, ldv, X, ldx, o.x_fp64, sweeps, rm, mb, st,
                           final8 ? &mf8 : nullptr));
  if (worst != DFISHER_OK) return fail(worst, "at least one lambda failed to factor (its x is not meaningful)");
  return DFISHER_OK;
}

dfisher_status dfisher_solve_uneven(dfisher_ctx* ctx, int32_t nprob, const float* const* S, const int64_t* n,
                                    const int64_t* m, const int64_t* lds, const float* const* v, const double* lambda,
                                    void* const* x, const dfisher_options* opt, void* stream, dfisher_info* infos) {
  DF_TRY(check_ctx(ctx));
  if (nprob < 1) return fail(DFISHER_E_INVALID_ARG, "nprob = %d < 1", nprob);
  if (nprob > 65535) return fail(DFISHER_E_UNSUPPORTED, "nprob = %d > 65535", nprob);
  if (!S || !n || !m || !lds || !v || !lambda || !x) return fail(DFISHER_E_INVALID_ARG, "NULL array argument");
  dfisher_options o;
  DF_TRY(check_opt(opt, &o));
  for (int32_t p = 0; p < nprob; ++p) {
    dfisher_status s = check_S(S[p], n[p], m[p], lds[p]);
    if (s != DFISHER_OK) return fail(s, "problem %d: %s", p, g_last_error.c_str());
    if (!v[p] || !x[p]) return fail(DFISHER_E_INVALID_ARG, "problem %d: v or x is NULL", p);
    if (!finite_pos(lambda[p])) return fail(DFISHER_E_INVALID_ARG, "problem %d: lambda must be finite and > 0", p);
    s = check_prec_layout(o.gram_prec, S[p], lds[p]);
    if (s != DFISHER_OK) return fail(s, "problem %d: %s", p, g_last_error.c_str());
  }
  DeviceGuard g(ctx->device);
  hipStream_t st = as_stream(stream);
  return uneven_solve(ctx, nprob, S, n, m, lds, v, lambda, x, o, st, infos);
}

int32_t dfisher_auto_sweeps(int32_t prec, int64_t n, int64_t m) {
  if (prec != DFISHER_GRAM_FP32 && prec != DFISHER_GRAM_BF16X3 && prec != DFISHER_GRAM_MXFP8) return -1;
  if (n < 1 || m < 1) return -1;
  return auto_sweeps(prec, n, m, 0.0);
}

dfisher_status dfisher_ctx_enable_autotune(dfisher_ctx* ctx, int32_t enable) {
  DF_TRY(check_ctx(ctx));
  ctx->autotune = enable != 0;
  return DFISHER_OK;
}

dfisher_status dfisher_autotune_gram(dfisher_ctx* ctx, const float* S, int64_t n, int64_t m, int64_t lds, int32_t prec,
                                     void* stream) {
  DF_TRY(check_ctx(ctx));
  DF_TRY(check_S(S, n, m, lds));
  if (prec != DFISHER_GRAM_FP32 && prec != DFISHER_GRAM_BF16X3 && prec != DFISHER_GRAM_MXFP8)
    return fail(DFISHER_E_INVALID_ARG, "unknown gram_prec %d", prec);
  DF_TRY(check_prec_layout(prec, S, lds));
  DeviceGuard g(ctx->device);
  return tune_gram(ctx, S, n, m, lds, prec, as_stream(stream));
}

// Text format, one size class per line: "prec tiles log2m aligned q mode".
dfisher_status dfisher_ctx_save_tuning(const dfisher_ctx* ctx, const char* path) {
  if (!ctx || !path) return fail(DFISHER_E_INVALID_ARG, "ctx or path is NULL");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(DFISHER_E_INVALID_ARG, "cannot open %s for writing", path);
  std::fprintf(f, "# dfisher gram tuning: prec tiles log2m aligned q mode\n");
  for (const auto& kv : ctx->tune)
    std::fprintf(f, "%d %lld %d %d %d %d\n", std::get<0>(kv.first), (long long)std::get<1>(kv.first),
                 std::get<2>(kv.first), std::get<3>(kv.first), kv.second.first, kv.second.second);
  const bool ok = std::fclose(f) == 0;
  return ok ? DFISHER_OK : fail(DFISHER_E_INVALID_ARG, "write to %s failed", path);
}

dfisher_status dfisher_ctx_load_tuning(dfisher_ctx* ctx, const char* path) {
  if (!ctx || !path) return fail(DFISHER_E_INVALID_ARG, "ctx or path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(DFISHER_E_INVALID_ARG, "cannot open %s", path);
  std::map<std::tuple<int, int64_t, int, int>, std::pair<int, int>> t;
  char line[256];
  int lineno = 0;
  dfisher_status st = DFISHER_OK;
  while (std::fgets(line, sizeof line, f)) {
    ++lineno;
    if (line[0] == '#' || line[0] == '\n') continue;
    int prec, lg, al, q, mode;
    long long tiles;
    if (std::sscanf(line, "%d %lld %d %d %d %d", &prec, &tiles, &lg, &al, &q, &mode) != 6 || prec < 0 || prec > 2 ||
        tiles < 1 || lg < 0 || lg > 62 || (al != 0 && al != 1) || q < 1 || q > 64 || mode < -1 || mode > 1) {
      st = fail(DFISHER_E_INVALID_ARG, "%s:%d: malformed tuning entry", path, lineno);
      break;
    }
    t[std::make_tuple(prec, (int64_t)tiles, lg, al)] = std::make_pair(q, mode);
  }
  std::fclose(f);
  if (st != DFISHER_OK) return st;
  for (const auto& kv : t) ctx->tune[kv.first] = kv.second;
  drop_graph(ctx);   // a captured uneven graph may have been laid out with the old plans
  return DFISHER_OK;
}

dfisher_status dfisher_ctx_enable_graphs(dfisher_ctx* ctx, int32_t enable) {
  DF_TRY(check_ctx(ctx));
  ctx->graphs = enable != 0;
  if (!ctx->graphs) drop_graph(ctx);
  return DFISHER_OK;
}

}  // extern "C"
