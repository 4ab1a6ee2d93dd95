/*
 * FP64 CPU oracle for the Cholesky solve of the damped Fisher system
 *
 *     (S^T S + lambda I_m) x = v,      S in R^{n x m}, x, v in R^m, lambda > 0     (Eq. 1)
 *
 * of Chen, Xie & Wang, "Efficient Numerical Algorithm for Large-Scale Damped Natural
 * Gradient Descent" (arXiv 2310.17556), Section 2, Algorithm 1.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously correct reference that the
 * HIP library is checked against. Only tests/, __graft_entry__.smoke() and the cpu_baseline
 * leg of bench.py may load it. It shares no code, header, table or helper with the HIP path
 * (paper_2310_17556_amd/), and the HIP path never calls it.
 *
 * Conventions
 *   - S is the caller's FP32 data, row-major n x m with row stride lds >= m (sample i's
 *     gradient is row i). Every FP32 value is converted to FP64 exactly before use.
 *   - All arithmetic is FP64 in the plain order of the definition: a sum over k runs
 *     k = 0, 1, ..., K-1 sequentially. There is no blocking or reassociation. OpenMP only
 *     distributes independent output entries over threads, which does not change any
 *     entry's summation order, so results are bitwise independent of the thread count.
 *   - Matrices W and L are n x n row-major FP64 (full storage).
 *
 * Precision-split helpers (oracle_split_bf16, oracle_gram3) define what the split-BF16 Gram
 * computes: S = hi + lo with hi = bf16 round-to-nearest-even of S and lo = bf16 RNE of the
 * (exact) remainder, and the Gram keeps the three products hi.hi + hi.lo + lo.hi.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))

static double sd(const float* S, int64_t lds, int64_t i, int64_t k) {
  return (double)S[i * lds + k];
}

/* Algorithm 1, step 1 (Section 2): W = S S^T + lambda * I_n   (I-tilde is the n x n identity).
 * W_ij = sum_k S_ik S_jk, k ascending; both triangles are written (W_ji = W_ij).
 * lambda = 0 gives the plain Gram G = S S^T. */
EXPORT void oracle_gram(const float* S, int64_t n, int64_t m, int64_t lds, double lambda, double* W) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j <= i; ++j) {
      double acc = 0.0;
      for (int64_t k = 0; k < m; ++k) acc += sd(S, lds, i, k) * sd(S, lds, j, k);
      if (i == j) acc += lambda;
      W[i * n + j] = acc;
      W[j * n + i] = acc;
    }
  }
}

/* Algorithm 1, step 2: L = Chol(W), W = L L^T with L lower triangular and L_jj > 0.
 * Textbook Cholesky-Banachiewicz, row by row:
 *   L_ij = (W_ij - sum_{k<j} L_ik L_jk) / L_jj          (j < i)
 *   L_ii = sqrt(W_ii - sum_{k<i} L_ik^2)
 * Reads only the lower triangle of W. Returns 0 on success, or the 1-based index i of the
 * first pivot d = W_ii - sum L_ik^2 with !(d > 0) (so a NaN pivot fails too); L is then
 * valid in rows < i-1 only. The strict upper triangle of L is set to zero. */
EXPORT int64_t oracle_cholesky(const double* W, int64_t n, double* L) {
  memset(L, 0, (size_t)(n * n) * sizeof(double));
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < i; ++j) {
      double acc = W[i * n + j];
      for (int64_t k = 0; k < j; ++k) acc -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = acc / L[j * n + j];
    }
    double d = W[i * n + i];
    for (int64_t k = 0; k < i; ++k) d -= L[i * n + k] * L[i * n + k];
    if (!(d > 0.0)) return i + 1;
    L[i * n + i] = sqrt(d);
  }
  return 0;
}

/* First product of the inlined right-to-left evaluation of Q^T Q v = S^T L^-T L^-1 S v
 * (Section 2, paragraph after Algorithm 1): b = S v, b_i = sum_k S_ik v_k. */
EXPORT void oracle_gemv(const float* S, int64_t n, int64_t m, int64_t lds, const double* v, double* b) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int64_t k = 0; k < m; ++k) acc += sd(S, lds, i, k) * v[k];
    b[i] = acc;
  }
}

/* Triangular solve L z = b by forward substitution: z_i = (b_i - sum_{k<i} L_ik z_k) / L_ii.
 * This applies L^-1 (Section 2, "triangular solve"). */
EXPORT void oracle_forward(const double* L, int64_t n, const double* b, double* z) {
  for (int64_t i = 0; i < n; ++i) {
    double acc = b[i];
    for (int64_t k = 0; k < i; ++k) acc -= L[i * n + k] * z[k];
    z[i] = acc / L[i * n + i];
  }
}

/* Triangular solve L^T y = z by back substitution: y_i = (z_i - sum_{k>i} L_ki y_k) / L_ii.
 * This applies L^-T. */
EXPORT void oracle_backward(const double* L, int64_t n, const double* z, double* y) {
  for (int64_t i = n - 1; i >= 0; --i) {
    double acc = z[i];
    for (int64_t k = i + 1; k < n; ++k) acc -= L[k * n + i] * y[k];
    y[i] = acc / L[i * n + i];
  }
}

/* Last steps of Algorithm 1 (step 4 with Q inlined): x = (v - S^T y) / lambda, where
 * y = L^-T L^-1 S v so that S^T y = Q^T Q v. (S^T y)_k = sum_i S_ik y_i, i ascending.
 * The loop runs i outer / k inner so that S is read row by row; each x_k still sums over i
 * in ascending order. */
EXPORT void oracle_apply(const float* S, int64_t n, int64_t m, int64_t lds, const double* v,
                         const double* y, double lambda, double* x) {
  const int64_t CB = 4096;
#pragma omp parallel for schedule(static)
  for (int64_t c0 = 0; c0 < m; c0 += CB) {
    int64_t c1 = c0 + CB < m ? c0 + CB : m;
    double t[4096];
    for (int64_t k = c0; k < c1; ++k) t[k - c0] = 0.0;
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = c0; k < c1; ++k) t[k - c0] += sd(S, lds, i, k) * y[i];
    for (int64_t k = c0; k < c1; ++k) x[k] = (v[k] - t[k - c0]) / lambda;
  }
}

/* Algorithm 1 end to end with Q inlined (Section 2):
 *   W = S S^T + lambda I;  L = Chol(W);  b = S v;  z = L^-1 b;  y = L^-T z;  x = (v - S^T y)/lambda.
 * x (m) is required; y (n) is optional (NULL to skip). Returns the Cholesky info (0 = ok);
 * on failure x is not written. */
EXPORT int64_t oracle_solve(const float* S, int64_t n, int64_t m, int64_t lds, const double* v,
                            double lambda, double* x, double* y_out) {
  double* W = (double*)malloc((size_t)(n * n) * sizeof(double));
  double* L = (double*)malloc((size_t)(n * n) * sizeof(double));
  double* b = (double*)malloc((size_t)n * sizeof(double));
  double* z = (double*)malloc((size_t)n * sizeof(double));
  double* y = (double*)malloc((size_t)n * sizeof(double));
  int64_t info = -1;
  if (W && L && b && z && y) {
    oracle_gram(S, n, m, lds, lambda, W);
    info = oracle_cholesky(W, n, L);
    if (info == 0) {
      oracle_gemv(S, n, m, lds, v, b);
      oracle_forward(L, n, b, z);
      oracle_backward(L, n, z, y);
      oracle_apply(S, n, m, lds, v, y, lambda, x);
      if (y_out) memcpy(y_out, y, (size_t)n * sizeof(double));
    }
  }
  free(W); free(L); free(b); free(z); free(y);
  return info;
}

/* Residual of Eq. 1 as written in the proof of Proposition 1 (Appendix A):
 * r = v - lambda x - S^T (S x). Computed as t = S x (n), then r_k = v_k - lambda x_k - sum_i S_ik t_i. */
EXPORT void oracle_residual(const float* S, int64_t n, int64_t m, int64_t lds, const double* v,
                            const double* x, double lambda, double* r) {
  double* t = (double*)malloc((size_t)n * sizeof(double));
  if (!t) return;
  oracle_gemv(S, n, m, lds, x, t);
  const int64_t CB = 4096;
#pragma omp parallel for schedule(static)
  for (int64_t c0 = 0; c0 < m; c0 += CB) {
    int64_t c1 = c0 + CB < m ? c0 + CB : m;
    double u[4096];
    for (int64_t k = c0; k < c1; ++k) u[k - c0] = 0.0;
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = c0; k < c1; ++k) u[k - c0] += sd(S, lds, i, k) * t[i];
    for (int64_t k = c0; k < c1; ++k) r[k] = v[k] - lambda * x[k] - u[k - c0];
  }
  free(t);
}

/* Round a finite FP64 value to the nearest bfloat16 (8 significant bits, FP32 exponent range,
 * subnormals with spacing 2^-133), ties to even, straight from the definition: write
 * a = f * 2^e with 0.5 <= |f| < 1 and round f * 2^8 to an integer with nearbyint (the default
 * rounding mode is round-half-to-even). */
static double round_bf16(double a) {
  if (a == 0.0 || !isfinite(a)) return a;
  int e;
  double f = frexp(a, &e);            /* a = f * 2^e */
  if (e - 1 < -126) {                 /* below the smallest normal 2^-126: fixed spacing 2^-133 */
    return ldexp(nearbyint(ldexp(a, 133)), -133);
  }
  return ldexp(nearbyint(ldexp(f, 8)), e - 8);
}

/* Split-BF16 representation of S (the precision split of the Gram's inputs):
 * hi = RNE_bf16(S), lo = RNE_bf16(S - hi). S - hi is exact in FP64 (and in FP32).
 * hi and lo are returned as FP32 arrays (bf16 values are exactly representable), n x m dense. */
EXPORT void oracle_split_bf16(const float* S, int64_t n, int64_t m, int64_t lds, float* hi, float* lo) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t k = 0; k < m; ++k) {
      double a = sd(S, lds, i, k);
      double h = round_bf16(a);
      double l = round_bf16(a - h);
      hi[i * m + k] = (float)h;
      lo[i * m + k] = (float)l;
    }
  }
}

/* Gram of a split representation A = hi + lo keeping three of the four products:
 * G_ij = sum_k (hi_ik hi_jk + hi_ik lo_jk + lo_ik hi_jk), k ascending, FP64, plus lambda on
 * the diagonal. hi, lo are n x m dense FP32. Both triangles are written. */
EXPORT void oracle_gram3(const float* hi, const float* lo, int64_t n, int64_t m, double lambda, double* W) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j <= i; ++j) {
      double acc = 0.0;
      for (int64_t k = 0; k < m; ++k) {
        double hi_i = hi[i * m + k], hi_j = hi[j * m + k];
        double lo_i = lo[i * m + k], lo_j = lo[j * m + k];
        acc += hi_i * hi_j + hi_i * lo_j + lo_i * hi_j;
      }
      if (i == j) acc += lambda;
      W[i * n + j] = acc;
      W[j * n + i] = acc;
    }
  }
}

/* Round a finite value to the nearest OCP FP8 E4M3 value, ties to even (1 sign, 4 exponent bits
 * with bias 7, 3 mantissa bits; normals 2^-6 .. 448, subnormals k * 2^-9). The caller keeps
 * |a| <= 448, so no saturation is needed. From the definition: the spacing of representable
 * values at magnitude |a| is 2^(floor(log2|a|) - 3) for |a| >= 2^-6 and 2^-9 below. */
static double round_e4m3(double a) {
  if (a == 0.0 || !isfinite(a)) return a;
  double q;
  if (fabs(a) < ldexp(1.0, -6)) {
    q = ldexp(1.0, -9);
  } else {
    int e;
    frexp(a, &e);               /* |a| = f 2^e, 0.5 <= f < 1, so floor(log2|a|) = e - 1 */
    q = ldexp(1.0, e - 1 - 3);
  }
  return nearbyint(a / q) * q;
}

/* Block-scaled FP8 representation of S (the scaled-FP8 form of the Gram's inputs). Row i is cut
 * into blocks of 32 consecutive columns [32b, 32b + 32) (the last may be shorter). Each block
 * gets a power-of-two scale 2^e with e the smallest integer such that amax <= 448 * 2^e
 * (amax = max |S_ik| over the block; e = -127 for an all-zero block), clamped to [-127, 127];
 * each element becomes q = round_e4m3(S_ik / 2^e). Outputs: deq (n x m, FP32) = q * 2^e, the
 * value the products use, and sexp (n x ceil(m/32), int32) = e. */
EXPORT void oracle_quant_mxfp8(const float* S, int64_t n, int64_t m, int64_t lds, float* deq, int32_t* sexp) {
  const int64_t nblk = (m + 31) / 32;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t b = 0; b < nblk; ++b) {
      const int64_t k0 = 32 * b, k1 = (k0 + 32 < m) ? k0 + 32 : m;
      double amax = 0.0;
      for (int64_t k = k0; k < k1; ++k) {
        const double a = fabs(sd(S, lds, i, k));
        if (a > amax) amax = a;
      }
      int e = -127;
      if (amax > 0.0) {
        e = -127;
        while (e < 127 && amax > 448.0 * ldexp(1.0, e)) ++e;
      }
      sexp[i * nblk + b] = e;
      for (int64_t k = k0; k < k1; ++k) {
        const double q = round_e4m3(ldexp(sd(S, lds, i, k), -e));
        deq[i * m + k] = (float)ldexp(q, e);
      }
    }
  }
}

/* Squared row norms d_i = sum_k S_ik^2 (the exact diagonal of S S^T). */
EXPORT void oracle_row_norms(const float* S, int64_t n, int64_t m, int64_t lds, double* d) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int64_t k = 0; k < m; ++k) acc += sd(S, lds, i, k) * sd(S, lds, i, k);
    d[i] = acc;
  }
}

/* Sampled Gram entries W_{ij} = sum_k S_ik S_jk (+ lambda if i == j) for index pairs (ii[p], jj[p]).
 * Lets a test check single entries of a Gram that is too large to form on the host. */
EXPORT void oracle_gram_entries(const float* S, int64_t m, int64_t lds, double lambda, const int64_t* ii,
                                const int64_t* jj, int64_t npairs, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < npairs; ++p) {
    double acc = 0.0;
    for (int64_t k = 0; k < m; ++k) acc += sd(S, lds, ii[p], k) * sd(S, lds, jj[p], k);
    if (ii[p] == jj[p]) acc += lambda;
    out[p] = acc;
  }
}

/* ---------------------------------------------------------------------------------------------
 * Structured right-hand side (Appendix B). When v = S^T f lies in the row space of S, the push-
 * through identity S^T (S S^T + lambda I)^-1 = (S^T S + lambda I)^-1 S^T gives
 *   x = S^T y,   y = (S S^T + lambda I)^-1 f,
 * so neither b = S v nor the subtraction v - S^T y is formed. Steps: W = S S^T + lambda I
 * (oracle_gram), L = Chol(W), z = L^-1 f, y = L^-T z, x_k = sum_i S_ik y_i (i ascending).
 * Returns the Cholesky info (0 = ok); x and y are written only on success (y may be NULL). */
EXPORT int64_t oracle_solve_rowspace(const float* S, int64_t n, int64_t m, int64_t lds, const double* f,
                                     double lambda, double* x, double* y_out) {
  double* W = (double*)malloc((size_t)(n * n) * sizeof(double));
  double* L = (double*)malloc((size_t)(n * n) * sizeof(double));
  double* z = (double*)malloc((size_t)n * sizeof(double));
  double* y = (double*)malloc((size_t)n * sizeof(double));
  int64_t info = -1;
  if (W && L && z && y) {
    oracle_gram(S, n, m, lds, lambda, W);
    info = oracle_cholesky(W, n, L);
    if (info == 0) {
      oracle_forward(L, n, f, z);
      oracle_backward(L, n, z, y);
#pragma omp parallel for schedule(static)
      for (int64_t k = 0; k < m; ++k) {
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) acc += sd(S, lds, i, k) * y[i];
        x[k] = acc;
      }
      if (y_out) memcpy(y_out, y, (size_t)n * sizeof(double));
    }
  }
  free(W); free(L); free(z); free(y);
  return info;
}

/* ---------------------------------------------------------------------------------------------
 * Stochastic-reconfiguration front end (Section 3). The score matrix of SR is the centered,
 * scaled log-derivative matrix S = (O - mean(O)) / sqrt(n), the mean taken over the n samples
 * (rows) for every parameter (column):
 *   mu_j = (sum_i O_ij) / n            (FP64, i ascending)
 *   S_ij = fl32((O_ij - mu_j) / sqrt(n))   (FP64 subtraction and division, one rounding to FP32)
 * O is n x m FP32 (row stride ldo); S is n x m FP32 (row stride lds). */
EXPORT void oracle_center(const float* O, int64_t n, int64_t m, int64_t ldo, float* S, int64_t lds) {
  const double rn = sqrt((double)n);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < m; ++j) {
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += (double)O[i * ldo + j];
    const double mu = acc / (double)n;
    for (int64_t i = 0; i < n; ++i) S[i * lds + j] = (float)(((double)O[i * ldo + j] - mu) / rn);
  }
}

/* Complex O (the log-derivatives of a complex wave function), n x m complex values stored as
 * interleaved (real, imaginary) FP32 pairs, row stride ldo complex elements. The complex mean is
 * taken componentwise, so the real and imaginary parts are centered as two real matrices, and the
 * result is written in the stacked real form Z (2n x m FP32, row stride ldz):
 *   Z_ij = Re S_ij (rows 0..n-1),  Z_(n+i)j = Im S_ij (rows n..2n-1).
 * Z is the concatenation of Re S and Im S in the sample dimension that the real-part variant of
 * SR, F = Re[S^H S] = Z^T Z, solves with (Section 3), and the planar form of S that the complex
 * variant takes. */
EXPORT void oracle_center_complex(const float* O, int64_t n, int64_t m, int64_t ldo, float* Z, int64_t ldz) {
  const double rn = sqrt((double)n);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < m; ++j) {
    double ar = 0.0, ai = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      ar += (double)O[2 * (i * ldo + j)];
      ai += (double)O[2 * (i * ldo + j) + 1];
    }
    const double mr = ar / (double)n, mi = ai / (double)n;
    for (int64_t i = 0; i < n; ++i) {
      Z[i * ldz + j] = (float)(((double)O[2 * (i * ldo + j)] - mr) / rn);
      Z[(n + i) * ldz + j] = (float)(((double)O[2 * (i * ldo + j) + 1] - mi) / rn);
    }
  }
}

/* ---------------------------------------------------------------------------------------------
 * Complex variant (Section 3): with a complex S every transpose of Eq. 1 and Algorithm 1 becomes
 * the Hermitian conjugate, (S^H S + lambda I) x = v with x, v in C^m:
 *   W = S S^H + lambda I_n       W_ij = sum_k S_ik conj(S_jk)                      (k ascending)
 *   W = L L^H                    L_ij = (W_ij - sum_{k<j} L_ik conj(L_jk)) / L_jj   (j < i)
 *                                L_ii = sqrt(W_ii - sum_{k<i} |L_ik|^2)   (real; fails unless > 0)
 *                                (every division is by the real L_jj, componentwise)
 *   b = S v,  z = L^-1 b,  y = L^-H z   (y_i = (z_i - sum_{k>i} conj(L_ki) y_k) / L_ii)
 *   x = (v - S^H y) / lambda     (S^H y)_k = sum_i conj(S_ik) y_i                   (i ascending)
 * in C99 complex FP64. S: n x m complex FP32 values as interleaved (re, im) pairs with row stride
 * lds complex elements; v, x (m) and y (n, may be NULL) are interleaved complex FP64. Returns the
 * Cholesky info (0 or the 1-based index of the first pivot that is not > 0); on failure x is not
 * written. */
static double complex cs(const float* S, int64_t lds, int64_t i, int64_t k) {
  return (double)S[2 * (i * lds + k)] + (double)S[2 * (i * lds + k) + 1] * I;
}

EXPORT int64_t oracle_solve_complex(const float* S, int64_t n, int64_t m, int64_t lds, const double* v,
                                    double lambda, double* x, double* y_out) {
  double complex* W = (double complex*)malloc((size_t)(n * n) * sizeof(double complex));
  double complex* L = (double complex*)calloc((size_t)(n * n), sizeof(double complex));
  double complex* b = (double complex*)malloc((size_t)n * sizeof(double complex));
  double complex* z = (double complex*)malloc((size_t)n * sizeof(double complex));
  double complex* y = (double complex*)malloc((size_t)n * sizeof(double complex));
  int64_t info = -1;
  if (!(W && L && b && z && y)) goto out;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j <= i; ++j) {
      double complex acc = 0.0;
      for (int64_t k = 0; k < m; ++k) acc += cs(S, lds, i, k) * conj(cs(S, lds, j, k));
      if (i == j) acc += lambda;
      W[i * n + j] = acc;
    }
  }
  info = 0;
  for (int64_t i = 0; i < n && info == 0; ++i) {
    for (int64_t j = 0; j < i; ++j) {
      double complex acc = W[i * n + j];
      for (int64_t k = 0; k < j; ++k) acc -= L[i * n + k] * conj(L[j * n + k]);
      L[i * n + j] = acc / creal(L[j * n + j]);
    }
    double d = creal(W[i * n + i]);
    for (int64_t k = 0; k < i; ++k) d -= creal(L[i * n + k]) * creal(L[i * n + k]) + cimag(L[i * n + k]) * cimag(L[i * n + k]);
    if (!(d > 0.0)) info = i + 1;
    else L[i * n + i] = sqrt(d);
  }
  if (info != 0) goto out;
  for (int64_t i = 0; i < n; ++i) {
    double complex acc = 0.0;
    for (int64_t k = 0; k < m; ++k) acc += cs(S, lds, i, k) * (v[2 * k] + v[2 * k + 1] * I);
    b[i] = acc;
  }
  for (int64_t i = 0; i < n; ++i) {
    double complex acc = b[i];
    for (int64_t k = 0; k < i; ++k) acc -= L[i * n + k] * z[k];
    z[i] = acc / creal(L[i * n + i]);
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double complex acc = z[i];
    for (int64_t k = i + 1; k < n; ++k) acc -= conj(L[k * n + i]) * y[k];
    y[i] = acc / creal(L[i * n + i]);
  }
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    double complex t = 0.0;
    for (int64_t i = 0; i < n; ++i) t += conj(cs(S, lds, i, k)) * y[i];
    const double complex xk = ((v[2 * k] + v[2 * k + 1] * I) - t) / lambda;
    x[2 * k] = creal(xk);
    x[2 * k + 1] = cimag(xk);
  }
  if (y_out)
    for (int64_t i = 0; i < n; ++i) {
      y_out[2 * i] = creal(y[i]);
      y_out[2 * i + 1] = cimag(y[i]);
    }
out:
  free(W); free(L); free(b); free(z); free(y);
  return info;
}

/* Preconditioner of a centered score matrix (Section 3: S = (O - mean O) / sqrt(n) has columns
 * that sum to zero over the samples, so S S^T has the all-ones vector as an exact null vector and
 * W = S S^T + lambda I maps it to lambda times itself). Given an n x n symmetric W (full storage)
 * and nseg equal contiguous segments of length l = n / nseg (nseg = 2 for the real embedding of
 * the complex variant, whose two null vectors are the indicators of the real and imaginary
 * halves), this writes
 *     M = P W P + lambda U U^T,    P = I - U U^T,    U = [u_1 .. u_nseg],  u_s = 1_{segment s} / sqrt(l)
 * i.e. W compressed to the complement of the indicators, with lambda on them. Computed as the
 * definition: P formed explicitly, then the two matrix products in plain loops. */
EXPORT void oracle_project_centered(const double* W, int64_t n, int64_t nseg, double lambda, double* M) {
  const int64_t l = n / nseg;
  double* P = (double*)malloc((size_t)(n * n) * sizeof(double));
  double* T = (double*)malloc((size_t)(n * n) * sizeof(double));
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      const double uu = (i / l == j / l) ? 1.0 / (double)l : 0.0;   /* (U U^T)_ij */
      P[i * n + j] = (i == j ? 1.0 : 0.0) - uu;
    }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int64_t k = 0; k < n; ++k) acc += P[i * n + k] * W[k * n + j];
      T[i * n + j] = acc;
    }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int64_t k = 0; k < n; ++k) acc += T[i * n + k] * P[k * n + j];
      const double uu = (i / l == j / l) ? 1.0 / (double)l : 0.0;
      M[i * n + j] = acc + lambda * uu;
    }
  free(P);
  free(T);
}

/* Number of OpenMP threads the oracle runs on (1 without OpenMP). */
EXPORT int oracle_num_threads(void) {
  int t = 1;
#pragma omp parallel
  {
#pragma omp single
    {
#ifdef _OPENMP
      extern int omp_get_num_threads(void);
      t = omp_get_num_threads();
#endif
    }
  }
  return t;
}
