"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each pin is chosen so that a plausible slip in the oracle (a dropped lambda, a wrong sign, a
transposed L, an off-by-one in a triangular loop, a missing square root) fails at least one:

* brute force: a dense FP64 solve of the m x m system of Eq. 1 (LU via numpy, not Cholesky);
* hand-derived worked examples (tests/golden/hand_examples.json);
* closed forms: S = 0, v orthogonal to the rows of S, n = 1 (Sherman-Morrison), orthogonal rows;
* Proposition 1 (Appendix A): S^T S x + lambda x = v, and the intermediate (S S^T + lambda I) S x = S v;
* Appendix B: for v = S^T f the solution equals S^T (S S^T + lambda I)^-1 f;
* Appendix C: the thin-SVD formula x = V (Sigma^2 + lambda)^-1 V^T v + (v - V V^T v)/lambda;
* Cholesky of the Pascal matrix, whose factor is the binomial-coefficient triangle, and of
  matrices with a known first bad pivot;
* exact scaling and permutation relations (metamorphic tests);
* the bf16 split against torch's round-to-nearest-even conversion and hand-computed ties.
"""
import json
import math
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
EPS = np.finfo(np.float64).eps


def _dense_solve(S, v, lam):
    S64 = S.astype(np.float64)
    A = S64.T @ S64 + lam * np.eye(S.shape[1])
    return np.linalg.solve(A, np.asarray(v, dtype=np.float64))


def _cond_tol(S, lam, c=50.0):
    s = np.linalg.svd(S.astype(np.float64), compute_uv=False)
    smax2 = float(s[0] ** 2) if s.size else 0.0
    return c * EPS * (smax2 + lam) / lam


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


# ------------------------------------------------------------------ brute force (Eq. 1)

@pytest.mark.parametrize("lam", [1e-2])
def test_bruteforce_smallest_workload(oracle_mod, lam):
    """The smallest workload (n=32, m=1024, iid column-centered S, iid v, lambda=1e-2) against a
    dense LU solve of the m x m system."""
    S = synth.make_S(32, 1024, synth.seed(1), "iid")
    v = synth.make_v(S, synth.seed(1), "iid")
    x = oracle_mod.solve(S, v, lam)
    xd = _dense_solve(S, v, lam)
    assert _rel(x, xd) <= _cond_tol(S, lam)


@pytest.mark.parametrize("n,m,lam,kind", [
    (16, 300, 1e-1, "iid"), (16, 300, 1e-4, "iid"), (16, 300, 1e-6, "iid"),
    (48, 200, 1e-3, "scaled"), (7, 513, 3.0, "iid"),
    (40, 30, 1e-2, "iid"),          # n > m is valid too (W stays SPD)
])
def test_bruteforce_shapes(oracle_mod, n, m, lam, kind):
    S = synth.make_S(n, m, synth.seed(9, n + m), kind)
    v = synth.make_v(S, synth.seed(9, n + m), kind)
    x = oracle_mod.solve(S, v, lam)
    assert _rel(x, _dense_solve(S, v, lam)) <= _cond_tol(S, lam)


def test_bruteforce_uncentered_and_strided(oracle_mod):
    """A non-contiguous row stride (ld > m) must read the same logical matrix."""
    S = synth.make_S(20, 333, 5, "iid", center=False)
    buf = np.zeros((20, 400), dtype=np.float32)
    buf[:, :333] = S
    v = synth.make_v(S, 5)
    x = oracle_mod.solve(buf[:, :333], v, 1e-2)
    assert _rel(x, _dense_solve(S, v, 1e-2)) <= _cond_tol(S, 1e-2)


# ------------------------------------------------------------------ hand-derived examples

def _golden():
    with open(os.path.join(HERE, "golden", "hand_examples.json")) as f:
        return json.load(f)["examples"]


@pytest.mark.parametrize("ex", _golden(), ids=lambda e: e["name"])
def test_hand_examples(oracle_mod, ex):
    S = np.array(ex["S"], dtype=np.float32)
    v = np.array(ex["v"])
    lam = ex["lambda"]
    W = oracle_mod.gram(S, lam)
    np.testing.assert_allclose(W, ex["W"], rtol=0, atol=1e-15)
    L, info = oracle_mod.cholesky(W)
    assert info == 0
    np.testing.assert_allclose(L, ex["L"], rtol=1e-15, atol=1e-15)
    x, y = oracle_mod.solve(S, v, lam, return_y=True)
    np.testing.assert_allclose(y, ex["y"], rtol=1e-14)
    np.testing.assert_allclose(x, ex["x"], rtol=1e-14, atol=1e-15)


# ------------------------------------------------------------------ Gram (Algorithm 1 step 1)

def test_gram_against_blas_and_invariants(oracle_mod):
    S = synth.make_S(70, 1500, 3, "scaled")
    lam = 0.25
    W = oracle_mod.gram(S, lam)
    S64 = S.astype(np.float64)
    ref = S64 @ S64.T + lam * np.eye(70)
    np.testing.assert_allclose(W, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    assert np.array_equal(W, W.T)
    d = oracle_mod.row_norms(S)
    np.testing.assert_allclose(np.diag(W), d + lam, rtol=1e-15)
    np.testing.assert_allclose(np.trace(W), (S64 ** 2).sum() + 70 * lam, rtol=1e-12)
    # |W_ij| <= sqrt(W_ii W_jj) (positive semidefinite Gram + lambda on the diagonal)
    dd = np.sqrt(np.outer(np.diag(W), np.diag(W)))
    assert np.all(np.abs(W) <= dd * (1 + 1e-12))


def test_gram_entries_match_full_gram(oracle_mod):
    S = synth.make_S(30, 700, 4)
    W = oracle_mod.gram(S, 0.5)
    ii = np.array([0, 5, 29, 17, 3])
    jj = np.array([0, 2, 29, 29, 12])
    np.testing.assert_array_equal(oracle_mod.gram_entries(S, ii, jj, 0.5), W[ii, jj])


def test_centered_gram_has_lambda_direction(oracle_mod):
    """For a column-centered S, 1^T S = 0 up to rounding, so W 1 = lambda 1 (Section 3 centering)."""
    S = synth.make_S(24, 4000, 6, "iid")
    lam = 1e-3
    W = oracle_mod.gram(S, lam)
    one = np.ones(24)
    S64 = S.astype(np.float64)
    c = S64.T @ one                      # column sums left by FP32 rounding of the centering
    assert np.abs(c).max() <= 24 * 2.0 ** -24 * np.abs(S64).max(axis=0).max()
    # W 1 - lambda 1 = S (S^T 1): bounded entrywise by |s_i| |S^T 1| (Cauchy-Schwarz)
    dev = np.abs(W @ one - lam * one)
    assert np.all(dev <= np.linalg.norm(S64, axis=1) * np.linalg.norm(c) * (1 + 1e-9) + 1e-15)


# ------------------------------------------------------------------ Cholesky (step 2)

def test_cholesky_pascal(oracle_mod):
    """The symmetric Pascal matrix P_ij = C(i+j, i) has the Cholesky factor L_ij = C(i, j)."""
    n = 12
    P = np.array([[math.comb(i + j, i) for j in range(n)] for i in range(n)], dtype=np.float64)
    Lx = np.array([[math.comb(i, j) if j <= i else 0 for j in range(n)] for i in range(n)], dtype=np.float64)
    L, info = oracle_mod.cholesky(P)
    assert info == 0
    np.testing.assert_allclose(L, Lx, rtol=1e-9, atol=1e-9)


def test_cholesky_diagonal_and_2x2(oracle_mod):
    L, info = oracle_mod.cholesky(np.diag([4.0, 9.0, 2.25]))
    assert info == 0
    np.testing.assert_array_equal(L, np.diag([2.0, 3.0, 1.5]))
    a, b, c = 5.0, 2.0, 3.0
    L, info = oracle_mod.cholesky(np.array([[a, b], [b, c]]))
    l11 = math.sqrt(a)
    np.testing.assert_allclose(L, [[l11, 0.0], [b / l11, math.sqrt(c - b * b / a)]], rtol=1e-15)


def test_cholesky_reads_lower_triangle_only(oracle_mod):
    rng = np.random.default_rng(0)
    A = rng.standard_normal((9, 9))
    W = A @ A.T + 9 * np.eye(9)
    Wl = np.tril(W) + np.triu(np.full((9, 9), 1e30), 1)
    L1, _ = oracle_mod.cholesky(W)
    L2, _ = oracle_mod.cholesky(Wl)
    np.testing.assert_array_equal(L1, L2)
    np.testing.assert_allclose(L1 @ L1.T, W, rtol=1e-13, atol=1e-13)
    assert np.all(np.diag(L1) > 0) and np.all(np.triu(L1, 1) == 0)


@pytest.mark.parametrize("W,info", [
    (np.diag([1.0, 2.0, -1.0, 3.0]), 3),
    (np.diag([0.0, 1.0]), 1),
    (np.array([[1.0, 2.0], [2.0, 1.0]]), 2),     # indefinite: second pivot 1 - 4 = -3
    (np.array([[1.0, 1.0], [1.0, 1.0]]), 2),     # singular: second pivot exactly 0
    (np.diag([1.0, np.nan, 1.0]), 2),            # NaN pivot fails the !(d > 0) test
])
def test_cholesky_breakdown_index(oracle_mod, W, info):
    _, got = oracle_mod.cholesky(W)
    assert got == info


# ------------------------------------------------------------------ triangular solves and GEMVs

def test_triangular_solves_pascal_inverse(oracle_mod):
    """The lower Pascal triangle L_ij = C(i,j) has inverse (-1)^(i-j) C(i,j)."""
    n = 10
    L = np.array([[math.comb(i, j) if j <= i else 0 for j in range(n)] for i in range(n)], dtype=np.float64)
    Linv = np.array([[(-1) ** (i - j) * math.comb(i, j) if j <= i else 0 for j in range(n)]
                     for i in range(n)], dtype=np.float64)
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        np.testing.assert_array_equal(oracle_mod.forward(L, e), Linv[:, k])
        np.testing.assert_array_equal(oracle_mod.backward(L, e), Linv.T[:, k])


def test_triangular_solves_residual(oracle_mod):
    rng = np.random.default_rng(1)
    n = 50
    L = np.tril(rng.standard_normal((n, n)) * 0.1) + np.diag(1.0 + rng.random(n))
    b = rng.standard_normal(n)
    z = oracle_mod.forward(L, b)
    y = oracle_mod.backward(L, b)
    np.testing.assert_allclose(L @ z, b, atol=1e-12)
    np.testing.assert_allclose(L.T @ y, b, atol=1e-12)


def test_gemv_and_apply_against_blas(oracle_mod):
    S = synth.make_S(33, 9000, 8)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(9000)
    y = rng.standard_normal(33)
    S64 = S.astype(np.float64)
    np.testing.assert_allclose(oracle_mod.gemv(S, v), S64 @ v, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle_mod.apply(S, v, y, 0.3), (v - S64.T @ y) / 0.3, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ closed forms

def test_zero_S_gives_v_over_lambda(oracle_mod):
    S = np.zeros((5, 40), dtype=np.float32)
    v = np.arange(40, dtype=np.float64) - 7.5
    np.testing.assert_array_equal(oracle_mod.solve(S, v, 0.5), v / 0.5)


def test_v_orthogonal_to_rows(oracle_mod):
    """v in the null space of S: S v = 0, hence x = v / lambda."""
    S = synth.make_S(10, 120, 11)
    S64 = S.astype(np.float64)
    g = np.random.default_rng(3).standard_normal(120)
    v = g - S64.T @ np.linalg.lstsq(S64.T, g, rcond=None)[0]
    lam = 1e-3
    x = oracle_mod.solve(S, v, lam)
    np.testing.assert_allclose(x, v / lam, rtol=1e-8, atol=1e-8 * np.abs(v / lam).max())


def test_single_row_sherman_morrison(oracle_mod):
    """n = 1: (s s^T + lambda I)^-1 v = v/lambda - s (s^T v) / (lambda (lambda + |s|^2))."""
    rng = np.random.default_rng(4)
    s = rng.standard_normal(500).astype(np.float32)
    v = rng.standard_normal(500)
    lam = 0.07
    s64 = s.astype(np.float64)
    ref = v / lam - s64 * (s64 @ v) / (lam * (lam + s64 @ s64))
    np.testing.assert_allclose(oracle_mod.solve(s[None, :], v, lam), ref, rtol=1e-11, atol=1e-11)


def test_orthogonal_rows(oracle_mod):
    """Rows with disjoint support: S S^T = diag(d), x = v/lambda - sum_i s_i (s_i^T v)/(lambda (d_i + lambda))."""
    rng = np.random.default_rng(5)
    n, m = 6, 60
    S = np.zeros((n, m), dtype=np.float32)
    for i in range(n):
        S[i, i * 10:(i + 1) * 10] = rng.standard_normal(10)
    v = rng.standard_normal(m)
    lam = 0.01
    S64 = S.astype(np.float64)
    ref = v / lam
    for i in range(n):
        d = S64[i] @ S64[i]
        ref = ref - S64[i] * (S64[i] @ v) / (lam * (d + lam))
    np.testing.assert_allclose(oracle_mod.solve(S, v, lam), ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


# ------------------------------------------------------------------ Proposition 1, Appendices B and C

def test_proposition1_identities(oracle_mod):
    """x from Algorithm 1 satisfies S^T S x + lambda x = v, and S x equals
    y = (S S^T + lambda I)^-1 S v (the intermediate step of the proof)."""
    S = synth.make_S(64, 5000, 12, "scaled")
    v = synth.make_v(S, 12, "iid").astype(np.float64)
    lam = 1e-2
    x, y = oracle_mod.solve(S, v, lam, return_y=True)
    r = oracle_mod.residual(S, v, x, lam)
    S64 = S.astype(np.float64)
    normSS = np.linalg.norm(S64, 2) ** 2
    eta = np.linalg.norm(r) / ((normSS + lam) * np.linalg.norm(x) + np.linalg.norm(v))
    assert eta <= 1e-14
    np.testing.assert_allclose(S64 @ x, y, rtol=1e-8, atol=1e-8 * np.abs(y).max())


def test_appendix_b_structured_rhs(oracle_mod):
    """For v = S^T f, x = S^T (S S^T + lambda I)^-1 f (the equivalence shown in Appendix B)."""
    S = synth.make_S(40, 3000, 13)
    S64 = S.astype(np.float64)
    f = np.random.default_rng(6).standard_normal(40)
    v = S64.T @ f
    lam = 1e-3
    x = oracle_mod.solve(S, v, lam)
    ref = S64.T @ np.linalg.solve(S64 @ S64.T + lam * np.eye(40), f)
    assert _rel(x, ref) <= _cond_tol(S, lam)


def test_appendix_c_svd_formula(oracle_mod):
    """x = V (Sigma^2 + lambda I)^-1 V^T v + (v - V V^T v)/lambda with the thin SVD S = U Sigma V^T."""
    S = synth.make_S(128, 6000, 14, "scaled")
    v = synth.make_v(S, 14, "iid").astype(np.float64)
    lam = 1e-4
    U, s, Vt = np.linalg.svd(S.astype(np.float64), full_matrices=False)
    Vtv = Vt @ v
    ref = Vt.T @ (Vtv / (s ** 2 + lam)) + (v - Vt.T @ Vtv) / lam
    assert _rel(oracle_mod.solve(S, v, lam), ref) <= _cond_tol(S, lam)


# ------------------------------------------------------------------ metamorphic relations

def test_power_of_two_scaling_is_exact(oracle_mod):
    """(2S, 4 lambda, v) -> x/4 exactly: every intermediate scales by a power of two."""
    S = synth.make_S(20, 800, 15)
    v = synth.make_v(S, 15)
    x = oracle_mod.solve(S, v, 1e-2)
    x2 = oracle_mod.solve((2 * S).astype(np.float32), v, 4e-2)
    np.testing.assert_array_equal(x2, x / 4)


def test_permutations(oracle_mod):
    S = synth.make_S(25, 900, 16)
    v = synth.make_v(S, 16).astype(np.float64)
    lam = 1e-3
    x = oracle_mod.solve(S, v, lam)
    rp = np.random.default_rng(7).permutation(25)
    cp = np.random.default_rng(8).permutation(900)
    np.testing.assert_allclose(oracle_mod.solve(S[rp], v, lam), x, rtol=1e-9, atol=1e-9 * np.abs(x).max())
    np.testing.assert_allclose(oracle_mod.solve(S[:, cp], v[cp], lam), x[cp], rtol=1e-9,
                               atol=1e-9 * np.abs(x).max())


def test_duplicated_rows(oracle_mod):
    """A rank-deficient S (duplicated rows) keeps W SPD for lambda > 0."""
    S = synth.make_S(10, 300, 17)
    S2 = np.concatenate([S, S[:4]], axis=0)
    v = synth.make_v(S, 17)
    lam = 1e-2
    assert _rel(oracle_mod.solve(S2, v, lam), _dense_solve(S2, v, lam)) <= _cond_tol(S2, lam)


def test_solve_batched_matches_single(oracle_mod):
    S = synth.make_S(12, 400, 18)
    V = synth.make_V(400, 3, 18)
    lams = [1e-1, 1e-3]
    X = oracle_mod.solve_batched(S, lams, V)
    for li, lam in enumerate(lams):
        for r in range(3):
            np.testing.assert_array_equal(X[li, r], oracle_mod.solve(S, V[r], lam))


# ------------------------------------------------------------------ split-BF16 definition

def test_split_bf16_against_torch_rne(oracle_mod):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(9)
    a = (rng.standard_normal(200_000) * 10.0 ** rng.uniform(-30, 30, 200_000)).astype(np.float32)
    a = np.concatenate([a, np.float32([0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-40, -2e-39])]).astype(np.float32)
    S = a.reshape(1, -1)
    hi, lo = oracle_mod.split_bf16(S)
    t = torch.from_numpy(a)
    hi_t = t.to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(hi[0], hi_t)
    lo_t = (t - torch.from_numpy(hi_t)).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(lo[0], lo_t)


def test_split_bf16_ties_and_remainder(oracle_mod):
    one = 1.0
    vals = np.float32([one + 2 ** -8, one + 3 * 2 ** -8, -(one + 2 ** -8), one + 2 ** -8 + 2 ** -20])
    hi, lo = oracle_mod.split_bf16(vals.reshape(1, -1))
    # ties go to the even significand; a value above the tie rounds up
    np.testing.assert_array_equal(hi[0], np.float32([1.0, 1.0 + 2 ** -6, -1.0, 1.0 + 2 ** -7]))
    S = synth.make_S(3, 1000, 19)
    hi, lo = oracle_mod.split_bf16(S)
    r = S.astype(np.float64) - hi.astype(np.float64)
    assert np.all(np.abs(r) <= np.abs(S.astype(np.float64)) * 2.0 ** -8 * (1 + 1e-12))
    assert np.all(np.abs(r - lo) <= np.abs(r) * 2.0 ** -8 * (1 + 1e-12))


def test_gram3_against_blas(oracle_mod):
    S = synth.make_S(21, 2000, 20)
    hi, lo = oracle_mod.split_bf16(S)
    h, l_ = hi.astype(np.float64), lo.astype(np.float64)
    ref = h @ h.T + h @ l_.T + l_ @ h.T + 0.5 * np.eye(21)
    np.testing.assert_allclose(oracle_mod.gram3(hi, lo, 0.5), ref, rtol=1e-12, atol=1e-12)
    # and it differs from the exact Gram by about the dropped lo*lo term (<= 2^-16 relative)
    W = oracle_mod.gram(S, 0.5)
    dd = np.sqrt(np.outer(np.diag(W), np.diag(W)))
    assert np.max(np.abs(oracle_mod.gram3(hi, lo, 0.5) - W) / dd) <= 2.0 ** -15


def test_gram3_hand_example(oracle_mod):
    """The split and the three-product Gram on a hand-derived example (tests/golden) in which
    lo.lo is nonzero in every entry: exact equality, so keeping the fourth product, dropping a
    cross term or splitting with another rounding each fails."""
    with open(os.path.join(HERE, "golden", "hand_examples.json")) as f:
        g = json.load(f)["split_bf16_gram3"]
    S = np.array(g["S"], dtype=np.float32)
    hi, lo = oracle_mod.split_bf16(S)
    np.testing.assert_array_equal(hi, np.array(g["hi"], dtype=np.float32))
    np.testing.assert_array_equal(lo, np.array(g["lo"], dtype=np.float32))
    W3 = oracle_mod.gram3(hi, lo, g["lambda"])
    np.testing.assert_array_equal(W3, np.array(g["W3"]))
    # the exact Gram is the three-product one plus lo lo^T, to the last bit
    np.testing.assert_array_equal(oracle_mod.gram(S, g["lambda"]), W3 + np.array(g["lolo"]))


# ------------------------------------------------------------------ scaled-FP8 (E4M3 + E8M0) form
def _e4m3_table():
    """Every finite non-negative E4M3 value, from the bit layout: exponent field E (bias 7) and
    mantissa field M; E = 0 is subnormal (M * 2^-9); E = 15, M = 7 is NaN, so 448 is the largest."""
    vals = []
    for E in range(16):
        for M in range(8):
            if E == 15 and M == 7:
                continue
            vals.append(M * 2.0 ** -9 if E == 0 else (1 + M / 8) * 2.0 ** (E - 7))
    return np.array(sorted(set(vals)))


def test_quant_mxfp8_matches_torch_e4m3_cast(oracle_mod):
    """A block whose largest magnitude lies in (224, 448] has scale 2^0, so its codes must equal
    torch's round-to-nearest-even cast to float8_e4m3fn."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    S = (rng.standard_normal((6, 96)) * 60.0).astype(np.float32)
    S[:, ::32] = np.float32(300.0)      # pins every block's maximum into (224, 448]
    S[1, 1:9] = [0.0, -0.0, 2.0 ** -10, 3 * 2.0 ** -10, 1.0625, 1.1875, -440.0, 2.0 ** -7 * 1.0625]
    deq, e = oracle_mod.quant_mxfp8(S)
    assert np.all(e == 0)
    ref = torch.from_numpy(S).to(torch.float8_e4m3fn).to(torch.float32).numpy()
    np.testing.assert_array_equal(deq, ref)


def test_quant_mxfp8_hand_values(oracle_mod):
    """Hand-computed roundings (block scale 2^0): ties go to the even mantissa."""
    S = np.zeros((1, 32), dtype=np.float32)
    S[0, :10] = [448.0, 1.0625, 1.1875, 3 * 2.0 ** -10, 2.0 ** -10, 5 * 2.0 ** -10, 17.0, 19.0, -0.0, -1.0625]
    want = [448.0, 1.0, 1.25, 2 * 2.0 ** -9, 0.0, 2 * 2.0 ** -9, 16.0, 20.0, 0.0, -1.0]
    deq, e = oracle_mod.quant_mxfp8(S)
    assert e[0, 0] == 0
    np.testing.assert_array_equal(deq[0, :10], np.array(want, dtype=np.float32))


def test_quant_mxfp8_scale_is_smallest_power(oracle_mod):
    """Scale exponent: smallest e with amax <= 448 * 2^e (-127 for an all-zero block), and every
    dequantised value is 2^e times a finite E4M3 value nearest to S / 2^e."""
    rng = np.random.default_rng(11)
    n, m = 5, 200
    S = (rng.standard_normal((n, m)) * 10.0 ** rng.uniform(-6, 3, size=(n, 1))).astype(np.float32)
    S[2, 32:64] = 0.0
    S[3, 64:96] = 448.0 * 2.0 ** -20      # amax exactly on a power-of-two boundary
    deq, e = oracle_mod.quant_mxfp8(S)
    table = _e4m3_table()
    for i in range(n):
        for b in range((m + 31) // 32):
            blk = S[i, 32 * b:32 * b + 32].astype(np.float64)
            amax = np.abs(blk).max()
            eb = int(e[i, b])
            if amax == 0.0:
                assert eb == -127
                continue
            assert amax <= 448.0 * 2.0 ** eb and amax > 448.0 * 2.0 ** (eb - 1)
            x = np.abs(blk) / 2.0 ** eb
            q = np.abs(deq[i, 32 * b:32 * b + 32].astype(np.float64)) / 2.0 ** eb
            assert np.all(np.isin(q, table))
            # nearest: no table value is strictly closer than the chosen one
            dist = np.abs(table[None, :] - x[:, None]).min(axis=1)
            np.testing.assert_array_equal(np.abs(q - x), dist)
            assert np.all(np.sign(deq[i, 32 * b:32 * b + 32]) * np.sign(blk) >= 0)
    assert e[3, 2] == -20


def test_quant_mxfp8_power_of_two_scaling(oracle_mod):
    """Scaling S by 2^k shifts every block exponent by k and scales the result exactly."""
    rng = np.random.default_rng(5)
    S = rng.standard_normal((3, 130)).astype(np.float32)
    d1, e1 = oracle_mod.quant_mxfp8(S)
    d2, e2 = oracle_mod.quant_mxfp8(S * np.float32(2.0 ** 13))
    np.testing.assert_array_equal(e2, e1 + 13)
    np.testing.assert_array_equal(d2, d1 * np.float32(2.0 ** 13))
