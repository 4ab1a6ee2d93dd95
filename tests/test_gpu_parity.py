"""GPU parity of every stage of the HIP path against the FP64 CPU oracle, through the C ABI.

Sizes are chosen so the oracle finishes in seconds while the GPU kernels still span several
256 x 256 Gram tiles, several 64-row Cholesky / triangular-solve blocks, several GEMV column
groups, and ragged tails in n, m and the row stride (including a stride that is not a multiple
of 4, which takes the scalar-load path).

Tolerances (derived from the arithmetic):
* Gram (FP32 or split-BF16 products, FP32 accumulation within a k-slice, FP64 across slices):
  max_ij |dW_ij| / sqrt(W_ii W_jj) <= 2e-6 against the oracle's Gram of the same products
  (exact Gram for FP32, the three-product split Gram for BF16x3); the diagonal is FP64.
* FP64 stages (Cholesky, triangular solves, GEMVs with exact FP32 x FP32 products): relative
  errors at the 1e-12 level, scaled by the conditioning where it matters.
* End to end: relative error ||x - x*|| / ||x*|| <= 1e-6 with at least one refinement sweep.
"""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dfl():
    import paper_2310_17556_amd as dfl
    return dfl


@pytest.fixture(scope="module")
def ctx(dfl):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = dfl.dfisher_ctx_create(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def dev_strided(S, ld):
    """Upload S (n x m) into a wider buffer with row stride ld and return the (n, m) view."""
    n, m = S.shape
    buf = torch.full((n, ld), float("nan"), dtype=torch.float32, device="cuda")
    buf[:, :m] = torch.from_numpy(S).cuda()
    return buf[:, :m]


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def scaled_err(W, Wref):
    d = np.sqrt(np.abs(np.outer(np.diag(Wref), np.diag(Wref))))
    return float(np.max(np.abs(W - Wref) / d))


GRAM_SHAPES = [
    # n, m, ld, kind
    (32, 1024, 1024, "iid"),        # smallest workload: one partial tile
    (300, 5000, 5003, "iid"),       # ragged n, stride not a multiple of 4 (scalar loads)
    (513, 20001, 20004, "scaled"),  # 3 tile rows, ragged m and n
    (1, 777, 777, "iid"),           # single row
    (700, 3000, 3072, "iid"),       # 3 tile rows, padded stride
    (257, 4099, 4100, "iid"),       # aligned rows, m mod 8 = 3 (tail left to the reduction), 1-row tile
]


@pytest.mark.parametrize("n,m,ld,kind", GRAM_SHAPES)
def test_gram_fp32(dfl, ctx, oracle_mod, n, m, ld, kind):
    print(f"[gram fp32] n={n} m={m} ld={ld}", flush=True)
    S = synth.make_S(n, m, synth.seed(20, n), kind, center=n > 1)   # one centered row is all zeros
    lam = 1e-3
    W = dfl.dfisher_gram(ctx, dev_strided(S, ld), dfl.DFISHER_GRAM_FP32, lam).cpu().numpy()
    Wref = oracle_mod.gram(S, lam)
    assert np.array_equal(W, W.T)
    np.testing.assert_allclose(np.diag(W), np.diag(Wref), rtol=1e-13)
    assert scaled_err(W, Wref) <= 2e-6


@pytest.mark.parametrize("n,m,ld,kind", GRAM_SHAPES)
def test_gram_bf16x3(dfl, ctx, oracle_mod, n, m, ld, kind):
    print(f"[gram bf16x3] n={n} m={m} ld={ld}", flush=True)
    S = synth.make_S(n, m, synth.seed(21, n), kind, center=n > 1)   # one centered row is all zeros
    W = dfl.dfisher_gram(ctx, dev_strided(S, ld), dfl.DFISHER_GRAM_BF16X3, 0.0).cpu().numpy()
    hi, lo = oracle_mod.split_bf16(S)
    W3 = oracle_mod.gram3(hi, lo, 0.0)
    Wex = oracle_mod.gram(S, 0.0)
    np.fill_diagonal(W3, np.diag(Wex))          # the library's diagonal is the exact row norm
    np.testing.assert_allclose(np.diag(W), np.diag(Wex), rtol=1e-13)
    assert scaled_err(W, W3) <= 2e-6            # same products as the split definition
    assert scaled_err(W, Wex) <= 3e-5           # within the split's 2^-16-level product error


def decode_e4m3(codes):
    """Values of OCP E4M3 codes (1 sign, 4 exponent bits with bias 7, 3 mantissa bits)."""
    c = codes.astype(np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    ex = (c >> 3) & 0xF
    mant = c & 7
    val = np.where(ex == 0, mant * 2.0 ** -9, (1.0 + mant / 8.0) * 2.0 ** (ex - 7))
    return sign * val


MX_SHAPES = [(32, 1024), (300, 5000), (513, 20001), (7, 100), (257, 4160)]


@pytest.mark.parametrize("n,m", MX_SHAPES)
def test_quantize_mxfp8_bit_exact(dfl, ctx, oracle_mod, n, m):
    """The device's E4M3 codes and block exponents equal the oracle's definition exactly."""
    print(f"[quantize mxfp8] n={n} m={m}", flush=True)
    S = synth.make_S(n, m, synth.seed(35, n), "scaled")
    S[0, :5] = [0.0, 448.0 * 2.0 ** -20, -(2.0 ** -30), 1e-38, 3.0]   # ties, tiny and zero values
    codes, scales, ldq = dfl.dfisher_quantize_mxfp8(ctx, dev_strided(S, (m + 3) // 4 * 4))
    codes = codes.cpu().numpy()[:, :m]
    e = scales.cpu().numpy().astype(np.int64)[:, :(m + 31) // 32] - 127
    deq_ref, e_ref = oracle_mod.quant_mxfp8(S)
    assert np.array_equal(e, e_ref)
    deq = decode_e4m3(codes) * 2.0 ** np.repeat(e, 32, axis=1)[:, :m]
    assert np.array_equal(deq.astype(np.float32), deq_ref)


@pytest.mark.parametrize("n,m", MX_SHAPES)
def test_gram_mxfp8(dfl, ctx, oracle_mod, n, m):
    """Scaled-FP8 Gram = Gram of the dequantized S (FP32 accumulation error only); exact diagonal."""
    print(f"[gram mxfp8] n={n} m={m}", flush=True)
    S = synth.make_S(n, m, synth.seed(36, n), "iid")
    W = dfl.dfisher_gram(ctx, dev_strided(S, (m + 3) // 4 * 4), dfl.DFISHER_GRAM_MXFP8, 0.0).cpu().numpy()
    deq, _ = oracle_mod.quant_mxfp8(S)
    # every column's products come from the quantized values; only the diagonal is exact
    Wq = oracle_mod.gram(deq, 0.0)
    Wex = oracle_mod.gram(S, 0.0)
    np.fill_diagonal(Wq, np.diag(Wex))
    np.testing.assert_allclose(np.diag(W), np.diag(Wex), rtol=1e-13)
    # the FP8 matrix-core instruction sums its 64 products with ~2^-20 relative precision
    assert scaled_err(W, Wq) <= 3e-5
    assert scaled_err(W, Wex) <= 0.13       # the scaled-FP8 product error bound


def test_mxfp8_rejects_unaligned_rows(dfl, ctx):
    S = synth.make_S(8, 101, 38)
    with pytest.raises(dfl.DfisherError) as ei:
        dfl.dfisher_gram(ctx, dev(S), dfl.DFISHER_GRAM_MXFP8, 0.0)
    assert ei.value.status == dfl.DFISHER_E_UNSUPPORTED


@pytest.mark.parametrize("n", [1, 5, 64, 65, 130, 1000])
def test_potrf(dfl, ctx, oracle_mod, n):
    print(f"[potrf] n={n}", flush=True)
    S = synth.make_S(n, 3 * n + 7, synth.seed(22, n))
    W = oracle_mod.gram(S, 0.5)
    Lref, info = oracle_mod.cholesky(W)
    assert info == 0
    Wd = dev(W)
    assert dfl.dfisher_potrf(ctx, Wd) == 0
    L = Wd.cpu().numpy()
    assert np.all(np.triu(L, 1) == 0)
    assert rel(L, Lref) <= 1e-12
    assert rel(L @ L.T, W) <= 1e-13


@pytest.mark.parametrize("n,bad", [(130, 71), (70, 1), (200, 200), (64, 64), (65, 65)])
def test_potrf_breakdown_index(dfl, ctx, oracle_mod, n, bad):
    """A matrix whose first non-positive pivot is at a known index: the device reports the same
    1-based index as the oracle (an integer result: exact)."""
    print(f"[potrf breakdown] n={n} bad={bad}", flush=True)
    rng = np.random.default_rng(n + bad)
    A = rng.standard_normal((n, n)) / math.sqrt(n)
    W = A @ A.T + np.eye(n)
    W[bad - 1, bad - 1] -= 1e6          # pivot bad-1 goes negative, earlier ones are untouched
    _, info_ref = oracle_mod.cholesky(W)
    assert info_ref == bad
    assert dfl.dfisher_potrf(ctx, dev(W)) == info_ref
    Wn = W.copy()
    Wn[3 % n, 3 % n] = np.nan
    _, info_nan = oracle_mod.cholesky(Wn)
    assert dfl.dfisher_potrf(ctx, dev(Wn)) == info_nan


def test_potrf_nan_row_in_later_block(dfl, ctx, oracle_mod):
    """A NaN row of S past the first block: the breakdown is found by the diagonal factor that runs
    inside a trailing update (block 1 of 4), at the oracle's 1-based index."""
    n, row = 200, 100
    print(f"[potrf nan row] n={n} row={row}", flush=True)
    S = synth.make_S(n, 3 * n + 7, synth.seed(25, n))
    S[row, 5] = np.nan
    W = oracle_mod.gram(S, 0.5)
    _, info_ref = oracle_mod.cholesky(W)
    assert info_ref == row + 1
    assert dfl.dfisher_potrf(ctx, dev(W)) == info_ref


@pytest.mark.parametrize("n", [1, 63, 64, 65, 300, 2000])
def test_trsv(dfl, ctx, oracle_mod, n):
    print(f"[trsv] n={n}", flush=True)
    S = synth.make_S(n, 2 * n + 3, synth.seed(23, n))
    L, info = oracle_mod.cholesky(oracle_mod.gram(S, 1.0))
    assert info == 0
    b = np.random.default_rng(n).standard_normal(n)
    Ld = dev(L)
    z = dfl.dfisher_trsv(ctx, Ld, dev(b), 0).cpu().numpy()
    y = dfl.dfisher_trsv(ctx, Ld, dev(b), 1).cpu().numpy()
    assert rel(z, oracle_mod.forward(L, b)) <= 1e-12
    assert rel(y, oracle_mod.backward(L, b)) <= 1e-12
    # in place (b and y alias)
    bd = dev(b)
    dfl.dfisher_trsv(ctx, Ld, bd, 0, y=bd)
    assert rel(bd.cpu().numpy(), oracle_mod.forward(L, b)) <= 1e-12


@pytest.mark.parametrize("n,m,ld", [(32, 1024, 1024), (300, 50001, 50004), (77, 2049, 2051), (1000, 40000, 40000)])
def test_gemv(dfl, ctx, oracle_mod, n, m, ld):
    print(f"[gemv] n={n} m={m} ld={ld}", flush=True)
    S = synth.make_S(n, m, synth.seed(24, n), "scaled")
    v = synth.make_v(S, synth.seed(24, n))
    b = dfl.dfisher_gemv(ctx, dev_strided(S, ld), dev(v)).cpu().numpy()
    bref = oracle_mod.gemv(S, v)
    # products of FP32 values are exact in FP64: only the summation order differs
    scale = np.abs(S.astype(np.float64)) @ np.abs(v.astype(np.float64))
    assert np.all(np.abs(b - bref) <= 1e-13 * scale + 1e-300)


@pytest.mark.parametrize("n,m,ld", [(32, 1024, 1024), (300, 50001, 50004), (1000, 3000, 3001)])
def test_apply(dfl, ctx, oracle_mod, n, m, ld):
    print(f"[apply] n={n} m={m} ld={ld}", flush=True)
    S = synth.make_S(n, m, synth.seed(25, n))
    v = synth.make_v(S, synth.seed(25, n))
    y = np.random.default_rng(n).standard_normal(n)
    lam = 1e-3
    x64 = dfl.dfisher_apply(ctx, dev_strided(S, ld), dev(v), dev(y), lam, x_fp64=True).cpu().numpy()
    xref = oracle_mod.apply(S, v, y, lam)
    scale = (np.abs(v.astype(np.float64)) + np.abs(S.astype(np.float64)).T @ np.abs(y)) / lam
    assert np.all(np.abs(x64 - xref) <= 1e-13 * scale)
    x32 = dfl.dfisher_apply(ctx, dev_strided(S, ld), dev(v), dev(y), lam).cpu().numpy()
    assert np.all(np.abs(x32.astype(np.float64) - xref) <= 2.0 ** -24 * np.abs(xref) + 1e-13 * scale)


SOLVE_CASES = [
    # n, m, lam, prec, sweeps, kind, bound
    (32, 1024, 1e-2, 0, 0, "iid", 1e-5),       # the smallest workload, plain FP32 path
    (32, 1024, 1e-2, 0, 1, "iid", 1e-6),
    (32, 1024, 1e-2, 1, 1, "iid", 1e-6),
    (300, 20001, 1e-2, 1, 1, "iid", 1e-6),
    (300, 20001, 1e-4, 1, 2, "iid", 1e-6),
    (300, 20001, 1e-6, 1, 2, "iid", 1e-6),
    (257, 30000, 1e-3, 0, 1, "scaled", 1e-6),   # row-space-heavy v (cancellation in v - S^T y)
    (257, 30000, 1e-3, 1, 2, "scaled", 1e-6),
    (600, 12000, 1e-4, 0, 2, "iid", 1e-6),
    (300, 20000, 1e-2, 2, 4, "iid", 1e-6),      # scaled-FP8 Gram + refinement (m/n = 67: slow contraction)
    (300, 20000, 1e-6, 2, 3, "iid", 1e-6),
    (257, 30000, 1e-3, 2, 3, "iid", 1e-6),
    # 16-byte aligned rows: the refinement product S S^T y takes the fused one-read pass (also in
    # the aligned cases above, n = 300 and 257 with a partial last row group)
    (320, 20004, 1e-2, 2, 4, "iid", 1e-6),      # m % 16 = 4: the last columns in the tail group
    (320, 20016, 1e-6, 2, 3, "iid", 1e-6),      # whole 16-column blocks only
    (320, 20008, 1e-3, 0, 1, "scaled", 1e-6),
    (1040, 9000, 1e-3, 1, 2, "iid", 1e-6),      # 8 loads per lane and block
    (2064, 5004, 1e-3, 1, 2, "iid", 1e-6),      # 16 loads per lane, rows past n in the last load
    (4200, 5000, 1e-2, 1, 1, "iid", 1e-6),      # n > 4096: the two-pass refinement product
    (40, 20, 1e-2, 0, 1, "iid", 1e-6),          # m < 32: one partial 32-column block in the fused pass
]


@pytest.mark.parametrize("n,m,lam,prec,sweeps,kind,bound", SOLVE_CASES)
def test_solve(dfl, ctx, oracle_mod, n, m, lam, prec, sweeps, kind, bound):
    print(f"[solve] n={n} m={m} lam={lam} prec={prec} sweeps={sweeps} kind={kind}", flush=True)
    S = synth.make_S(n, m, synth.seed(26, n), kind)
    v = synth.make_v(S, synth.seed(26, n), kind)
    xref = oracle_mod.solve(S, v, lam)
    policy = dfl.DFISHER_SHIFT_ALWAYS if prec == 2 else dfl.DFISHER_SHIFT_ON_FAILURE
    x, info = dfl.dfisher_solve(ctx, dev(S), dev(v), lam, gram_prec=prec, sweeps=sweeps, shift_policy=policy,
                                x_fp64=True)
    err = rel(x.cpu().numpy(), xref)
    print(f"    rel err {err:.3e}  info {info}", flush=True)
    assert info["sweeps_done"] == sweeps
    assert err <= bound
    # FP32 output: the same solution rounded once
    x32, _ = dfl.dfisher_solve(ctx, dev(S), dev(v), lam, gram_prec=prec, sweeps=sweeps, shift_policy=policy)
    assert rel(x32.cpu().numpy(), xref) <= bound + 2.0 ** -23


@pytest.mark.parametrize("lam", [1e-2, 1e-6])
def test_solve_fp8_unshifted(dfl, ctx, oracle_mod, lam):
    """Scaled-FP8 Gram under the default policy (shift only on failure) at m/n = 1024, the aspect
    ratio of the full-size workload: one refinement sweep reaches the 1e-6 target."""
    n, m = 128, 131072
    print(f"[solve fp8 on-failure] n={n} m={m} lam={lam}", flush=True)
    S = synth.make_S(n, m, synth.seed(31, n), "iid")
    v = synth.make_v(S, synth.seed(31, n), "iid")
    xref = oracle_mod.solve(S, v, lam)
    x, info = dfl.dfisher_solve(ctx, dev(S), dev(v), lam, gram_prec=dfl.DFISHER_GRAM_MXFP8, sweeps=1, x_fp64=True)
    err = rel(x.cpu().numpy(), xref)
    print(f"    rel err {err:.3e}  info {info}", flush=True)
    assert err <= 1e-6


def test_solve_tolerance(dfl, ctx, oracle_mod):
    """opt.tol: the sweeps stop once a measured relative residual |b - W y| / |b| meets tol (sweeps
    is the cap); an unreachable tol returns DFISHER_E_NOT_CONVERGED with x still written. Split-BF16
    Gram (each sweep contracts the residual by orders of magnitude, down to the FP64 floor)."""
    n, m, lam = 320, 20016, 1e-2
    print(f"[solve tol] n={n} m={m} lam={lam}", flush=True)
    S = synth.make_S(n, m, synth.seed(34, n))
    v = synth.make_v(S, synth.seed(34, n))
    xref = oracle_mod.solve(S, v, lam)
    Sd, vd = dev(S), dev(v)
    x, info = dfl.dfisher_solve(ctx, Sd, vd, lam, gram_prec=1, sweeps=16, x_fp64=True, tol=1e-12)
    print(f"    tol 1e-12: {info}", flush=True)
    assert info["converged"] and 1 <= info["sweeps_done"] <= 16 and 0.0 <= info["resid"] <= 1e-12
    assert rel(x.cpu().numpy(), xref) <= 1e-6
    # a loose tolerance stops after the first measured residual
    _, infl = dfl.dfisher_solve(ctx, Sd, vd, lam, gram_prec=1, sweeps=16, tol=1.0)
    assert infl["converged"] and infl["sweeps_done"] == 1
    # fixed sweeps measure nothing
    _, info0 = dfl.dfisher_solve(ctx, Sd, vd, lam, gram_prec=1, sweeps=2)
    assert info0["resid"] == -1.0 and info0["converged"] and info0["sweeps_done"] == 2
    # unreachable tolerance: every allowed sweep runs, the result equals the fixed-sweep one
    x1, info1 = dfl.dfisher_solve(ctx, Sd, vd, lam, gram_prec=1, sweeps=1, x_fp64=True, tol=1e-30)
    assert not info1["converged"] and info1["sweeps_done"] == 1 and info1["resid"] > 1e-30
    x1b, _ = dfl.dfisher_solve(ctx, Sd, vd, lam, gram_prec=1, sweeps=1, x_fp64=True)
    assert torch.equal(x1, x1b)
    # the residual contracts from sweep to sweep
    _, info3 = dfl.dfisher_solve(ctx, Sd, vd, lam, gram_prec=1, sweeps=3, tol=1e-30)
    print(f"    rho after 1 and 3 sweeps: {info1['resid']:.3e} {info3['resid']:.3e}", flush=True)
    assert info3["sweeps_done"] == 3 and info3["resid"] < info1["resid"]


@pytest.mark.parametrize("n", [300, 320])   # two-pass and fused refinement products
def test_solve_deterministic(dfl, ctx, n):
    S = synth.make_S(n, 20004, 27)
    v = synth.make_v(S, 27)
    Sd, vd = dev(S), dev(v)
    x1, _ = dfl.dfisher_solve(ctx, Sd, vd, 1e-3, gram_prec=1, sweeps=1)
    x2, _ = dfl.dfisher_solve(ctx, Sd, vd, 1e-3, gram_prec=1, sweeps=1)
    assert torch.equal(x1, x2)


def test_solve_x_aliases_v(dfl, ctx, oracle_mod):
    S = synth.make_S(64, 4096, 28)
    v = synth.make_v(S, 28)
    xref = oracle_mod.solve(S, v, 1e-2)
    vd = dev(v)
    dfl.dfisher_solve(ctx, dev(S), vd, 1e-2, sweeps=1, x=vd)
    assert rel(vd.cpu().numpy(), xref) <= 1e-6


@pytest.mark.parametrize("n,ld", [(200, 10001), (208, 10004)])   # two-pass / fused refinement product
def test_solve_strided_S(dfl, ctx, oracle_mod, n, ld):
    S = synth.make_S(n, 9999, 29)
    v = synth.make_v(S, 29)
    xref = oracle_mod.solve(S, v, 1e-3)
    x, _ = dfl.dfisher_solve(ctx, dev_strided(S, ld), dev(v), 1e-3, sweeps=1, x_fp64=True)
    assert rel(x.cpu().numpy(), xref) <= 1e-6


def test_factor_reuse(dfl, ctx, oracle_mod):
    S = synth.make_S(200, 10000, 30)
    V = synth.make_V(10000, 3, 30)
    lam = 1e-3
    Sd = dev(S)
    f, info = dfl.dfisher_factor_create(ctx, Sd, lam, gram_prec=1, sweeps=1, x_fp64=True)
    X = dfl.dfisher_factor_solve(f, dev(V)).cpu().numpy()
    for r in range(3):
        assert rel(X[r], oracle_mod.solve(S, V[r], lam)) <= 1e-6
    # the factor is Cholesky of the (BF16x3) Gram + lambda: compare with the oracle's factor
    L = dfl.dfisher_factor_copy_L(f).cpu().numpy()
    Lref, _ = oracle_mod.cholesky(oracle_mod.gram(S, lam))
    assert rel(L, Lref) <= 1e-4
    # the one-shot solve forms the same Gram and factor (deterministic kernels); its passes over S
    # sum in another order than the multi-vector ones, so the two agree to rounding level
    x1, _ = dfl.dfisher_solve(ctx, Sd, dev(V[1]), lam, gram_prec=1, sweeps=1, x_fp64=True)
    assert rel(x1.cpu().numpy(), X[1]) <= 1e-10
    dfl.dfisher_factor_destroy(f)


def test_batched(dfl, ctx, oracle_mod):
    n, m = 150, 8000
    S = synth.make_S(n, m, 31)
    V = synth.make_V(m, 2, 31)
    lams = [1e-6, 1e-4, 1e-1]
    X, infos = dfl.dfisher_solve_batched(ctx, dev(S), lams, dev(V), gram_prec=1, sweeps=2, x_fp64=True)
    Xref = oracle_mod.solve_batched(S, lams, V)
    X = X.cpu().numpy()
    for li in range(len(lams)):
        for r in range(2):
            err = rel(X[li, r], Xref[li, r])
            print(f"    lam={lams[li]} rhs={r} rel err {err:.3e} info {infos[li]}", flush=True)
            assert err <= 1e-6


@pytest.mark.parametrize("n,m,ld,nlam,nrhs,prec,sweeps,policy", [
    (200, 12001, 12001, 5, 3, 1, 2, "on_failure"),   # 15 vectors: one ragged group of 16; unaligned rows
    (96, 8192, 8200, 2, 9, 0, 1, "on_failure"),      # 18 vectors: a full and a ragged group, padded stride
    (128, 9000, 9000, 2, 17, 1, 1, "on_failure"),    # 34 vectors; 17 right-hand sides: S V in two passes
    (64, 7001, 7001, 4, 12, 1, 2, "on_failure"),     # 48 vectors: a two-group pass, then one group; odd stride
    (5, 3001, 3004, 3, 6, 1, 1, "on_failure"),       # fewer rows than one 16-row tile, padded stride
    (1, 2000, 2000, 2, 2, 2, 1, "on_failure"),       # n = 1 with the scaled-FP8 Gram
    (256, 65536, 65536, 3, 2, 2, 3, "always"),       # scaled-FP8 Gram with the up-front shift
])
def test_batched_groups(dfl, ctx, oracle_mod, n, m, ld, nlam, nrhs, prec, sweeps, policy):
    """Every (lambda, rhs) pair of the multi-vector path matches Algorithm 1 run on its own."""
    print(f"[batched] n={n} m={m} ld={ld} nlam={nlam} nrhs={nrhs} prec={prec} sweeps={sweeps} {policy}", flush=True)
    S = synth.make_S(n, m, synth.seed(38, n), "iid")
    V = synth.make_V(m, nrhs, synth.seed(38, n))
    lams = list(np.logspace(-6, -1, nlam))
    pol = dfl.DFISHER_SHIFT_ALWAYS if policy == "always" else dfl.DFISHER_SHIFT_ON_FAILURE
    Vd = dev_strided(V, m + 5)                      # row stride of V not equal to m
    X, infos = dfl.dfisher_solve_batched(ctx, dev_strided(S, ld), lams, Vd, gram_prec=prec, sweeps=sweeps,
                                         shift_policy=pol, x_fp64=True)
    Xref = oracle_mod.solve_batched(S, lams, V)
    X = X.cpu().numpy()
    for li in range(nlam):
        assert infos[li]["potrf_info"] == 0 and infos[li]["sweeps_done"] == sweeps
        for r in range(nrhs):
            err = rel(X[li, r], Xref[li, r])
            assert err <= 1e-6, (li, r, err, infos[li])
    X32, _ = dfl.dfisher_solve_batched(ctx, dev_strided(S, ld), lams, Vd, gram_prec=prec, sweeps=sweeps,
                                       shift_policy=pol)
    assert rel(X32.cpu().numpy(), Xref) <= 1e-6 + 2.0 ** -23


def test_batched_huge_row_stride(dfl, ctx, oracle_mod):
    """A row stride beyond 2^25 floats (padding NaN): the multi-vector row pass over T takes its
    vector-ALU form (16 row strides do not fit a 32-bit buffer offset) and the refinement runs as a
    column pass plus a row pass instead of the fused one; every (lambda, rhs) pair still matches
    Algorithm 1 run on its own."""
    n, m, ld = 40, 3000, (1 << 25) + 64
    print(f"[batched huge stride] n={n} m={m} ld={ld}", flush=True)
    S = synth.make_S(n, m, synth.seed(40, n), "iid")
    V = synth.make_V(m, 3, synth.seed(40, n))
    lams = [1e-5, 1e-2]
    Sd = dev_strided(S, ld)
    X, infos = dfl.dfisher_solve_batched(ctx, Sd, lams, dev(V), gram_prec=1, sweeps=2, x_fp64=True)
    Xref = oracle_mod.solve_batched(S, lams, V)
    X = X.cpu().numpy()
    for li in range(len(lams)):
        assert infos[li]["potrf_info"] == 0
        for r in range(3):
            assert rel(X[li, r], Xref[li, r]) <= 1e-6, (li, r)
    del Sd
    torch.cuda.empty_cache()


def test_factor_solve_many(dfl, ctx, oracle_mod):
    """Factor reuse with 19 right-hand sides (two groups of the multi-vector passes)."""
    n, m, lam = 160, 9000, 1e-4
    S = synth.make_S(n, m, synth.seed(39, n))
    V = synth.make_V(m, 19, synth.seed(39, n))
    f, _ = dfl.dfisher_factor_create(ctx, dev(S), lam, gram_prec=1, sweeps=2, x_fp64=True)
    X = dfl.dfisher_factor_solve(f, dev(V)).cpu().numpy()
    dfl.dfisher_factor_destroy(f)
    for r in range(19):
        assert rel(X[r], oracle_mod.solve(S, V[r], lam)) <= 1e-6


def test_uneven(dfl, ctx, oracle_mod):
    shapes = [(40, 3000, 1e-3), (300, 9000, 1e-5), (1, 500, 1e-2), (129, 7777, 3e-4)]
    Ss = [synth.make_S(n, m, synth.seed(32, p)) for p, (n, m, _) in enumerate(shapes)]
    vs = [synth.make_v(S, synth.seed(32, p)) for p, S in enumerate(Ss)]
    xs, infos = dfl.dfisher_solve_uneven(ctx, [dev(S) for S in Ss], [dev(v) for v in vs], [s[2] for s in shapes],
                                         gram_prec=1, sweeps=2, x_fp64=True)
    for p, (S, v, (_, _, lam)) in enumerate(zip(Ss, vs, shapes)):
        err = rel(xs[p].cpu().numpy(), oracle_mod.solve(S, v, lam))
        print(f"    problem {p} rel err {err:.3e}", flush=True)
        assert err <= 1e-6


UNEVEN_SHAPES = [(256, 20000, 1e-3), (40, 3000, 1e-2), (700, 30001, 1e-5), (1, 512, 1e-2), (129, 7777, 3e-4),
                 (512, 16384, 1e-4), (48, 1000, 1e-2)]


def _uneven_inputs(shapes, seed_base, aligned):
    Ss = [synth.make_S(n, m, synth.seed(seed_base, p)) for p, (n, m, _) in enumerate(shapes)]
    vs = [synth.make_v(S, synth.seed(seed_base, p)) for p, S in enumerate(Ss)]
    Sd = [dev_strided(S, (S.shape[1] + 3) // 4 * 4) if aligned else dev(S) for S in Ss]
    return Ss, vs, Sd, [dev(v) for v in vs]


@pytest.mark.parametrize("prec,sweeps,policy", [(1, 2, "on_failure"), (2, 4, "always"), (0, 1, "on_failure")])
def test_uneven_grouped(dfl, ctx, oracle_mod, prec, sweeps, policy):
    """Problems of different sizes through the grouped path each match Algorithm 1 on their own."""
    print(f"[uneven] prec={prec} sweeps={sweeps} {policy}", flush=True)
    Ss, vs, Sd, vd = _uneven_inputs(UNEVEN_SHAPES, 40 + prec, aligned=True)
    pol = dfl.DFISHER_SHIFT_ALWAYS if policy == "always" else dfl.DFISHER_SHIFT_ON_FAILURE
    lams = [s[2] for s in UNEVEN_SHAPES]
    xs, infos = dfl.dfisher_solve_uneven(ctx, Sd, vd, lams, gram_prec=prec, sweeps=sweeps, shift_policy=pol,
                                         x_fp64=True)
    for p, (S, v, lam) in enumerate(zip(Ss, vs, lams)):
        err = rel(xs[p].cpu().numpy(), oracle_mod.solve(S, v, lam))
        print(f"    problem {p} {S.shape} rel err {err:.3e} info {infos[p]}", flush=True)
        assert err <= 1e-6
        assert infos[p]["sweeps_done"] == sweeps


def test_uneven_breakdown_stays_in_its_problem(dfl, ctx, oracle_mod):
    """One problem of an uneven call has a NaN row in its second block: with no shift policy it
    reports its 1-based pivot index (found by the diagonal factor inside the grouped update) and
    the call returns DFISHER_E_NOT_SPD, while the problems that share every grouped launch with it
    still match Algorithm 1."""
    shapes = [(200, 20000, 1e-3), (300, 24000, 1e-2), (150, 16000, 1e-4)]
    bad, row = 1, 100
    print(f"[uneven breakdown] {shapes} problem {bad} row {row}", flush=True)
    Ss, vs = [], []
    for k, (n, m, _) in enumerate(shapes):
        S = synth.make_S(n, m, synth.seed(77, k), "iid", center=False)
        v = synth.make_v(S, synth.seed(77, k), "iid")
        if k == bad:
            S[row, 7] = np.nan
        Ss.append(S)
        vs.append(v)
    lams = [s[2] for s in shapes]
    with pytest.raises(dfl.DfisherError) as ei:
        dfl.dfisher_solve_uneven(ctx, [dev(S) for S in Ss], [dev(v) for v in vs], lams, gram_prec=0, sweeps=1,
                                 shift_policy=dfl.DFISHER_SHIFT_NONE, x_fp64=True)
    assert ei.value.status == dfl.DFISHER_E_NOT_SPD
    infos, xs = ei.value.infos, ei.value.xs
    assert infos[bad]["potrf_info"] == row + 1
    for k, (S, v, lam) in enumerate(zip(Ss, vs, lams)):
        if k == bad:
            continue
        assert infos[k]["potrf_info"] == 0
        xref = oracle_mod.solve(S, v, lam)
        assert rel(xs[k].cpu().numpy(), xref) <= 1e-6, k


def test_uneven_graph_replays_match_eager(dfl, ctx):
    """The captured graph, replayed with other work and synchronisations in between, gives the
    eager result bit for bit on every replay."""
    shapes = UNEVEN_SHAPES[:4]
    _, _, Sd, vd = _uneven_inputs(shapes, 44, aligned=True)
    lams = [s[2] for s in shapes]
    dfl.dfisher_ctx_enable_graphs(ctx, False)
    x_eager, _ = dfl.dfisher_solve_uneven(ctx, Sd, vd, lams, gram_prec=2, sweeps=1, x_fp64=True)
    x_eager = [x.clone() for x in x_eager]
    dfl.dfisher_ctx_enable_graphs(ctx, True)
    xs = [torch.empty_like(x) for x in x_eager]
    other_S = dev(synth.make_S(64, 4096, 45))
    other_v = dev(synth.make_v(synth.make_S(64, 4096, 45), 45))
    for rep in range(3):
        for x in xs:
            x.fill_(float("nan"))
        dfl.dfisher_solve_uneven(ctx, Sd, vd, lams, gram_prec=2, sweeps=1, x_fp64=True, xs=xs)
        torch.cuda.synchronize()
        for p in range(len(shapes)):
            assert torch.equal(xs[p], x_eager[p]), (rep, p)
        dfl.dfisher_solve(ctx, other_S, other_v, 1e-2, sweeps=1)   # eager work in between
        torch.cuda.synchronize()


def test_uneven_graph_after_tuning_change(dfl, oracle_mod, tmp_path):
    """Loading a tuning table that changes a problem's split-K factor moves the uneven layout; the
    next call with the same arguments must not replay the graph captured with the old layout."""
    shapes = [(300, 40000, 1e-3), (129, 7777, 3e-4), (40, 3000, 1e-2)]
    Ss, vs, Sd, vd = _uneven_inputs(shapes, 47, aligned=True)
    lams = [s[2] for s in shapes]
    c = dfl.dfisher_ctx_create(0)
    dfl.dfisher_ctx_enable_graphs(c, True)
    path = tmp_path / "tune.txt"
    try:
        xs = [torch.empty(S.shape[1], dtype=torch.float64, device="cuda") for S in Ss]
        for q in (2, 1, 2):   # the (split-BF16, 2 tile rows, m in [2^15, 2^16), aligned) class
            path.write_text(f"1 2 15 1 {q} 1\n")
            dfl.dfisher_ctx_load_tuning(c, str(path))
            for x in xs:
                x.fill_(float("nan"))
            dfl.dfisher_solve_uneven(c, Sd, vd, lams, gram_prec=1, sweeps=2, x_fp64=True, xs=xs)
            torch.cuda.synchronize()
            for p, (S, v, lam) in enumerate(zip(Ss, vs, lams)):
                err = rel(xs[p].cpu().numpy(), oracle_mod.solve(S, v, lam))
                print(f"    q={q} problem {p} rel err {err:.3e}", flush=True)
                assert err <= 1e-6
    finally:
        dfl.dfisher_ctx_destroy(c)


def test_autotune_save_load(dfl, oracle_mod, tmp_path):
    """Tuning a size class records a valid (q, mode); a saved table loads into a fresh context,
    whose solves stay within the bound; automatic tuning adds unseen classes; bad files fail."""
    n, m, lam = 300, 40000, 1e-3
    S = synth.make_S(n, m, synth.seed(46, n))
    v = synth.make_v(S, synth.seed(46, n))
    Sd, vd = dev(S), dev(v)
    c1 = dfl.dfisher_ctx_create(0)
    dfl.dfisher_autotune_gram(c1, Sd, dfl.DFISHER_GRAM_BF16X3)
    path = str(tmp_path / "tune.txt")
    dfl.dfisher_ctx_save_tuning(c1, path)
    rows = [l.split() for l in open(path) if not l.startswith("#")]
    assert len(rows) == 1
    prec, tiles, lg, al, q, mode = map(int, rows[0])
    assert (prec, tiles, lg, al) == (1, 2, 15, 1) and 1 <= q <= 64 and mode in (0, 1)
    c2 = dfl.dfisher_ctx_create(0)
    dfl.dfisher_ctx_load_tuning(c2, path)
    x, _ = dfl.dfisher_solve(c2, Sd, vd, lam, gram_prec=1, sweeps=2, x_fp64=True)
    assert rel(x.cpu().numpy(), oracle_mod.solve(S, v, lam)) <= 1e-6
    dfl.dfisher_ctx_enable_autotune(c2, True)
    S2 = synth.make_S(64, 8192, synth.seed(46, 64))
    v2 = synth.make_v(S2, synth.seed(46, 64))
    x2, _ = dfl.dfisher_solve(c2, dev(S2), dev(v2), 1e-2, gram_prec=2, sweeps=4, x_fp64=True,
                              shift_policy=dfl.DFISHER_SHIFT_ALWAYS)
    assert rel(x2.cpu().numpy(), oracle_mod.solve(S2, v2, 1e-2)) <= 1e-6
    dfl.dfisher_ctx_save_tuning(c2, path)
    assert len([l for l in open(path) if not l.startswith("#")]) == 2
    bad = tmp_path / "bad.txt"
    bad.write_text("1 2 15 1 99 0\n")
    with pytest.raises(dfl.DfisherError):
        dfl.dfisher_ctx_load_tuning(c2, str(bad))
    dfl.dfisher_ctx_destroy(c1)
    dfl.dfisher_ctx_destroy(c2)


def test_shift_always_contracts(dfl, ctx, oracle_mod):
    """With the up-front shift every sweep shrinks the error (the factored matrix dominates W)."""
    S = synth.make_S(300, 20000, 37)
    v = synth.make_v(S, 37)
    xref = oracle_mod.solve(S, v, 1e-6)
    errs = []
    for sweeps in range(3):
        x, info = dfl.dfisher_solve(ctx, dev(S), dev(v), 1e-6, gram_prec=2, sweeps=sweeps,
                                    shift_policy=dfl.DFISHER_SHIFT_ALWAYS, x_fp64=True)
        errs.append(rel(x.cpu().numpy(), xref))
        assert info["shift"] > 0 and info["attempts"] == 1
    print(f"    errors by sweep {errs}", flush=True)
    assert errs[1] < errs[0] and errs[2] <= max(errs[1], 1e-12) * 1.01


def test_nan_input_reports_not_spd(dfl, ctx):
    S = synth.make_S(64, 1000, 33)
    S[5, 17] = np.nan
    v = synth.make_v(S, 33)
    for policy in (dfl.DFISHER_SHIFT_NONE, dfl.DFISHER_SHIFT_ON_FAILURE):
        with pytest.raises(dfl.DfisherError) as ei:
            dfl.dfisher_solve(ctx, dev(S), dev(v), 1e-2, shift_policy=policy)
        assert ei.value.status == dfl.DFISHER_E_NOT_SPD


def test_stage_timing(dfl, ctx):
    S = synth.make_S(300, 20001, 34)
    v = synth.make_v(S, 34)
    dfl.dfisher_ctx_enable_timing(ctx, True)
    dfl.dfisher_solve(ctx, dev(S), dev(v), 1e-3, sweeps=1)
    t = dfl.dfisher_ctx_last_timing(ctx)
    dfl.dfisher_ctx_enable_timing(ctx, False)
    assert t["gram_ms"] > 0 and t["total_ms"] >= t["gram_ms"]


def test_full_size_bench_workload(dfl, ctx, oracle_mod):
    """The workload bench.py times, at full size and in its launch configuration (n = 4096,
    m = 4M, scaled-FP8 Gram, one refinement sweep, shift on failure, lambda = 1e-6). The reference
    x is formed from FP64 products on the device (torch, independent of the library); it is pinned
    to the oracle on sampled Gram entries and sampled outputs, each of which the oracle computes
    one dot product at a time, and its y is checked against the definition W y = S v."""
    n, m, lam = 4096, 4_000_000, 1e-6
    dv = torch.device("cuda:0")
    print(f"[full size] n={n} m={m} lam={lam}: generating", flush=True)
    S = synth.make_S_torch(n, m, synth.seed(3), dv, kind="iid")
    v = synth.make_v_torch(S, synth.seed(3), kind="iid")
    x, info = dfl.dfisher_solve(ctx, S, v, lam, gram_prec=dfl.DFISHER_GRAM_MXFP8, sweeps=1, x_fp64=True)
    torch.cuda.synchronize()
    print(f"    solved: {info}; FP64 reference", flush=True)
    chunk = 131072
    G = torch.zeros((n, n), dtype=torch.float64, device=dv)
    b = torch.zeros(n, dtype=torch.float64, device=dv)
    v64 = v.double()
    for c0 in range(0, m, chunk):
        blk = S[:, c0:c0 + chunk].double()
        G += blk @ blk.T
        b += blk @ v64[c0:c0 + chunk]
        del blk
    W = G + lam * torch.eye(n, dtype=torch.float64, device=dv)
    y = torch.cholesky_solve(b[:, None], torch.linalg.cholesky(W))[:, 0]
    assert float(torch.linalg.norm(W @ y - b) / torch.linalg.norm(b)) <= 1e-9
    xref = torch.empty(m, dtype=torch.float64, device=dv)
    for c0 in range(0, m, chunk):
        xref[c0:c0 + chunk] = (v64[c0:c0 + chunk] - S[:, c0:c0 + chunk].double().T @ y) / lam
    err = float(torch.linalg.norm(x - xref) / torch.linalg.norm(xref))
    print(f"    rel err vs FP64 reference {err:.3e}", flush=True)
    assert err <= 1e-6
    # pins: sampled Gram entries (one 4M-term dot product each) and sampled outputs
    rng = np.random.default_rng(11)
    ii, jj = rng.integers(0, n, 6), rng.integers(0, n, 6)
    rows = np.unique(np.concatenate([ii, jj]))
    pos = {int(r): k for k, r in enumerate(rows)}
    Srows = S[torch.from_numpy(rows).to(dv)].cpu().numpy()
    ent = oracle_mod.gram_entries(Srows, [pos[int(i)] for i in ii], [pos[int(j)] for j in jj])
    Gh = G.cpu().numpy()
    d = np.sqrt(np.diag(Gh)[ii] * np.diag(Gh)[jj])
    assert np.all(np.abs(Gh[ii, jj] - ent) <= 1e-12 * d)
    J = np.sort(rng.choice(m, 512, replace=False))
    Jt = torch.from_numpy(J).to(dv)
    xJ = oracle_mod.apply(S[:, Jt].cpu().numpy(), v[Jt].cpu().numpy(), y.cpu().numpy(), lam)
    assert rel(xref[Jt].cpu().numpy(), xJ) <= 1e-12
    assert rel(x[Jt].cpu().numpy(), xJ) <= 1e-6
    del S, v, x, xref, G, W
    torch.cuda.empty_cache()
