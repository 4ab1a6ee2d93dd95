"""The final step x = (v - S^T y) / lambda with the last refinement correction taken through the
scaled-FP8 copy of S (apply8.hip), through the C ABI.

* Against the FP64 oracle (Algorithm 1, plain definition): the solve with the FP8 final step meets
  1e-6 in ||x - x*|| / ||x*|| and in eps_Sy = lambda ||x - x*|| / ||v - lambda x*|| on a centered S at
  m/n = 1000 with two sweeps, for a small and a large lambda, with a ragged m (a partial 64-column
  block of codes), FP32 and FP64 output.
* That the FP8 step was taken (x differs from the call with DFISHER_EXACT_APPLY) and how far it moves x
  from the exact step: eps <= 2e-7 of |S^T y| (the device test allows an estimated 1e-7), for the three
  whole-line pass shapes (n <= 512, n <= 1024, the row halves split over workgroup pairs) and a
  non-centered S.
* That it is refused where the correction is large (one sweep): x then equals the exact step's bit for
  bit.
* The uneven call: every problem keeps its codes and takes the FP8 final step where the device allows
  it; each problem against the oracle (1e-6) and against the exact final pass (2e-7), eager and as a
  graph replay (bitwise equal); the sizes cover the three classes of the grouped refinement passes.
* The batched call: every (lambda, rhs) pair's correction through the codes in one bf16 matrix-core
  product, against the oracle (1e-6) and the exact final passes (2e-7), for one and several groups of
  16 vectors, ragged m and n, FP32 and FP64 x; refused for every pair when one pair's correction is too
  large (one sweep): then bitwise the exact passes' result.
"""
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


def dev_aligned(S):
    n, m = S.shape
    ld = (m + 3) // 4 * 4
    buf = torch.zeros((n, ld), dtype=torch.float32, device="cuda")
    buf[:, :m] = torch.from_numpy(S).cuda()
    return buf[:, :m]


def eps_pair(x, xref, v, lam):
    x = np.asarray(x, dtype=np.float64)
    d = np.linalg.norm(x - xref)
    return d / np.linalg.norm(xref), lam * d / np.linalg.norm(v.astype(np.float64) - lam * xref)


ORACLE_CASES = [
    # n, m, lam, x_fp64
    (128, 128037, 1e-2, True),
    (128, 128037, 1e-6, True),
    (128, 128037, 1e-4, False),
]


@pytest.mark.parametrize("n,m,lam,x64", ORACLE_CASES)
def test_final8_against_oracle(dfl, ctx, oracle_mod, n, m, lam, x64):
    print(f"[final8 oracle] n={n} m={m} lam={lam} x64={x64}", flush=True)
    S = synth.make_S(n, m, synth.seed(71, n), "iid")
    v = synth.make_v(S, synth.seed(71, n), "iid")
    xref = oracle_mod.solve(S, v, lam)
    Sd, vd = dev_aligned(S), dev(v)
    kw = dict(gram_prec=2, sweeps=2, centered=True, x_fp64=x64)
    x8, _ = dfl.dfisher_solve(ctx, Sd, vd, lam, **kw)
    xe, _ = dfl.dfisher_solve(ctx, Sd, vd, lam, exact_apply=True, **kw)
    x8, xe = x8.cpu().numpy(), xe.cpu().numpy()
    r8, e8 = eps_pair(x8, xref, v, lam)
    re, ee = eps_pair(xe, xref, v, lam)
    print(f"    fp8 step: rel {r8:.3e} eps_Sy {e8:.3e}; exact step: rel {re:.3e} eps_Sy {ee:.3e}", flush=True)
    assert not np.array_equal(x8, xe)   # the FP8 step was taken
    assert r8 <= 1e-6 and e8 <= 1e-6
    if x64:
        assert e8 <= 2e-7


STEP_CASES = [
    # n, m, lam, sweeps, centered, kind: the line kernel with 8 / 16 loads per lane, the split pairs
    (300, 150000, 1e-3, 2, True, "iid"),
    (1000, 200000, 1e-5, 3, True, "iid"),
    (2100, 120000, 1e-3, 3, True, "iid"),
    (256, 256000, 1e-2, 2, False, "uncentered"),
]


@pytest.mark.parametrize("n,m,lam,sweeps,centered,kind", STEP_CASES)
def test_final8_against_exact_step(dfl, ctx, n, m, lam, sweeps, centered, kind):
    print(f"[final8 vs exact] n={n} m={m} lam={lam} sweeps={sweeps} centered={centered} {kind}", flush=True)
    if kind == "uncentered":
        S = synth.make_S(n, m, synth.seed(72, n), "iid", center=False)
    else:
        S = synth.make_S(n, m, synth.seed(72, n), kind)
    v = synth.make_v(S, synth.seed(72, n), "iid")
    Sd, vd = dev_aligned(S), dev(v)
    kw = dict(gram_prec=2, sweeps=sweeps, centered=centered, x_fp64=True)
    x8, _ = dfl.dfisher_solve(ctx, Sd, vd, lam, **kw)
    xe, _ = dfl.dfisher_solve(ctx, Sd, vd, lam, exact_apply=True, **kw)
    x8, xe = x8.cpu().numpy(), xe.cpu().numpy()
    d = lam * np.linalg.norm(x8 - xe) / np.linalg.norm(v.astype(np.float64) - lam * xe)
    print(f"    |S^T (y8 - y)| / |S^T y| = {d:.3e}", flush=True)
    assert not np.array_equal(x8, xe)
    assert d <= 2e-7


def test_final8_refused_for_a_large_correction(dfl, ctx):
    n, m, lam = 256, 100000, 1e-4
    print(f"[final8 refused] n={n} m={m} lam={lam} sweeps=1", flush=True)
    S = synth.make_S(n, m, synth.seed(73, n), "iid")
    v = synth.make_v(S, synth.seed(73, n), "iid")
    Sd, vd = dev_aligned(S), dev(v)
    kw = dict(gram_prec=2, sweeps=1, centered=True, x_fp64=True)
    x8, _ = dfl.dfisher_solve(ctx, Sd, vd, lam, **kw)
    xe, _ = dfl.dfisher_solve(ctx, Sd, vd, lam, exact_apply=True, **kw)
    assert torch.equal(x8, xe)


def test_final8_uneven(dfl, ctx, oracle_mod):
    # n = 160 and 300, 520 and 1100: the grouped refinement passes' three load-width classes
    shapes = [(300, 120000, 1e-3), (160, 96000, 1e-5), (520, 140000, 1e-2), (1100, 150000, 1e-4)]
    print(f"[final8 uneven] {shapes}", flush=True)
    Ss, vs, lams, refs = [], [], [], []
    for k, (n, m, lam) in enumerate(shapes):
        S = synth.make_S(n, m, synth.seed(74, k), "iid")
        v = synth.make_v(S, synth.seed(74, k), "iid")
        Ss.append(dev_aligned(S))
        vs.append(dev(v))
        lams.append(lam)
        refs.append((oracle_mod.solve(S, v, lam), v))
    kw = dict(gram_prec=2, sweeps=-1, centered=True, x_fp64=True)
    x8, _ = dfl.dfisher_solve_uneven(ctx, Ss, vs, lams, **kw)
    x8 = [x.cpu().numpy() for x in x8]
    x8b, _ = dfl.dfisher_solve_uneven(ctx, Ss, vs, lams, **kw)   # the graph replay
    xe, _ = dfl.dfisher_solve_uneven(ctx, Ss, vs, lams, exact_apply=True, **kw)
    taken = 0
    for a, b, e, (xr, v), lam in zip(x8, x8b, xe, refs, lams):
        e = e.cpu().numpy()
        assert np.array_equal(a, b.cpu().numpy())
        r8, e8 = eps_pair(a, xr, v, lam)
        d = lam * np.linalg.norm(a - e) / np.linalg.norm(v.astype(np.float64) - lam * e)
        print(f"    rel {r8:.3e} eps_Sy {e8:.3e}; vs exact step {d:.3e}", flush=True)
        assert r8 <= 1e-6 and e8 <= 1e-6
        assert d <= 2e-7
        taken += 0 if np.array_equal(a, e) else 1
    assert taken >= 1


BATCHED_CASES = [
    # n, m, nlam, nrhs, sweeps, x64: one partial group; 3 groups (a partial 128-vector block of the
    # product is not reached); ragged n (not a multiple of 64) and m (not of 256)
    (128, 128000, 3, 2, 2, True),
    (64, 64000, 5, 7, 2, True),
    (100, 90037, 4, 3, 3, False),
]


@pytest.mark.parametrize("n,m,nlam,nrhs,sweeps,x64", BATCHED_CASES)
def test_final8_batched(dfl, ctx, oracle_mod, n, m, nlam, nrhs, sweeps, x64):
    print(f"[final8 batched] n={n} m={m} nlam={nlam} nrhs={nrhs} sweeps={sweeps} x64={x64}", flush=True)
    S = synth.make_S(n, m, synth.seed(75, n), "iid")
    V = synth.make_V(m, nrhs, synth.seed(75, n))
    lams = list(np.logspace(-6, -2, nlam))
    Sd, Vd = dev_aligned(S), dev(V)
    kw = dict(gram_prec=2, sweeps=sweeps, centered=True, x_fp64=x64)
    X8, _ = dfl.dfisher_solve_batched(ctx, Sd, lams, Vd, **kw)
    Xe, _ = dfl.dfisher_solve_batched(ctx, Sd, lams, Vd, exact_apply=True, **kw)
    X8, Xe = X8.cpu().numpy(), Xe.cpu().numpy()
    Xref = oracle_mod.solve_batched(S, lams, V)
    assert not np.array_equal(X8, Xe)   # the codes were used
    worst = 0.0
    for li in range(nlam):
        for r in range(nrhs):
            r8, e8 = eps_pair(X8[li, r], Xref[li, r], V[r], lams[li])
            d = lams[li] * np.linalg.norm(X8[li, r].astype(np.float64) - Xe[li, r]) / np.linalg.norm(
                V[r].astype(np.float64) - lams[li] * Xe[li, r])
            worst = max(worst, d)
            assert r8 <= 1e-6 and e8 <= 1e-6, (li, r, r8, e8)
            if x64:
                assert d <= 2e-7, (li, r, d)
    print(f"    worst |S^T (y8 - y)| / |S^T y| {worst:.3e}", flush=True)


def test_final8_batched_refused(dfl, ctx):
    n, m = 128, 50000
    S = synth.make_S(n, m, synth.seed(76, n), "iid")
    V = synth.make_V(m, 3, synth.seed(76, n))
    lams = [1e-5, 1e-3]
    Sd, Vd = dev_aligned(S), dev(V)
    kw = dict(gram_prec=2, sweeps=1, centered=True, x_fp64=True)
    X8, _ = dfl.dfisher_solve_batched(ctx, Sd, lams, Vd, **kw)
    Xe, _ = dfl.dfisher_solve_batched(ctx, Sd, lams, Vd, exact_apply=True, **kw)
    assert torch.equal(X8, Xe)
