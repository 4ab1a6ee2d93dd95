"""dfisher_factor_solve_noalloc (the entry point for callers that cannot allocate) against
dfisher_factor_solve on the same factor and right-hand side, through the C ABI: two calls in a
row, the second with a smaller problem (factor), each compared element by element with the
existing entry point (both compute Algorithm 1 steps 3-4 with the factor's refinement sweeps, in
a different summation order) and with the FP64 oracle. Device free memory must not move across a
no-alloc call."""
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


@pytest.mark.parametrize("x_fp64", [True, False])
def test_noalloc_matches_factor_solve(dfl, ctx, oracle_mod, x_fp64):
    # (n, m, lam, gram precision, sweeps): the second problem is smaller in both n and m
    shapes = [(520, 40000, 1e-2, 1, 2), (96, 9000, 1e-3, 2, 6)]
    for call, (n, m, lam, prec, sweeps) in enumerate(shapes):
        print(f"[noalloc] call {call}: n={n} m={m} lam={lam} prec={prec} sweeps={sweeps} x_fp64={x_fp64}", flush=True)
        S = synth.make_S(n, m, synth.seed(80, n))
        v = synth.make_v(S, synth.seed(80, n))
        Sd, vd = dev(S), dev(v)
        f, _ = dfl.dfisher_factor_create(ctx, Sd, lam, gram_prec=prec, sweeps=sweeps, x_fp64=x_fp64)
        try:
            x_ref = dfl.dfisher_factor_solve(f, vd)
            dt = torch.float64 if x_fp64 else torch.float32
            x = torch.full((m,), float("nan"), dtype=dt, device="cuda")
            info = dfl.dfisher_factor_solve_noalloc(f, vd, x)          # warm (first launches)
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            x.fill_(float("nan"))
            info = dfl.dfisher_factor_solve_noalloc(f, vd, x)
            torch.cuda.synchronize()
            assert torch.cuda.mem_get_info()[0] == free0
            assert info["sweeps_done"] == sweeps
            a = x.double().cpu().numpy()
            b = x_ref.double().cpu().numpy()
            assert np.all(np.isfinite(a))
            if x_fp64:
                assert np.max(np.abs(a - b)) <= 1e-10 * np.max(np.abs(b))
            else:   # the same FP64 value rounded once, up to FP64 summation-order differences
                assert np.all(np.abs(a - b) <= 2.0 ** -23 * np.abs(b) + 1e-30)
            xo = oracle_mod.solve(S, v, lam)
            err = float(np.linalg.norm(a - xo) / np.linalg.norm(xo))
            print(f"    max |noalloc - factor_solve| / max|x| {np.max(np.abs(a - b)) / np.max(np.abs(b)):.3e}, "
                  f"rel err vs oracle {err:.3e}", flush=True)
            assert err <= 1e-6
        finally:
            f.close()


def test_noalloc_rejects_unsupported(dfl, ctx):
    """Refinement on rows that are not 16-byte aligned has no one-read product: refused before any
    device work, with the output untouched."""
    n, m = 64, 3001
    S = synth.make_S(n, m, 81)
    buf = torch.zeros((n, m + 1), dtype=torch.float32, device="cuda")
    buf[:, :m] = torch.from_numpy(S).cuda()
    Sd = buf[:, :m]   # row stride 3002 floats: not a multiple of 4
    f, _ = dfl.dfisher_factor_create(ctx, Sd, 1e-2, gram_prec=0, sweeps=1, x_fp64=True)
    try:
        x = torch.full((m,), 7.0, dtype=torch.float64, device="cuda")
        with pytest.raises(dfl.DfisherError) as ei:
            dfl.dfisher_factor_solve_noalloc(f, dev(synth.make_v(S, 81)), x)
        assert ei.value.status == dfl.DFISHER_E_UNSUPPORTED
        torch.cuda.synchronize()
        assert bool(torch.all(x == 7.0))
    finally:
        f.close()
