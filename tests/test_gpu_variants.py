"""GPU parity of the variants of the solve against the FP64 CPU oracle, through the C ABI:

* the structured right-hand side of Appendix B (dfisher_solve_rowspace: v = S^T f, solved as
  x = S^T (S S^T + lambda I)^-1 f without forming v) against oracle.solve_rowspace.

Tolerances: x = S^T y comes straight from y (no subtraction v - S^T y), so its error relative to
|x| is the error of S^T y: the refinement sweeps bring it toward the FP64 level (1e-9 asked with
the FP32 and split-BF16 Grams after 2 sweeps, 1e-8 with the scaled-FP8 Gram after 6); an FP32 x adds
its own rounding (<= 2^-24 relative per entry). Cases without sweeps or with lambda = 1e-6 on a
centered S get looser bounds, stated where they are listed.
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


def dev_strided(S, ld):
    n, m = S.shape
    buf = torch.full((n, ld), float("nan"), dtype=torch.float32, device="cuda")
    buf[:, :m] = torch.from_numpy(S).cuda()
    return buf[:, :m]


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    dt = np.complex128 if (np.iscomplexobj(a) or np.iscomplexobj(b)) else np.float64
    a, b = a.astype(dt), b.astype(dt)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


ROWSPACE_CASES = [
    # n, m, ld, lam, prec, sweeps, kind, bound
    (32, 1024, 1024, 1e-2, 0, 2, "iid", 1e-9),        # smallest workload
    (300, 20001, 20004, 1e-4, 1, 2, "iid", 1e-9),     # ragged n and m, padded stride (two-pass products)
    (257, 30000, 30000, 1e-6, 1, 2, "scaled", 1e-7),  # fused product, column-scaled S, small lambda (*)
    (320, 20016, 20016, 1e-3, 2, 6, "iid", 1e-8),     # scaled-FP8 Gram
    (1, 777, 777, 1e-1, 0, 1, "iid", 1e-12),          # one (uncentered) sample: x = s f / (lambda + |s|^2)
    (200, 10001, 10001, 1e-2, 0, 0, "iid", 2e-4),     # stride not a multiple of 4, no sweep: the FP32
]                                                     # Gram's own error (m / n = 50)
# (*) at lambda = 1e-6 the all-ones direction of the centered S has W's eigenvalue ~ lambda: f's
# component along it makes y's large, and x = S^T y carries its error through the small but
# nonzero S^T 1; the sweeps reach that direction after the bulk.


@pytest.mark.parametrize("n,m,ld,lam,prec,sweeps,kind,bound", ROWSPACE_CASES)
def test_rowspace(dfl, ctx, oracle_mod, n, m, ld, lam, prec, sweeps, kind, bound):
    print(f"[rowspace] n={n} m={m} ld={ld} lam={lam} prec={prec} sweeps={sweeps} kind={kind}", flush=True)
    S = synth.make_S(n, m, synth.seed(70, n), kind, center=n > 1)   # a centered single row is 0
    f = np.random.default_rng(n).standard_normal(n)
    xref = oracle_mod.solve_rowspace(S, f, lam)
    Sd = dev_strided(S, ld) if ld != m else dev(S)
    x, info = dfl.dfisher_solve_rowspace(ctx, Sd, dev(f), lam, gram_prec=prec, sweeps=sweeps, x_fp64=True)
    err = rel(x.cpu().numpy(), xref)
    print(f"    rel err {err:.3e} info {info}", flush=True)
    assert err <= bound
    # FP32 output: the same x rounded once
    x32, _ = dfl.dfisher_solve_rowspace(ctx, Sd, dev(f), lam, gram_prec=prec, sweeps=sweeps)
    assert x32.dtype == torch.float32
    xr = x.cpu().numpy()
    assert np.all(np.abs(x32.cpu().numpy().astype(np.float64) - xr) <= np.abs(xr) * 2.0 ** -24 + 1e-300)


def test_rowspace_equals_general_solve(dfl, ctx, oracle_mod):
    """Appendix B on the device: the structured solve and dfisher_solve with v = S^T f (formed in FP64
    and rounded to FP32 on the host) agree with their oracles, and the structured one is the more
    accurate on the part that cancels (x = v / lambda - S^T y / lambda for a v in the row space)."""
    n, m, lam = 256, 16384, 1e-3
    S = synth.make_S(n, m, synth.seed(71, n), "scaled")
    f = np.random.default_rng(7).standard_normal(n)
    v = (S.astype(np.float64).T @ f).astype(np.float32)
    x_s, _ = dfl.dfisher_solve_rowspace(ctx, dev(S), dev(f), lam, gram_prec=1, sweeps=2, x_fp64=True)
    x_g, _ = dfl.dfisher_solve(ctx, dev(S), dev(v), lam, gram_prec=1, sweeps=2, x_fp64=True)
    e_s = rel(x_s.cpu().numpy(), oracle_mod.solve_rowspace(S, f, lam))
    e_g = rel(x_g.cpu().numpy(), oracle_mod.solve(S, v, lam))
    print(f"    structured {e_s:.3e}  general {e_g:.3e}", flush=True)
    assert e_s <= 1e-9 and e_g <= 1e-5 and e_s <= e_g


def test_rowspace_tolerance_and_final_resid(dfl, ctx, oracle_mod):
    """tol and final_resid act on W y = f as in dfisher_solve: the measured residual meets tol and the
    final residual of the returned y is at most about it."""
    n, m, lam = 320, 20016, 1e-2
    S = synth.make_S(n, m, synth.seed(72, n))
    f = np.random.default_rng(3).standard_normal(n)
    x, info = dfl.dfisher_solve_rowspace(ctx, dev(S), dev(f), lam, gram_prec=2, sweeps=16, tol=1e-10,
                                         final_resid=True, x_fp64=True)
    print(f"    {info}", flush=True)
    assert info["converged"] and info["resid"] <= 1e-10 and 0.0 <= info["w_resid"] <= 1e-9
    assert rel(x.cpu().numpy(), oracle_mod.solve_rowspace(S, f, lam)) <= 1e-8


# ------------------------------------------------------------------ Section 3: SR front end

def _ulp_ok(got, ref):
    """|got - ref| <= one FP32 ulp of ref everywhere, and nearly all equal: the FP64 column means differ
    from the oracle's sequential ones only in summation order, which can move the FP64 value across a
    rounding boundary of the final FP32 rounding."""
    got = np.asarray(got, dtype=np.float32)
    ref = np.asarray(ref, dtype=np.float32)
    d = np.abs(got.astype(np.float64) - ref.astype(np.float64))
    ok = bool(np.all(d <= np.spacing(np.abs(ref)).astype(np.float64)))
    same = float(np.mean(got == ref))
    return ok, same


@pytest.mark.parametrize("n,m,ldo,lds", [(7, 33, 33, 40), (300, 20001, 20004, 20001), (64, 4096, 4096, 4096),
                                          (1, 100, 100, 100)])
def test_sr_center(dfl, ctx, oracle_mod, n, m, ldo, lds):
    print(f"[sr center] n={n} m={m} ldo={ldo} lds={lds}", flush=True)
    O = synth.make_O(n, m, synth.seed(73, n))
    Od = dev_strided(O, ldo) if ldo != m else dev(O)
    Sbuf = torch.full((n, lds), float("nan"), dtype=torch.float32, device="cuda")
    S = dfl.dfisher_sr_center(ctx, Od, S=Sbuf[:, :m])
    ref = oracle_mod.center(O)
    ok, same = _ulp_ok(S.cpu().numpy(), ref)
    print(f"    within 1 ulp: {ok}, identical: {same:.5f}", flush=True)
    assert ok and same >= 0.99
    # in place (same array, same stride)
    Oi = dev(O)
    dfl.dfisher_sr_center(ctx, Oi, S=Oi)
    np.testing.assert_array_equal(Oi.cpu().numpy(), S.cpu().numpy())


@pytest.mark.parametrize("n,m", [(5, 77), (257, 9000)])
def test_sr_center_complex(dfl, ctx, oracle_mod, n, m):
    print(f"[sr center complex] n={n} m={m}", flush=True)
    O = synth.make_O(n, m, synth.seed(74, n), complex_=True)
    Z = dfl.dfisher_sr_center(ctx, dev(O))
    assert tuple(Z.shape) == (2 * n, m)
    ok, same = _ulp_ok(Z.cpu().numpy(), oracle_mod.center_complex(O))
    print(f"    within 1 ulp: {ok}, identical: {same:.5f}", flush=True)
    assert ok and same >= 0.99


def test_real_part_variant(dfl, ctx, oracle_mod):
    """The real-part variant end to end on the device: Z = [Re S; Im S] from a complex O, then the
    unchanged solve with 2n samples, against the oracle's solve on the same Z (the bytes the device
    wrote) and against the dense solve of (Re[S^H S] + lambda I) x = v."""
    n, m, lam = 150, 12000, 1e-3
    O = synth.make_O(n, m, synth.seed(75, n), complex_=True)
    Zd = dfl.dfisher_sr_center(ctx, dev(O))
    Z = Zd.cpu().numpy()
    v = synth.make_v(Z, synth.seed(75, n))
    x, info = dfl.dfisher_solve(ctx, Zd, dev(v), lam, gram_prec=1, sweeps=2, x_fp64=True)
    xo = oracle_mod.solve(Z, v, lam)
    err = rel(x.cpu().numpy(), xo)
    Sc = Z[:n].astype(np.float64) + 1j * Z[n:].astype(np.float64)
    xd = np.linalg.solve(np.real(Sc.conj().T @ Sc) + lam * np.eye(m), v.astype(np.float64))
    print(f"    rel err vs oracle {err:.3e}, oracle vs dense {rel(xo, xd):.3e}", flush=True)
    assert err <= 1e-9 and rel(xo, xd) <= 1e-8


# ------------------------------------------------------------------ Section 3: complex variant

COMPLEX_CASES = [
    # n, m, lam, prec, sweeps, bound
    (20, 700, 1e-2, 0, 2, 1e-9),
    (130, 9001, 1e-3, 0, 2, 1e-8),       # ragged n and m, unaligned rows (two-vector passes, any stride)
    (300, 20000, 1e-5, 1, 3, 1e-8),      # 2n = 600: several 64-row blocks and 256-row tiles
    (96, 16384, 1e-4, 2, 8, 1e-6),       # scaled-FP8 Gram of Z
    (1, 500, 1e-1, 0, 1, 1e-12),         # one sample
]


@pytest.mark.parametrize("n,m,lam,prec,sweeps,bound", COMPLEX_CASES)
def test_solve_complex(dfl, ctx, oracle_mod, n, m, lam, prec, sweeps, bound):
    print(f"[complex] n={n} m={m} lam={lam} prec={prec} sweeps={sweeps}", flush=True)
    O = synth.make_O(n, m, synth.seed(76, n), complex_=True)
    Z = oracle_mod.center_complex(O) if n > 1 else np.concatenate([O.real, O.imag]).astype(np.float32)
    S = (Z[:n].astype(np.float64) + 1j * Z[n:].astype(np.float64)).astype(np.complex64)
    v = synth.make_vc(m, synth.seed(76, n))
    xo = oracle_mod.solve_complex(S, v, lam)
    if prec == 2:   # 16-byte aligned rows
        ld = (m + 3) // 4 * 4
        Zd = torch.zeros((2 * n, ld), dtype=torch.float32, device="cuda")
        Zd[:, :m] = torch.from_numpy(Z).cuda()
        Zd = Zd[:, :m]
    else:
        Zd = dev(Z)
    x, info = dfl.dfisher_solve_complex(ctx, Zd, dev(v), lam, gram_prec=prec, sweeps=sweeps, x_fp64=True,
                                        final_resid=True)
    err = rel(x.cpu().numpy(), xo)
    print(f"    rel err {err:.3e} info {info}", flush=True)
    assert err <= bound
    assert info["sweeps_done"] == sweeps and (sweeps == 0 or info["w_resid"] >= 0.0)
    # complex64 output: the same x rounded once per component
    x32, _ = dfl.dfisher_solve_complex(ctx, Zd, dev(v), lam, gram_prec=prec, sweeps=sweeps)
    a, b = x32.cpu().numpy(), x.cpu().numpy()
    assert np.all(np.abs(a.real - b.real) <= np.abs(b.real) * 2.0 ** -24 + 1e-300)
    assert np.all(np.abs(a.imag - b.imag) <= np.abs(b.imag) * 2.0 ** -24 + 1e-300)


def test_solve_complex_on_real_data(dfl, ctx, oracle_mod):
    """Zero imaginary parts: the complex solve returns the real solve's x with zero imaginary part."""
    n, m, lam = 64, 5000, 1e-2
    S = synth.make_S(n, m, synth.seed(77, n))
    v = synth.make_v(S, synth.seed(77, n))
    Z = np.concatenate([S, np.zeros_like(S)])
    x, _ = dfl.dfisher_solve_complex(ctx, dev(Z), dev(v.astype(np.complex64)), lam, gram_prec=0, sweeps=2, x_fp64=True)
    x = x.cpu().numpy()
    assert rel(x.real, oracle_mod.solve(S, v, lam)) <= 1e-9
    assert np.max(np.abs(x.imag)) <= 1e-12 * np.max(np.abs(x.real))
