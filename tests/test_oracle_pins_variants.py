"""Pins of the oracle's variants of the solve against facts that do not come from the oracle:

* the structured right-hand side of Appendix B, x = S^T (S S^T + lambda I)^-1 f: hand-derived
  examples, a dense LU solve of Eq. 1 with v = S^T f, the n = 1 closed form, exact power-of-two
  scaling;
* the SR front end of Section 3, S = (O - mean O) / sqrt(n): hand-derived examples, invariance
  under adding a constant row to O, zero column sums, numpy's mean, the componentwise complex mean;
* the real-part variant of Section 3, F = Re[S^H S] = Z^T Z for the stacked Z = [Re S; Im S]:
  numpy's complex products, and a dense solve with Re[S^H S];
* the complex variant of Section 3 ((S^H S + lambda I) x = v): hand-derived examples, a dense
  complex LU solve, the n = 1 closed form, equality with the real oracle on real data, the real
  embedding [[A, -B], [B, A]] solved by the real oracle, invariance under a phase per sample.
"""
import json
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
EPS = np.finfo(np.float64).eps


def _golden(key):
    with open(os.path.join(HERE, "golden", "hand_examples.json")) as f:
        return json.load(f)[key]


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _cond_tol(A64, lam, c=50.0):
    s = np.linalg.svd(A64, compute_uv=False)
    return c * EPS * (float(s[0]) ** 2 + lam) / lam


def _ulp32(a):
    a = np.abs(np.asarray(a, dtype=np.float32))
    return np.spacing(a).astype(np.float64)


# ------------------------------------------------------------------ Appendix B: v = S^T f

@pytest.mark.parametrize("ex", _golden("rowspace_examples"), ids=lambda e: e["name"])
def test_rowspace_hand_examples(oracle_mod, ex):
    S = np.array(ex["S"], dtype=np.float32)
    x, y = oracle_mod.solve_rowspace(S, ex["f"], ex["lambda"], return_y=True)
    np.testing.assert_allclose(y, ex["y"], rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(x, ex["x"], rtol=1e-15, atol=1e-16)


@pytest.mark.parametrize("n,m,lam", [(8, 40, 1e-2), (16, 300, 1e-5), (30, 20, 0.5)])
def test_rowspace_dense(oracle_mod, n, m, lam):
    """Against a dense LU solve of Eq. 1 with v = S^T f (the m x m system, no push-through)."""
    S = synth.make_S(n, m, synth.seed(60, n), "iid")
    f = np.random.default_rng(n).standard_normal(n)
    S64 = S.astype(np.float64)
    v = S64.T @ f
    xd = np.linalg.solve(S64.T @ S64 + lam * np.eye(m), v)
    x = oracle_mod.solve_rowspace(S, f, lam)
    assert _rel(x, xd) <= _cond_tol(S64, lam)


def test_rowspace_n1_closed_form(oracle_mod):
    """n = 1: (s s^T + lambda I)^-1 s f = s f / (lambda + |s|^2)."""
    s = np.random.default_rng(3).standard_normal(100).astype(np.float32)
    x = oracle_mod.solve_rowspace(s.reshape(1, -1), [2.5], 0.3)
    s64 = s.astype(np.float64)
    np.testing.assert_allclose(x, s64 * 2.5 / (0.3 + s64 @ s64), rtol=1e-14)


def test_rowspace_power_of_two_scaling(oracle_mod):
    """(2S, 4 lambda, f) gives x / 2 to the last bit (every operation scales exactly)."""
    S = synth.make_S(12, 200, 7, "iid")
    f = np.random.default_rng(5).standard_normal(12)
    x = oracle_mod.solve_rowspace(S, f, 1e-2)
    x2 = oracle_mod.solve_rowspace((2 * S).astype(np.float32), f, 4e-2)
    np.testing.assert_array_equal(x2, x / 2)


# ------------------------------------------------------------------ Section 3: SR centering

def test_center_hand_examples(oracle_mod):
    ex1, ex2 = _golden("center_examples")
    S = oracle_mod.center(np.array(ex1["O"], dtype=np.float32))
    expect = (np.array(ex1["S_times_sqrt_n"]) / np.sqrt(2.0)).astype(np.float32)
    np.testing.assert_array_equal(S, expect)
    S = oracle_mod.center(np.array(ex2["O"], dtype=np.float32))
    np.testing.assert_array_equal(S, np.array(ex2["S"], dtype=np.float32))


def test_center_row_offset_invariance(oracle_mod):
    """Adding the same row c to every sample leaves S unchanged, bit for bit (values are dyadic
    with few bits, so every FP64 step is exact); a per-row instead of per-column mean fails."""
    rng = np.random.default_rng(11)
    O = (rng.integers(-64, 64, size=(16, 50)) / 8.0).astype(np.float32)
    c = (rng.integers(-64, 64, size=50) / 4.0).astype(np.float32)
    np.testing.assert_array_equal(oracle_mod.center(O + c), oracle_mod.center(O))
    # a per-sample constant is not removed
    assert not np.array_equal(oracle_mod.center(O + c[:16, None]), oracle_mod.center(O))


@pytest.mark.parametrize("n,m", [(7, 33), (64, 500), (300, 41)])
def test_center_against_numpy(oracle_mod, n, m):
    """Against numpy's mean (pairwise summation) in FP64: equal within one FP32 ulp (the two means
    differ only in rounding, which can move a result across a rounding boundary), nearly always
    equal; column sums of S vanish to rounding; the scale is 1/sqrt(n), not 1/n."""
    O = synth.make_O(n, m, synth.seed(61, n))
    S = oracle_mod.center(O)
    O64 = O.astype(np.float64)
    ref = (O64 - O64.mean(axis=0)) / np.sqrt(n)
    d = np.abs(S.astype(np.float64) - ref)
    assert np.all(d <= _ulp32(ref) * 0.5 + 1e-300 + np.abs(ref) * 1e-15 * n)
    np.testing.assert_allclose(np.sum(S.astype(np.float64), axis=0), 0.0,
                               atol=float(n * np.max(_ulp32(S))))
    np.testing.assert_allclose(np.sum(S.astype(np.float64) ** 2),
                               np.sum((O64 - O64.mean(axis=0)) ** 2) / n, rtol=1e-6)


def test_center_complex_componentwise(oracle_mod):
    """The complex mean is componentwise: the stacked Z equals the real centering of Re O and of
    Im O, bit for bit, rows 0..n-1 and n..2n-1."""
    O = synth.make_O(40, 77, 5, complex_=True)
    Z = oracle_mod.center_complex(O)
    np.testing.assert_array_equal(Z[:40], oracle_mod.center(np.ascontiguousarray(O.real)))
    np.testing.assert_array_equal(Z[40:], oracle_mod.center(np.ascontiguousarray(O.imag)))
    ref = (O.astype(np.complex128) - O.astype(np.complex128).mean(axis=0)) / np.sqrt(40)
    assert np.all(np.abs(Z[:40] - ref.real) <= _ulp32(ref.real) * 0.5 + np.abs(ref.real) * 1e-13)
    assert np.all(np.abs(Z[40:] - ref.imag) <= _ulp32(ref.imag) * 0.5 + np.abs(ref.imag) * 1e-13)


# ------------------------------------------------------------------ Section 3: real-part variant

def test_real_part_variant_is_stacked_gram(oracle_mod):
    """Re[S^H S] = Z^T Z for Z = [Re S; Im S] (concatenation in the sample dimension), and the
    oracle's solve on Z solves (Re[S^H S] + lambda I) x = v (dense complex products by numpy)."""
    O = synth.make_O(12, 60, 8, complex_=True)
    Z = oracle_mod.center_complex(O)
    Sc = Z[:12].astype(np.float64) + 1j * Z[12:].astype(np.float64)
    F = np.real(Sc.conj().T @ Sc)
    Z64 = Z.astype(np.float64)
    np.testing.assert_allclose(Z64.T @ Z64, F, rtol=1e-13, atol=1e-14)
    v = np.random.default_rng(2).standard_normal(60)
    lam = 1e-2
    xd = np.linalg.solve(F + lam * np.eye(60), v)
    x = oracle_mod.solve(Z, v, lam)
    assert _rel(x, xd) <= _cond_tol(Z64, lam)


# ------------------------------------------------------------------ Section 3: complex variant

@pytest.mark.parametrize("ex", _golden("complex_examples"), ids=lambda e: e["name"])
def test_complex_hand_examples(oracle_mod, ex):
    S = (np.array(ex["S_re"]) + 1j * np.array(ex["S_im"])).astype(np.complex64)
    v = np.array(ex["v_re"]) + 1j * np.array(ex["v_im"])
    x, y = oracle_mod.solve_complex(S, v, ex["lambda"], return_y=True)
    np.testing.assert_allclose(y, np.array(ex["y_re"]) + 1j * np.array(ex["y_im"]), rtol=1e-15, atol=1e-16)
    np.testing.assert_allclose(x, np.array(ex["x_re"]) + 1j * np.array(ex["x_im"]), rtol=1e-15, atol=1e-16)


@pytest.mark.parametrize("n,m,lam", [(6, 40, 1e-2), (16, 200, 1e-5), (25, 20, 0.3)])
def test_complex_dense(oracle_mod, n, m, lam):
    """Against numpy's dense complex LU solve of (S^H S + lambda I) x = v."""
    O = synth.make_O(n, m, synth.seed(62, n), complex_=True)
    Z = oracle_mod.center_complex(O)
    S = (Z[:n] + 1j * Z[n:].astype(np.float64)).astype(np.complex64)
    v = synth.make_vc(m, n).astype(np.complex128)
    S128 = S.astype(np.complex128)
    xd = np.linalg.solve(S128.conj().T @ S128 + lam * np.eye(m), v)
    x = oracle_mod.solve_complex(S, v, lam)
    assert _rel(x, xd) <= _cond_tol(S128, lam)


def test_complex_n1_closed_form(oracle_mod):
    """n = 1, S = s^T: (conj(s) s^T + lambda I)^-1 v = (v - conj(s) (s^T v) / (lambda + |s|^2)) / lambda."""
    rng = np.random.default_rng(9)
    s = (rng.standard_normal(50) + 1j * rng.standard_normal(50)).astype(np.complex64)
    v = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    lam = 0.7
    x = oracle_mod.solve_complex(s.reshape(1, -1), v, lam)
    s128 = s.astype(np.complex128)
    ref = (v - s128.conj() * (s128 @ v) / (lam + np.vdot(s128, s128).real)) / lam
    np.testing.assert_allclose(x, ref, rtol=1e-13)


def test_complex_on_real_data_is_real_solve(oracle_mod):
    """With zero imaginary parts the complex algorithm is the real one."""
    S = synth.make_S(20, 150, 4, "iid")
    v = synth.make_v(S, 4)
    x = oracle_mod.solve_complex(S.astype(np.complex64), v.astype(np.complex128), 1e-3)
    xr = oracle_mod.solve(S, v, 1e-3)
    np.testing.assert_allclose(x.real, xr, rtol=1e-14, atol=1e-14 * np.max(np.abs(xr)))
    assert np.all(x.imag == 0)


def test_complex_real_embedding(oracle_mod):
    """(S^H S + lambda I) x = v with S = A + iB is the real system of the 2n x 2m matrix
    [[A, -B], [B, A]] with v = [Re v; Im v] and x = [Re x; Im x]; the real oracle solves it."""
    n, m, lam = 10, 70, 1e-2
    O = synth.make_O(n, m, 21, complex_=True)
    Z = oracle_mod.center_complex(O)
    A, B = Z[:n], Z[n:]
    S = (A + 1j * B.astype(np.float64)).astype(np.complex64)
    v = synth.make_vc(m, 21).astype(np.complex128)
    x = oracle_mod.solve_complex(S, v, lam)
    E = np.block([[A, -B], [B, A]]).astype(np.float32)
    xe = oracle_mod.solve(E, np.concatenate([v.real, v.imag]), lam)
    np.testing.assert_allclose(np.concatenate([x.real, x.imag]), xe, rtol=0,
                               atol=_cond_tol(E.astype(np.float64), lam) * np.linalg.norm(xe))


def test_complex_sample_phase_invariance(oracle_mod):
    """Multiplying a sample (row of S) by i leaves S^H S, and so x, unchanged."""
    n, m, lam = 9, 60, 1e-2
    O = synth.make_O(n, m, 22, complex_=True)
    Z = oracle_mod.center_complex(O)
    S = (Z[:n] + 1j * Z[n:].astype(np.float64)).astype(np.complex64)
    v = synth.make_vc(m, 22).astype(np.complex128)
    S2 = S.copy()
    S2[3] *= 1j
    S2[5] *= -1j
    x = oracle_mod.solve_complex(S, v, lam)
    x2 = oracle_mod.solve_complex(S2, v, lam)
    assert _rel(x2, x) <= 1e-12
