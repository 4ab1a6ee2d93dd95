"""Pins of the oracle's preconditioner for a centered score matrix (Section 3: the columns of
S = (O - mean O) / sqrt(n) sum to zero over the samples), M = P W P + lambda U U^T with
P = I - U U^T and U the normalised indicators of nseg equal segments, against facts that do not
come from the oracle:

* hand-derived 2 x 2 and 4 x 4 examples (tests/golden/hand_examples.json);
* an exactly centered integer S, for which W = S S^T + lambda I already maps the indicators to
  lambda times themselves, so M = W bit for bit (real case, and the complex variant's real
  embedding [[A, -B], [B, A]] with nseg = 2);
* the defining properties on a random symmetric W: M u_s = lambda u_s, x^T M x = x^T W x for x
  orthogonal to every indicator, symmetry, and M - W of rank at most 2 nseg.
"""
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _examples():
    with open(os.path.join(HERE, "golden", "hand_examples.json")) as f:
        return json.load(f)["project_examples"]


@pytest.mark.parametrize("ex", _examples(), ids=lambda e: e["name"])
def test_project_hand_examples(oracle_mod, ex):
    M = oracle_mod.project_centered(np.array(ex["W"]), ex["lambda"], ex["nseg"])
    np.testing.assert_allclose(M, np.array(ex["M"]), rtol=0, atol=1e-15)


def _centered_int(rng, n, m):
    A = rng.integers(-3, 4, size=(n, m)).astype(np.float64)
    A[-1] = -A[:-1].sum(axis=0)   # every column sums to zero exactly
    return A


def test_project_identity_on_exactly_centered(oracle_mod):
    rng = np.random.default_rng(11)
    n, m, lam = 16, 40, 0.5
    S = _centered_int(rng, n, m)
    W = S @ S.T + lam * np.eye(n)   # small integers and halves: exact in FP64
    M = oracle_mod.project_centered(W, lam, 1)
    assert np.array_equal(M, W)


def test_project_identity_on_complex_embedding(oracle_mod):
    rng = np.random.default_rng(12)
    n, m, lam = 8, 24, 0.25
    A, B = _centered_int(rng, n, m), _centered_int(rng, n, m)
    E = np.block([[A, -B], [B, A]])
    W = E @ E.T + lam * np.eye(2 * n)
    M = oracle_mod.project_centered(W, lam, 2)
    assert np.array_equal(M, W)
    # with one segment the embedding is not centered along the all-ones vector of 2n entries
    # only if the halves differ; here both halves are centered, so nseg = 1 also leaves W alone
    M1 = oracle_mod.project_centered(W, lam, 1)
    assert np.array_equal(M1, W)


def _indicators(n, nseg):
    l = n // nseg
    U = np.zeros((n, nseg))
    for s in range(nseg):
        U[s * l:(s + 1) * l, s] = 1.0 / np.sqrt(l)
    return U


@pytest.mark.parametrize("n,nseg", [(7, 1), (30, 1), (64, 2), (90, 2), (96, 3)])
def test_project_defining_properties(oracle_mod, n, nseg):
    rng = np.random.default_rng(n + nseg)
    X = rng.standard_normal((n, 3 * n))
    W = X @ X.T / n + 0.1 * np.eye(n)
    lam = 0.37
    M = oracle_mod.project_centered(W, lam, nseg)
    U = _indicators(n, nseg)
    scale = np.abs(W).max()
    np.testing.assert_allclose(M @ U, lam * U, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(M, M.T, rtol=0, atol=1e-14 * scale)
    Y = rng.standard_normal((n, 5))
    Y -= U @ (U.T @ Y)
    np.testing.assert_allclose(np.einsum("ik,ij,jk->k", Y, M, Y), np.einsum("ik,ij,jk->k", Y, W, Y),
                               rtol=1e-12)
    sv = np.linalg.svd(M - W, compute_uv=False)
    assert np.sum(sv > 1e-10 * sv[0]) <= 2 * nseg
