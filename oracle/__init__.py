"""FP64 CPU oracle for the damped Fisher solve (Eq. 1, Algorithm 1 of arXiv 2310.17556).

Test infrastructure only: tests/, ``__graft_entry__.smoke()`` and bench.py's cpu_baseline leg
are the only users. It shares no code with the HIP library in ``paper_2310_17556_amd`` and never
imports it. The arithmetic lives in ``dfisher_oracle.c`` (plain C loops, FP64, sequential sums);
this module only marshals numpy arrays through ctypes.

Every function states the passage of the paper it follows:

* :func:`gram`       - Algorithm 1 step 1, W = S S^T + lambda I_n.
* :func:`cholesky`   - Algorithm 1 step 2, W = L L^T.
* :func:`gemv`, :func:`forward`, :func:`backward`, :func:`apply`
                     - the right-to-left evaluation of Q^T Q v = S^T L^-T L^-1 S v that
                       Section 2 recommends instead of forming Q (Algorithm 1 steps 3-4).
* :func:`solve`      - Algorithm 1 end to end.
* :func:`residual`   - v - lambda x - S^T S x, the identity of Proposition 1 (Appendix A).
* :func:`split_bf16`, :func:`gram3` - definition of the split-BF16 Gram (three products).
* :func:`quant_mxfp8` - definition of the block-scaled FP8 inputs of the scaled-FP8 Gram.
* :func:`solve_rowspace` - the structured right-hand side v = S^T f of Appendix B,
                       x = S^T (S S^T + lambda I)^-1 f.
* :func:`center`, :func:`center_complex` - the SR score matrix S = (O - mean O) / sqrt(n) of
                       Section 3; the complex form in the stacked real layout [Re S; Im S].
* :func:`solve_complex` - the complex variant of Section 3 (transposes become Hermitian
                       conjugates), in complex FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dfisher_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, FP64, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-std=c11", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        D = ctypes.c_double
        sigs = {
            "oracle_gram": ([P, I, I, I, D, P], None),
            "oracle_cholesky": ([P, I, P], I),
            "oracle_gemv": ([P, I, I, I, P, P], None),
            "oracle_forward": ([P, I, P, P], None),
            "oracle_backward": ([P, I, P, P], None),
            "oracle_apply": ([P, I, I, I, P, P, D, P], None),
            "oracle_solve": ([P, I, I, I, P, D, P, P], I),
            "oracle_residual": ([P, I, I, I, P, P, D, P], None),
            "oracle_split_bf16": ([P, I, I, I, P, P], None),
            "oracle_gram3": ([P, P, I, I, D, P], None),
            "oracle_row_norms": ([P, I, I, I, P], None),
            "oracle_quant_mxfp8": ([P, I, I, I, P, P], None),
            "oracle_gram_entries": ([P, I, I, D, P, P, I, P], None),
            "oracle_num_threads": ([], ctypes.c_int),
            "oracle_solve_rowspace": ([P, I, I, I, P, D, P, P], I),
            "oracle_center": ([P, I, I, I, P, I], None),
            "oracle_center_complex": ([P, I, I, I, P, I], None),
            "oracle_solve_complex": ([P, I, I, I, P, D, P, P], I),
            "oracle_project_centered": ([P, I, I, D, P], None),
        }
        for name, (args, res) in sigs.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _S(S) -> tuple[np.ndarray, int, int, int]:
    S = np.asarray(S)
    if S.dtype != np.float32 or S.ndim != 2:
        raise TypeError("S must be a 2-D float32 array (the library's input format)")
    if S.strides[1] != 4 or S.strides[0] % 4 != 0 or S.strides[0] < 4 * S.shape[1]:
        S = np.ascontiguousarray(S)
    n, m = S.shape
    return S, n, m, S.strides[0] // 4


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def gram(S, lam: float = 0.0) -> np.ndarray:
    """Algorithm 1 step 1: W = S S^T + lam * I_n (full symmetric n x n, FP64)."""
    S, n, m, lds = _S(S)
    W = np.empty((n, n), dtype=np.float64)
    _load().oracle_gram(_p(S), n, m, lds, float(lam), _p(W))
    return W


def cholesky(W) -> tuple[np.ndarray, int]:
    """Algorithm 1 step 2: lower-triangular L with W = L L^T. Returns (L, info); info is 0 or the
    1-based index of the first pivot that is not > 0."""
    W = _f64(W)
    n = W.shape[0]
    if W.shape != (n, n):
        raise ValueError("W must be square")
    L = np.empty((n, n), dtype=np.float64)
    info = _load().oracle_cholesky(_p(W), n, _p(L))
    return L, int(info)


def gemv(S, v) -> np.ndarray:
    """b = S v (first product of the right-to-left evaluation)."""
    S, n, m, lds = _S(S)
    v = _f64(v, (m,))
    b = np.empty(n, dtype=np.float64)
    _load().oracle_gemv(_p(S), n, m, lds, _p(v), _p(b))
    return b


def forward(L, b) -> np.ndarray:
    """z = L^-1 b by forward substitution."""
    L = _f64(L)
    n = L.shape[0]
    b = _f64(b, (n,))
    z = np.empty(n, dtype=np.float64)
    _load().oracle_forward(_p(L), n, _p(b), _p(z))
    return z


def backward(L, z) -> np.ndarray:
    """y = L^-T z by back substitution."""
    L = _f64(L)
    n = L.shape[0]
    z = _f64(z, (n,))
    y = np.empty(n, dtype=np.float64)
    _load().oracle_backward(_p(L), n, _p(z), _p(y))
    return y


def apply(S, v, y, lam: float) -> np.ndarray:
    """x = (v - S^T y) / lam (Algorithm 1 step 4 with Q inlined)."""
    S, n, m, lds = _S(S)
    v = _f64(v, (m,))
    y = _f64(y, (n,))
    x = np.empty(m, dtype=np.float64)
    _load().oracle_apply(_p(S), n, m, lds, _p(v), _p(y), float(lam), _p(x))
    return x


def solve(S, v, lam: float, return_y: bool = False):
    """Algorithm 1 end to end in FP64. Raises ``np.linalg.LinAlgError`` if the Cholesky fails."""
    S, n, m, lds = _S(S)
    v = _f64(v, (m,))
    x = np.empty(m, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    info = _load().oracle_solve(_p(S), n, m, lds, _p(v), float(lam), _p(x), _p(y))
    if info != 0:
        raise np.linalg.LinAlgError(f"oracle Cholesky failed at pivot {info}")
    return (x, y) if return_y else x


def residual(S, v, x, lam: float) -> np.ndarray:
    """r = v - lam x - S^T (S x): zero for the exact solution (Proposition 1, Appendix A)."""
    S, n, m, lds = _S(S)
    v = _f64(v, (m,))
    x = _f64(x, (m,))
    r = np.empty(m, dtype=np.float64)
    _load().oracle_residual(_p(S), n, m, lds, _p(v), _p(x), float(lam), _p(r))
    return r


def split_bf16(S) -> tuple[np.ndarray, np.ndarray]:
    """hi = bf16_RNE(S), lo = bf16_RNE(S - hi), returned as float32 arrays."""
    S, n, m, lds = _S(S)
    hi = np.empty((n, m), dtype=np.float32)
    lo = np.empty((n, m), dtype=np.float32)
    _load().oracle_split_bf16(_p(S), n, m, lds, _p(hi), _p(lo))
    return hi, lo


def gram3(hi, lo, lam: float = 0.0) -> np.ndarray:
    """sum_k hi_i hi_j + hi_i lo_j + lo_i hi_j (+ lam on the diagonal), FP64."""
    hi = np.ascontiguousarray(hi, dtype=np.float32)
    lo = np.ascontiguousarray(lo, dtype=np.float32)
    if hi.shape != lo.shape or hi.ndim != 2:
        raise ValueError("hi and lo must be matching 2-D arrays")
    n, m = hi.shape
    W = np.empty((n, n), dtype=np.float64)
    _load().oracle_gram3(_p(hi), _p(lo), n, m, float(lam), _p(W))
    return W


def quant_mxfp8(S) -> tuple[np.ndarray, np.ndarray]:
    """Block-scaled FP8 (E4M3) form of S: 32-column blocks per row, power-of-two scale 2^e with the
    smallest e such that no element exceeds 448 * 2^e, elements rounded to nearest even.
    Returns (deq, e): deq = q * 2^e as float32 (n x m), e as int32 (n x ceil(m/32))."""
    S, n, m, lds = _S(S)
    deq = np.empty((n, m), dtype=np.float32)
    e = np.empty((n, (m + 31) // 32), dtype=np.int32)
    _load().oracle_quant_mxfp8(_p(S), n, m, lds, _p(deq), _p(e))
    return deq, e


def row_norms(S) -> np.ndarray:
    """d_i = sum_k S_ik^2 (the diagonal of S S^T)."""
    S, n, m, lds = _S(S)
    d = np.empty(n, dtype=np.float64)
    _load().oracle_row_norms(_p(S), n, m, lds, _p(d))
    return d


def gram_entries(S, ii, jj, lam: float = 0.0) -> np.ndarray:
    """Entries W_{ii[p], jj[p]} of S S^T + lam I, one dot product each."""
    S, n, m, lds = _S(S)
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    if ii.shape != jj.shape or ii.ndim != 1:
        raise ValueError("index arrays must be 1-D and equal length")
    if ii.size and (ii.min() < 0 or jj.min() < 0 or ii.max() >= n or jj.max() >= n):
        raise IndexError("row index out of range")
    out = np.empty(ii.shape[0], dtype=np.float64)
    _load().oracle_gram_entries(_p(S), m, lds, float(lam), _p(ii), _p(jj), ii.shape[0], _p(out))
    return out


def solve_batched(S, lams, V) -> np.ndarray:
    """Algorithm 1 for every (lambda_l, v_r) pair: X[l, r] solves (S^T S + lambda_l I) x = v_r.
    Each pair is an independent application of Algorithm 1 (the Gram is shared)."""
    S, n, m, lds = _S(S)
    V = np.asarray(V, dtype=np.float64)
    if V.ndim == 1:
        V = V[None, :]
    G = gram(S, 0.0)
    out = np.empty((len(lams), V.shape[0], m), dtype=np.float64)
    for li, lam in enumerate(lams):
        W = G + float(lam) * np.eye(n)
        L, info = cholesky(W)
        if info != 0:
            raise np.linalg.LinAlgError(f"oracle Cholesky failed at pivot {info} (lambda={lam})")
        for r in range(V.shape[0]):
            y = backward(L, forward(L, gemv(S, V[r])))
            out[li, r] = apply(S, V[r], y, float(lam))
    return out


def solve_rowspace(S, f, lam: float, return_y: bool = False):
    """Appendix B: x = S^T (S S^T + lam I)^-1 f, the solution of Eq. 1 for v = S^T f, without
    forming v. Raises ``np.linalg.LinAlgError`` if the Cholesky fails."""
    S, n, m, lds = _S(S)
    f = _f64(f, (n,))
    x = np.empty(m, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    info = _load().oracle_solve_rowspace(_p(S), n, m, lds, _p(f), float(lam), _p(x), _p(y))
    if info != 0:
        raise np.linalg.LinAlgError(f"oracle Cholesky failed at pivot {info}")
    return (x, y) if return_y else x


def center(O) -> np.ndarray:
    """Section 3: S = (O - mean over samples of O) / sqrt(n), FP64 arithmetic, FP32 result."""
    O, n, m, ldo = _S(O)
    S = np.empty((n, m), dtype=np.float32)
    _load().oracle_center(_p(O), n, m, ldo, _p(S), m)
    return S


def center_complex(O) -> np.ndarray:
    """Section 3 for a complex O (complex64, n x m): the centered, scaled S in the stacked real form
    Z = [Re S; Im S], a 2n x m float32 array with rows 0..n-1 the real parts and rows n..2n-1 the
    imaginary parts."""
    O = np.ascontiguousarray(O, dtype=np.complex64)
    if O.ndim != 2:
        raise ValueError("O must be 2-D")
    n, m = O.shape
    Z = np.empty((2 * n, m), dtype=np.float32)
    _load().oracle_center_complex(_p(O), n, m, m, _p(Z), m)
    return Z


def project_centered(W, lam: float, nseg: int = 1) -> np.ndarray:
    """Preconditioner for a centered S (Section 3): M = P W P + lam U U^T, P = I - U U^T, U the
    normalised indicators of nseg equal contiguous segments of the n indices (1: the all-ones
    vector; 2: the real and imaginary halves of the complex variant's real embedding)."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    n = W.shape[0]
    if W.shape != (n, n) or nseg < 1 or n % nseg != 0:
        raise ValueError("W must be square with n divisible by nseg")
    M = np.empty((n, n), dtype=np.float64)
    _load().oracle_project_centered(_p(W), n, nseg, float(lam), _p(M))
    return M


def solve_complex(S, v, lam: float, return_y: bool = False):
    """Section 3, complex variant: x solving (S^H S + lam I) x = v by Algorithm 1 with Hermitian
    conjugates, in complex FP64. S: complex64 n x m; v: complex m. Raises
    ``np.linalg.LinAlgError`` if the Cholesky fails."""
    S = np.ascontiguousarray(S, dtype=np.complex64)
    if S.ndim != 2:
        raise ValueError("S must be 2-D")
    n, m = S.shape
    v = np.ascontiguousarray(v, dtype=np.complex128)
    if v.shape != (m,):
        raise ValueError(f"expected v of shape ({m},)")
    x = np.empty(m, dtype=np.complex128)
    y = np.empty(n, dtype=np.complex128)
    info = _load().oracle_solve_complex(_p(S), n, m, m, _p(v), float(lam), _p(x), _p(y))
    if info != 0:
        raise np.linalg.LinAlgError(f"oracle Cholesky failed at pivot {info}")
    return (x, y) if return_y else x
