"""Seeded synthetic inputs for the damped Fisher solve.

This module only draws inputs: it holds none of the solve's arithmetic, and both the HIP
library's tests and the FP64 oracle receive the arrays it produces. The recipes follow the
score-matrix structure of the paper (S_ij = n^-1/2 d log P(x_i)/d theta_j, Section 2) with the
stochastic-reconfiguration centering S = (O - mean(O)) / sqrt(n) (Section 3):

* ``iid``     - S = fl32(G / sqrt(n)), G iid N(0,1), then column-centered; v iid N(0,1).
* ``scaled``  - S = fl32(G * d_j / sqrt(n)) with column scales d_j = 10^U(-3,0) (log-uniform in
                [1e-3, 1]), then column-centered; v = fl32(S^T u + e), u iid N(0,1)^n,
                e iid N(0, (1e-3)^2). v then lies almost entirely in the row space of S.

Column centering: mu_j = mean_i S_ij in FP64, S_ij <- fl32(S_ij - mu_j).

Two back ends draw the same recipe: numpy on the host (``make_*``), for sizes the oracle can
handle, and torch on a device (``make_*_torch``), for the full-scale workloads that would not
fit the host. The two back ends use different random streams; a test always hands the same
bytes to both sides.

* ``make_O``  - the raw matrix the SR front end centers: per-column offsets 3 N(0,1) plus iid
                N(0,1) samples (real, or complex with independent parts); ``make_vc`` draws a
                complex right-hand side.

Seeds: ``seed(c, p) = 2310017556 + 100 c + p`` for workload c and problem p.
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 2310017556


def seed(workload: int, problem: int = 0) -> int:
    return BASE_SEED + 100 * workload + problem


# --------------------------------------------------------------------------- host (numpy)

def _center_columns(S: np.ndarray) -> np.ndarray:
    mu = S.astype(np.float64).mean(axis=0)
    return (S.astype(np.float64) - mu).astype(np.float32)


def make_S(n: int, m: int, seed_: int, kind: str = "iid", center: bool = True) -> np.ndarray:
    """n x m float32 score-like matrix (row-major, contiguous)."""
    rng = np.random.default_rng(seed_)
    G = rng.standard_normal((n, m), dtype=np.float64)
    if kind == "iid":
        S = (G / math.sqrt(n)).astype(np.float32)
    elif kind == "scaled":
        d = 10.0 ** rng.uniform(-3.0, 0.0, size=m)
        S = (G * d / math.sqrt(n)).astype(np.float32)
    else:
        raise ValueError(f"unknown kind {kind!r}")
    return _center_columns(S) if center else np.ascontiguousarray(S)


def make_v(S: np.ndarray, seed_: int, kind: str = "iid") -> np.ndarray:
    """Right-hand side of length m (float32)."""
    rng = np.random.default_rng(seed_ + 7)
    n, m = S.shape
    if kind == "iid":
        return rng.standard_normal(m).astype(np.float32)
    if kind == "scaled":
        u = rng.standard_normal(n)
        e = rng.normal(0.0, 1e-3, size=m)
        return (S.astype(np.float64).T @ u + e).astype(np.float32)
    raise ValueError(f"unknown kind {kind!r}")


def make_O(n: int, m: int, seed_: int, complex_: bool = False) -> np.ndarray:
    """Raw log-derivative-like matrix O (n samples x m parameters) for the SR front end: every
    column has its own offset mu_j ~ 3 N(0,1) plus iid N(0,1) sample noise, so that centering
    removes a mean larger than the spread. float32 (n x m) or, with complex_, complex64 whose real
    and imaginary parts are drawn independently the same way."""
    rng = np.random.default_rng(seed_ + 17)
    if not complex_:
        mu = 3.0 * rng.standard_normal(m)
        return (mu + rng.standard_normal((n, m))).astype(np.float32)
    mr, mi = 3.0 * rng.standard_normal(m), 3.0 * rng.standard_normal(m)
    re = (mr + rng.standard_normal((n, m))).astype(np.float32)
    im = (mi + rng.standard_normal((n, m))).astype(np.float32)
    return (re + 1j * im.astype(np.float64)).astype(np.complex64)


def make_vc(m: int, seed_: int) -> np.ndarray:
    """Complex right-hand side of length m (complex64), real and imaginary parts iid N(0,1)."""
    rng = np.random.default_rng(seed_ + 19)
    return (rng.standard_normal(m) + 1j * rng.standard_normal(m)).astype(np.complex64)


def make_V(m: int, nrhs: int, seed_: int) -> np.ndarray:
    """nrhs x m float32 right-hand sides, iid N(0,1) (row r is v_r)."""
    rng = np.random.default_rng(seed_ + 11)
    return rng.standard_normal((nrhs, m)).astype(np.float32)


def lambdas_logspaced(lo: float, hi: float, count: int) -> np.ndarray:
    """count values 10^(log10 lo + k (log10 hi - log10 lo)/(count-1)), both ends included."""
    if count == 1:
        return np.array([lo], dtype=np.float64)
    k = np.arange(count, dtype=np.float64)
    return 10.0 ** (math.log10(lo) + k * (math.log10(hi) - math.log10(lo)) / (count - 1))


def uneven_shapes(nprob: int, seed_: int, n_range=(256, 2048), m_range=(100_000, 2_000_000),
                  lam_range=(1e-5, 1e-2)):
    """Per-problem (n, m, lambda): log-uniform in the given ranges, n and m rounded to the
    nearest integer (no rounding to tile multiples)."""
    rng = np.random.default_rng(seed_ + 13)

    def logu(lo, hi, size):
        return np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))

    ns = np.rint(logu(*n_range, nprob)).astype(np.int64)
    ms = np.rint(logu(*m_range, nprob)).astype(np.int64)
    lams = logu(*lam_range, nprob)
    return ns, ms, lams


# --------------------------------------------------------------------------- device (torch)

def make_S_torch(n: int, m: int, seed_: int, device, kind: str = "iid", center: bool = True,
                 row_chunk: int = 256, ld: int | None = None):
    """Same recipe as :func:`make_S`, drawn on ``device`` with torch's generator, for sizes the
    host cannot hold. Returns an (n, ld) float32 tensor whose first m columns hold S (ld >= m);
    pass ``out[:, :m]`` or use ld as the row stride. Centering accumulates column means in FP64
    chunk by chunk and subtracts them in FP64 before rounding to FP32."""
    import torch

    ld = m if ld is None else ld
    if ld < m:
        raise ValueError("ld < m")
    g = torch.Generator(device=device)
    g.manual_seed(seed_)
    buf = torch.empty((n, ld), dtype=torch.float32, device=device)
    S = buf[:, :m]
    scale = None
    if kind == "scaled":
        scale = torch.pow(10.0, torch.empty(m, dtype=torch.float64, device=device).uniform_(-3.0, 0.0,
                                                                                           generator=g))
    elif kind != "iid":
        raise ValueError(f"unknown kind {kind!r}")
    inv = 1.0 / math.sqrt(n)
    for r0 in range(0, n, row_chunk):
        r1 = min(n, r0 + row_chunk)
        blk = torch.randn((r1 - r0, m), dtype=torch.float32, device=device, generator=g)
        if scale is None:
            S[r0:r1] = (blk.double() * inv).float()
        else:
            S[r0:r1] = (blk.double() * scale * inv).float()
        del blk
    if center:
        mu = torch.zeros(m, dtype=torch.float64, device=device)
        for r0 in range(0, n, row_chunk):
            mu += S[r0:min(n, r0 + row_chunk)].double().sum(dim=0)
        mu /= n
        for r0 in range(0, n, row_chunk):
            r1 = min(n, r0 + row_chunk)
            S[r0:r1] = (S[r0:r1].double() - mu).float()
    if ld > m:
        buf[:, m:] = 0.0
    return buf


def make_v_torch(S, seed_: int, kind: str = "iid", m: int | None = None):
    """Same recipe as :func:`make_v` on S's device. S may carry padding columns; m is the
    logical column count (defaults to S.shape[1])."""
    import torch

    n = S.shape[0]
    m = S.shape[1] if m is None else m
    g = torch.Generator(device=S.device)
    g.manual_seed(seed_ + 7)
    if kind == "iid":
        return torch.randn(m, dtype=torch.float32, device=S.device, generator=g)
    if kind == "scaled":
        u = torch.randn(n, dtype=torch.float64, device=S.device, generator=g)
        acc = torch.zeros(m, dtype=torch.float64, device=S.device)
        for r0 in range(0, n, 256):
            r1 = min(n, r0 + 256)
            acc += (S[r0:r1, :m].double() * u[r0:r1, None]).sum(dim=0)
        acc += torch.randn(m, dtype=torch.float64, device=S.device, generator=g) * 1e-3
        return acc.float()
    raise ValueError(f"unknown kind {kind!r}")


def make_V_torch(m: int, nrhs: int, seed_: int, device):
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed_ + 11)
    return torch.randn((nrhs, m), dtype=torch.float32, device=device, generator=g)
