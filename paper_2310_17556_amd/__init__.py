"""Python binding of the dfisher C ABI (include/dfisher.h): damped Fisher solves on MI355X.

Thin marshalling only: every function here has the name of a C entry point, checks tensor
dtypes/devices/layouts, allocates outputs with torch (device memory plumbing), passes raw device
pointers and torch's current HIP stream, and raises :class:`DfisherError` on a non-zero status.
All arithmetic happens in the HIP kernels of ``libdfisher.so``. There is no fallback: importing
this package works without the library, but the first call into it raises ImportError when
``libdfisher.so`` has not been built.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "DfisherError", "Info", "Timing", "lib",
    "DFISHER_OK", "DFISHER_E_INVALID_ARG", "DFISHER_E_NOT_SPD", "DFISHER_E_NO_MEMORY", "DFISHER_E_DEVICE",
    "DFISHER_E_UNSUPPORTED", "DFISHER_E_NOT_CONVERGED", "DFISHER_GRAM_FP32", "DFISHER_GRAM_BF16X3", "DFISHER_GRAM_MXFP8", "DFISHER_SHIFT_NONE",
    "DFISHER_SHIFT_ON_FAILURE", "DFISHER_SHIFT_ALWAYS",
    "dfisher_ctx_create", "dfisher_ctx_destroy", "dfisher_ctx_enable_timing", "dfisher_ctx_last_timing",
    "dfisher_ctx_enable_graphs", "dfisher_ctx_enable_autotune", "dfisher_autotune_gram", "dfisher_ctx_save_tuning",
    "dfisher_ctx_load_tuning",
    "dfisher_gram", "dfisher_quantize_mxfp8", "dfisher_potrf", "dfisher_gemv",
    "dfisher_trsv", "dfisher_apply", "dfisher_solve", "dfisher_factor_create", "dfisher_factor_solve",
    "dfisher_factor_copy_L", "dfisher_factor_destroy", "dfisher_solve_batched", "dfisher_solve_uneven",
    "dfisher_status_string", "dfisher_last_error", "dfisher_auto_sweeps", "DFISHER_SWEEPS_AUTO",
    "dfisher_solve_rowspace", "dfisher_factor_solve_noalloc", "dfisher_sr_center", "dfisher_solve_complex",
]

DFISHER_OK = 0
DFISHER_E_INVALID_ARG = 1
DFISHER_E_NOT_SPD = 2
DFISHER_E_NO_MEMORY = 3
DFISHER_E_DEVICE = 4
DFISHER_E_NOT_CONVERGED = 5
DFISHER_SWEEPS_AUTO = -1
DFISHER_E_UNSUPPORTED = 6
DFISHER_GRAM_FP32 = 0
DFISHER_GRAM_BF16X3 = 1
DFISHER_GRAM_MXFP8 = 2
DFISHER_SHIFT_NONE = 0
DFISHER_SHIFT_ON_FAILURE = 1
DFISHER_SHIFT_ALWAYS = 2
DFISHER_CENTERED = 1
DFISHER_ASYNC = 2
DFISHER_EXACT_APPLY = 4

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdfisher.so")


class _Options(ctypes.Structure):
    _fields_ = [("gram_prec", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("shift_policy", ctypes.c_int32), ("x_fp64", ctypes.c_int32), ("tol", ctypes.c_double),
                ("final_resid", ctypes.c_int32), ("flags", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("potrf_info", ctypes.c_int64), ("shift", ctypes.c_double),
                ("attempts", ctypes.c_int32), ("sweeps_done", ctypes.c_int32), ("resid", ctypes.c_double),
                ("w_resid", ctypes.c_double)]

    def as_dict(self):
        return {"potrf_info": self.potrf_info, "shift": self.shift, "attempts": self.attempts,
                "sweeps_done": self.sweeps_done, "resid": self.resid, "w_resid": self.w_resid}


class Timing(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in ("rowpass_ms", "gram_ms", "gram_reduce_ms", "potrf_ms", "trsv_ms",
                                                "refine_ms", "apply_ms", "total_ms")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2310_17556_amd.build` "
                          "(the HIP library is required; there is no fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "dfisher_ctx_create": ([ctypes.c_int, PP], I32),
        "dfisher_ctx_destroy": ([P], I32),
        "dfisher_gram": ([P, P, I64, I64, I64, I32, D, P, P], I32),
        "dfisher_potrf": ([P, P, I64, ctypes.POINTER(I64), P], I32),
        "dfisher_quantize_mxfp8": ([P, P, I64, I64, I64, P, I64, P, P], I32),
        "dfisher_gemv": ([P, P, I64, I64, I64, P, P, P], I32),
        "dfisher_trsv": ([P, P, I64, I32, P, P, P], I32),
        "dfisher_apply": ([P, P, I64, I64, I64, P, P, D, P, I32, P], I32),
        "dfisher_solve": ([P, P, I64, I64, I64, P, D, P, ctypes.POINTER(_Options), P, ctypes.POINTER(Info)], I32),
        "dfisher_solve_rowspace": ([P, P, I64, I64, I64, P, D, P, ctypes.POINTER(_Options), P,
                                    ctypes.POINTER(Info)], I32),
        "dfisher_factor_create": ([P, P, I64, I64, I64, D, ctypes.POINTER(_Options), P, PP, ctypes.POINTER(Info)], I32),
        "dfisher_factor_solve": ([P, P, I64, I64, P, I64, P, ctypes.POINTER(Info)], I32),
        "dfisher_factor_copy_L": ([P, P, P], I32),
        "dfisher_factor_solve_noalloc": ([P, P, P, P, ctypes.POINTER(Info)], I32),
        "dfisher_sr_center": ([P, P, I64, I64, I64, I32, P, I64, P], I32),
        "dfisher_solve_complex": ([P, P, I64, I64, I64, P, D, P, ctypes.POINTER(_Options), P,
                                   ctypes.POINTER(Info)], I32),
        "dfisher_factor_destroy": ([P], I32),
        "dfisher_solve_batched": ([P, P, I64, I64, I64, ctypes.POINTER(D), I32, P, I32, I64, P, I64,
                                   ctypes.POINTER(_Options), P, P], I32),   # infos: host, or device (ASYNC)
        "dfisher_solve_uneven": ([P, I32, PP, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64), PP,
                                  ctypes.POINTER(D), PP, ctypes.POINTER(_Options), P, ctypes.POINTER(Info)], I32),
        "dfisher_ctx_enable_timing": ([P, I32], I32),
        "dfisher_ctx_enable_graphs": ([P, I32], I32),
        "dfisher_ctx_enable_autotune": ([P, I32], I32),
        "dfisher_autotune_gram": ([P, P, I64, I64, I64, I32, P], I32),
        "dfisher_ctx_save_tuning": ([P, ctypes.c_char_p], I32),
        "dfisher_ctx_load_tuning": ([P, ctypes.c_char_p], I32),
        "dfisher_ctx_last_timing": ([P, ctypes.POINTER(Timing)], I32),
        "dfisher_auto_sweeps": ([I32, I64, I64], I32),
        "dfisher_status_string": ([I32], ctypes.c_char_p),
        "dfisher_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


_LIB = None


def _lib():
    """The loaded libdfisher.so (loaded on first use; raises ImportError if it was not built)."""
    global _LIB
    if _LIB is None:
        _LIB = _load()
    return _LIB


def __getattr__(name):
    if name == "lib":
        return _lib()
    raise AttributeError(name)


class DfisherError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = int(status)
        msg = _lib().dfisher_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib().dfisher_status_string(status).decode()} ({status}): {msg}")


def _check(status: int, where: str):
    if status != DFISHER_OK:
        raise DfisherError(status, where)


def dfisher_status_string(status: int) -> str:
    return _lib().dfisher_status_string(int(status)).decode()


def dfisher_last_error() -> str:
    return _lib().dfisher_last_error().decode(errors="replace")


# ----------------------------------------------------------------------------- marshalling helpers

def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _S_args(S):
    torch = _torch()
    if not isinstance(S, torch.Tensor) or S.dtype != torch.float32 or S.dim() != 2 or not S.is_cuda:
        raise TypeError("S must be a 2-D float32 CUDA tensor")
    if S.stride(1) != 1 or S.stride(0) < S.shape[1]:
        raise ValueError("S must be row-major with unit column stride and row stride >= m")
    n, m = S.shape
    return n, m, S.stride(0)


def _vec(t, length, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda:
        raise TypeError(f"{name} must be a {dtype} CUDA tensor")
    if t.numel() != length or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with {length} elements")


def _options(gram_prec, sweeps, shift_policy, x_fp64, final_resid=False, centered=False):
    o = _Options(int(gram_prec), int(sweeps), int(shift_policy), 1 if x_fp64 else 0)
    o.final_resid = 1 if final_resid else 0
    o.flags = DFISHER_CENTERED if centered else 0
    return o


def dfisher_auto_sweeps(gram_prec: int, n: int, m: int) -> int:
    """The sweep count DFISHER_SWEEPS_AUTO picks for an n x m problem (no shift); -1 for bad input."""
    return int(_lib().dfisher_auto_sweeps(int(gram_prec), int(n), int(m)))


class _Handle:
    """Owns a C handle and releases it with its destroy function."""

    def __init__(self, ptr, destroy, owner=None):
        self._ptr = ptr
        self._destroy = destroy
        self.owner = owner  # keeps borrowed tensors (S) alive

    @property
    def ptr(self):
        if not self._ptr:
            raise ValueError("handle already destroyed")
        return self._ptr

    def close(self):
        if self._ptr:
            self._destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- entry points

def dfisher_ctx_create(device: int = 0) -> _Handle:
    out = ctypes.c_void_p()
    _check(_lib().dfisher_ctx_create(int(device), ctypes.byref(out)), "dfisher_ctx_create")
    return _Handle(out.value, _lib().dfisher_ctx_destroy)


def dfisher_ctx_destroy(ctx: _Handle) -> None:
    ctx.close()


def dfisher_ctx_enable_timing(ctx, enable: bool = True) -> None:
    _check(_lib().dfisher_ctx_enable_timing(ctx.ptr, 1 if enable else 0), "dfisher_ctx_enable_timing")


def dfisher_ctx_enable_graphs(ctx, enable: bool = True) -> None:
    _check(_lib().dfisher_ctx_enable_graphs(ctx.ptr, 1 if enable else 0), "dfisher_ctx_enable_graphs")


def dfisher_ctx_enable_autotune(ctx, enable: bool = True) -> None:
    _check(_lib().dfisher_ctx_enable_autotune(ctx.ptr, 1 if enable else 0), "dfisher_ctx_enable_autotune")


def dfisher_autotune_gram(ctx, S, prec: int, stream=None) -> None:
    """Time the Gram stage's split-K candidates on S and keep the fastest for S's size class."""
    n, m, lds = _S_args(S)
    _check(_lib().dfisher_autotune_gram(ctx.ptr, _ptr(S), n, m, lds, int(prec), _stream(stream)),
           "dfisher_autotune_gram")


def dfisher_ctx_save_tuning(ctx, path: str) -> None:
    _check(_lib().dfisher_ctx_save_tuning(ctx.ptr, os.fsencode(path)), "dfisher_ctx_save_tuning")


def dfisher_ctx_load_tuning(ctx, path: str) -> None:
    _check(_lib().dfisher_ctx_load_tuning(ctx.ptr, os.fsencode(path)), "dfisher_ctx_load_tuning")


def dfisher_ctx_last_timing(ctx) -> dict:
    t = Timing()
    _check(_lib().dfisher_ctx_last_timing(ctx.ptr, ctypes.byref(t)), "dfisher_ctx_last_timing")
    return t.as_dict()


def dfisher_gram(ctx, S, prec: int = DFISHER_GRAM_FP32, lam: float = 0.0, W=None, stream=None):
    """W = S S^T + lam I (FP64 n x n, both triangles)."""
    torch = _torch()
    n, m, lds = _S_args(S)
    if W is None:
        W = torch.empty((n, n), dtype=torch.float64, device=S.device)
    _vec(W, n * n, torch.float64, "W")
    _check(_lib().dfisher_gram(ctx.ptr, _ptr(S), n, m, lds, int(prec), float(lam), _ptr(W), _stream(stream)),
           "dfisher_gram")
    return W


def dfisher_quantize_mxfp8(ctx, S, stream=None):
    """Scaled-FP8 form of S: returns (codes uint8 (n, ldq), scales uint8 (n, ldq // 32), ldq)."""
    torch = _torch()
    n, m, lds = _S_args(S)
    ldq = (m + 63) // 64 * 64
    codes = torch.empty((n, ldq), dtype=torch.uint8, device=S.device)
    scales = torch.empty((n, ldq // 32), dtype=torch.uint8, device=S.device)
    _check(_lib().dfisher_quantize_mxfp8(ctx.ptr, _ptr(S), n, m, lds, _ptr(codes), ldq, _ptr(scales),
                                         _stream(stream)), "dfisher_quantize_mxfp8")
    return codes, scales, ldq


def dfisher_potrf(ctx, W, stream=None) -> int:
    """In-place Cholesky of the FP64 n x n matrix W. Returns the info (0 on success); raises on
    failure with the info in the message."""
    torch = _torch()
    n = W.shape[0]
    _vec(W, n * n, torch.float64, "W")
    info = ctypes.c_int64(0)
    st = _lib().dfisher_potrf(ctx.ptr, _ptr(W), n, ctypes.byref(info), _stream(stream))
    if st == DFISHER_E_NOT_SPD:
        return int(info.value)
    _check(st, "dfisher_potrf")
    return 0


def dfisher_gemv(ctx, S, v, b=None, stream=None):
    torch = _torch()
    n, m, lds = _S_args(S)
    _vec(v, m, torch.float32, "v")
    if b is None:
        b = torch.empty(n, dtype=torch.float64, device=S.device)
    _vec(b, n, torch.float64, "b")
    _check(_lib().dfisher_gemv(ctx.ptr, _ptr(S), n, m, lds, _ptr(v), _ptr(b), _stream(stream)), "dfisher_gemv")
    return b


def dfisher_trsv(ctx, L, b, trans: int, y=None, stream=None):
    torch = _torch()
    n = L.shape[0]
    _vec(L, n * n, torch.float64, "L")
    _vec(b, n, torch.float64, "b")
    if y is None:
        y = torch.empty(n, dtype=torch.float64, device=L.device)
    _vec(y, n, torch.float64, "y")
    _check(_lib().dfisher_trsv(ctx.ptr, _ptr(L), n, int(trans), _ptr(b), _ptr(y), _stream(stream)), "dfisher_trsv")
    return y


def dfisher_apply(ctx, S, v, y, lam: float, x=None, x_fp64: bool = False, stream=None):
    torch = _torch()
    n, m, lds = _S_args(S)
    _vec(v, m, torch.float32, "v")
    _vec(y, n, torch.float64, "y")
    dt = torch.float64 if x_fp64 else torch.float32
    if x is None:
        x = torch.empty(m, dtype=dt, device=S.device)
    _vec(x, m, dt, "x")
    _check(_lib().dfisher_apply(ctx.ptr, _ptr(S), n, m, lds, _ptr(v), _ptr(y), float(lam), _ptr(x), 1 if x_fp64 else 0,
                             _stream(stream)), "dfisher_apply")
    return x


def dfisher_solve(ctx, S, v, lam: float, gram_prec: int = DFISHER_GRAM_FP32, sweeps: int = 0,
                  shift_policy: int = DFISHER_SHIFT_ON_FAILURE, x_fp64: bool = False, x=None, stream=None,
                  tol: float = 0.0, final_resid: bool = False, centered: bool = False, exact_apply: bool = False):
    """x solving (S^T S + lam I) x = v. Returns (x, info_dict). With tol > 0 the refinement stops at
    the tolerance (sweeps is the cap); info_dict["converged"] is False (and x is still the result)
    when the library returns DFISHER_E_NOT_CONVERGED. exact_apply sets DFISHER_EXACT_APPLY (the final
    step never takes the last correction through the FP8 codes)."""
    torch = _torch()
    n, m, lds = _S_args(S)
    _vec(v, m, torch.float32, "v")
    dt = torch.float64 if x_fp64 else torch.float32
    if x is None:
        x = torch.empty(m, dtype=dt, device=S.device)
    _vec(x, m, dt, "x")
    opt = _options(gram_prec, sweeps, shift_policy, x_fp64, final_resid, centered)
    opt.tol = float(tol)
    if exact_apply:
        opt.flags |= DFISHER_EXACT_APPLY
    info = Info()
    st = _lib().dfisher_solve(ctx.ptr, _ptr(S), n, m, lds, _ptr(v), float(lam), _ptr(x), ctypes.byref(opt),
                              _stream(stream), ctypes.byref(info))
    if st != DFISHER_E_NOT_CONVERGED:
        _check(st, "dfisher_solve")
    d = info.as_dict()
    d["converged"] = st == DFISHER_OK
    return x, d


def dfisher_solve_rowspace(ctx, S, f, lam: float, gram_prec: int = DFISHER_GRAM_FP32, sweeps: int = 0,
                           shift_policy: int = DFISHER_SHIFT_ON_FAILURE, x_fp64: bool = False, x=None, stream=None,
                           tol: float = 0.0, final_resid: bool = False, centered: bool = False):
    """x solving (S^T S + lam I) x = S^T f for an FP64 f of length n (the right-hand side in the row
    space of S), as x = S^T (S S^T + lam I)^-1 f. Returns (x, info_dict) like dfisher_solve."""
    torch = _torch()
    n, m, lds = _S_args(S)
    _vec(f, n, torch.float64, "f")
    dt = torch.float64 if x_fp64 else torch.float32
    if x is None:
        x = torch.empty(m, dtype=dt, device=S.device)
    _vec(x, m, dt, "x")
    opt = _options(gram_prec, sweeps, shift_policy, x_fp64, final_resid, centered)
    opt.tol = float(tol)
    info = Info()
    st = _lib().dfisher_solve_rowspace(ctx.ptr, _ptr(S), n, m, lds, _ptr(f), float(lam), _ptr(x), ctypes.byref(opt),
                                       _stream(stream), ctypes.byref(info))
    if st != DFISHER_E_NOT_CONVERGED:
        _check(st, "dfisher_solve_rowspace")
    d = info.as_dict()
    d["converged"] = st == DFISHER_OK
    return x, d


def dfisher_sr_center(ctx, O, S=None, stream=None):
    """Section 3: S = (O - mean over samples) / sqrt(n). O: 2-D float32 (n x m) or complex64 CUDA tensor
    with unit column stride. Returns S (n x m float32) for a real O, or the stacked Z = [Re S; Im S]
    (2n x m float32) for a complex O. For a real O, S may be O itself (in place)."""
    torch = _torch()
    if not isinstance(O, torch.Tensor) or O.dim() != 2 or not O.is_cuda or O.stride(1) != 1:
        raise TypeError("O must be a 2-D CUDA tensor with unit column stride")
    if O.dtype not in (torch.float32, torch.complex64):
        raise TypeError("O must be float32 or complex64")
    cplx = O.dtype == torch.complex64
    n, m = O.shape
    rows = 2 * n if cplx else n
    if S is None:
        S = torch.empty((rows, m), dtype=torch.float32, device=O.device)
    if S.dtype != torch.float32 or S.dim() != 2 or tuple(S.shape) != (rows, m) or S.stride(1) != 1:
        raise ValueError(f"S must be a ({rows}, {m}) float32 tensor with unit column stride")
    Op = torch.view_as_real(O) if cplx else O
    _check(_lib().dfisher_sr_center(ctx.ptr, _ptr(Op), n, m, O.stride(0), 1 if cplx else 0, _ptr(S), S.stride(0),
                                    _stream(stream)), "dfisher_sr_center")
    return S


def dfisher_solve_complex(ctx, Z, v, lam: float, gram_prec: int = DFISHER_GRAM_FP32, sweeps: int = 0,
                          shift_policy: int = DFISHER_SHIFT_ON_FAILURE, x_fp64: bool = False, x=None, stream=None,
                          tol: float = 0.0, final_resid: bool = False, centered: bool = False):
    """x solving (S^H S + lam I) x = v for S = A + iB given as Z = [A; B] (2n x m float32); v complex64
    of length m; x complex64 (or complex128 with x_fp64). Returns (x, info_dict) like dfisher_solve."""
    torch = _torch()
    N, m, lds = _S_args(Z)
    if N % 2:
        raise ValueError("Z must have an even number of rows ([Re S; Im S])")
    _vec(v, m, torch.complex64, "v")
    dt = torch.complex128 if x_fp64 else torch.complex64
    if x is None:
        x = torch.empty(m, dtype=dt, device=Z.device)
    _vec(x, m, dt, "x")
    opt = _options(gram_prec, sweeps, shift_policy, x_fp64, final_resid, centered)
    opt.tol = float(tol)
    info = Info()
    st = _lib().dfisher_solve_complex(ctx.ptr, _ptr(Z), N // 2, m, lds, _ptr(v), float(lam), _ptr(x),
                                      ctypes.byref(opt), _stream(stream), ctypes.byref(info))
    if st != DFISHER_E_NOT_CONVERGED:
        _check(st, "dfisher_solve_complex")
    d = info.as_dict()
    d["converged"] = st == DFISHER_OK
    return x, d


def dfisher_factor_create(ctx, S, lam: float, gram_prec: int = DFISHER_GRAM_FP32, sweeps: int = 0,
                          shift_policy: int = DFISHER_SHIFT_ON_FAILURE, x_fp64: bool = False, stream=None,
                          centered: bool = False):
    """Gram + Cholesky once. Returns (factor_handle, info_dict). The handle keeps S alive."""
    n, m, lds = _S_args(S)
    opt = _options(gram_prec, sweeps, shift_policy, x_fp64, centered=centered)
    out = ctypes.c_void_p()
    info = Info()
    _check(_lib().dfisher_factor_create(ctx.ptr, _ptr(S), n, m, lds, float(lam), ctypes.byref(opt), _stream(stream),
                                     ctypes.byref(out), ctypes.byref(info)), "dfisher_factor_create")
    h = _Handle(out.value, _lib().dfisher_factor_destroy, owner=(ctx, S))
    h.n, h.m, h.x_fp64 = n, m, bool(x_fp64)
    return h, info.as_dict()


def dfisher_factor_solve(f, V, X=None, stream=None):
    """Solve for the rows of V (nrhs x m, or a single m-vector). Returns X (same leading shape)."""
    torch = _torch()
    squeeze = V.dim() == 1
    V2 = V.unsqueeze(0) if squeeze else V
    if V2.dtype != torch.float32 or not V2.is_cuda or V2.stride(1) != 1:
        raise TypeError("V must be a float32 CUDA tensor with unit column stride")
    nrhs, m = V2.shape
    if m != f.m:
        raise ValueError("V has the wrong number of columns")
    dt = torch.float64 if f.x_fp64 else torch.float32
    if X is None:
        X = torch.empty((nrhs, m), dtype=dt, device=V.device)
    X2 = X.unsqueeze(0) if X.dim() == 1 else X
    if X2.dtype != dt or X2.stride(1) != 1 or tuple(X2.shape) != (nrhs, m):
        raise ValueError("X has the wrong dtype or shape")
    info = Info()
    _check(_lib().dfisher_factor_solve(f.ptr, _ptr(V2), nrhs, V2.stride(0), _ptr(X2), X2.stride(0), _stream(stream),
                                    ctypes.byref(info)), "dfisher_factor_solve")
    return X2[0] if squeeze else X2


def dfisher_factor_solve_noalloc(f, v, x, stream=None):
    """One right-hand side through the factor without any device allocation (the library's built-in
    scratch): x must be preallocated (length m, FP32 or FP64 per the factor's options). Returns
    the info dict."""
    torch = _torch()
    m = f.m
    _vec(v, m, torch.float32, "v")
    _vec(x, m, torch.float64 if f.x_fp64 else torch.float32, "x")
    info = Info()
    _check(_lib().dfisher_factor_solve_noalloc(f.ptr, _ptr(v), _ptr(x), _stream(stream), ctypes.byref(info)),
           "dfisher_factor_solve_noalloc")
    return info.as_dict()


def dfisher_factor_copy_L(f, L=None, stream=None):
    torch = _torch()
    if L is None:
        L = torch.empty((f.n, f.n), dtype=torch.float64, device="cuda")
    _vec(L, f.n * f.n, torch.float64, "L")
    _check(_lib().dfisher_factor_copy_L(f.ptr, _ptr(L), _stream(stream)), "dfisher_factor_copy_L")
    return L


def dfisher_factor_destroy(f) -> None:
    f.close()


def dfisher_solve_batched(ctx, S, lams, V, gram_prec: int = DFISHER_GRAM_FP32, sweeps: int = 0,
                          shift_policy: int = DFISHER_SHIFT_ON_FAILURE, x_fp64: bool = False, X=None, stream=None,
                          centered: bool = False, enqueue_only: bool = False, exact_apply: bool = False):
    """X[l, r] solves (S^T S + lams[l] I) x = V[r]. Returns (X of shape (nlam, nrhs, m), infos).

    enqueue_only sets DFISHER_ASYNC: nothing waits (the call may run under CUDA-graph capture) and
    infos is then a uint8 CUDA tensor of nlam records, decoded by batch_infos() once the stream is done."""
    torch = _torch()
    n, m, lds = _S_args(S)
    if V.dtype != torch.float32 or V.dim() != 2 or V.stride(1) != 1 or V.shape[1] != m:
        raise TypeError("V must be an (nrhs, m) float32 CUDA tensor with unit column stride")
    nrhs = V.shape[0]
    lam_arr = (ctypes.c_double * len(lams))(*[float(a) for a in lams])
    nlam = len(lams)
    dt = torch.float64 if x_fp64 else torch.float32
    if X is None:
        X = torch.empty((nlam, nrhs, m), dtype=dt, device=S.device)
    if X.dtype != dt or not X.is_contiguous() or tuple(X.shape) != (nlam, nrhs, m):
        raise ValueError("X must be a contiguous (nlam, nrhs, m) tensor of the output dtype")
    opt = _options(gram_prec, sweeps, shift_policy, x_fp64, centered=centered)
    if exact_apply:
        opt.flags |= DFISHER_EXACT_APPLY
    if enqueue_only:
        opt.flags |= DFISHER_ASYNC
        dinfos = torch.empty((nlam, ctypes.sizeof(Info)), dtype=torch.uint8, device=S.device)
        _check(_lib().dfisher_solve_batched(ctx.ptr, _ptr(S), n, m, lds, lam_arr, nlam, _ptr(V), nrhs, V.stride(0),
                                            _ptr(X), m, ctypes.byref(opt), _stream(stream),
                                            ctypes.c_void_p(dinfos.data_ptr())), "dfisher_solve_batched")
        return X, dinfos
    infos = (Info * nlam)()
    _check(_lib().dfisher_solve_batched(ctx.ptr, _ptr(S), n, m, lds, lam_arr, nlam, _ptr(V), nrhs, V.stride(0), _ptr(X),
                                     m, ctypes.byref(opt), _stream(stream), infos), "dfisher_solve_batched")
    return X, [i.as_dict() for i in infos]


def batch_infos(dinfos):
    """Decode the device records of an enqueue_only batched call (after its stream has finished)."""
    raw = bytes(dinfos.cpu().numpy().tobytes())
    k = len(raw) // ctypes.sizeof(Info)
    arr = (Info * k).from_buffer_copy(raw)
    return [i.as_dict() for i in arr]


def dfisher_solve_uneven(ctx, Ss, vs, lams, gram_prec: int = DFISHER_GRAM_FP32, sweeps: int = 0,
                         shift_policy: int = DFISHER_SHIFT_ON_FAILURE, x_fp64: bool = False, xs=None, stream=None,
                         final_resid: bool = False, tol: float = 0.0, centered: bool = False,
                         exact_apply: bool = False):
    """Independent problems of different shapes. Returns (list of x, infos); "converged" is False in
    every info when the library returned DFISHER_E_NOT_CONVERGED (a tolerance, given or automatic,
    missed at some problem's sweep cap; every x is still written). When a problem fails to factor
    the DfisherError (status DFISHER_E_NOT_SPD) carries .infos and .xs of every problem.
    exact_apply sets DFISHER_EXACT_APPLY."""
    torch = _torch()
    k = len(Ss)
    if not (len(vs) == len(lams) == k):
        raise ValueError("Ss, vs and lams must have the same length")
    dims = [_S_args(S) for S in Ss]
    for (n, m, _), v in zip(dims, vs):
        _vec(v, m, torch.float32, "v")
    dt = torch.float64 if x_fp64 else torch.float32
    if xs is None:
        xs = [torch.empty(m, dtype=dt, device=S.device) for (n, m, _), S in zip(dims, Ss)]
    PArr = ctypes.c_void_p * k
    I64Arr = ctypes.c_int64 * k
    s_arr = PArr(*[S.data_ptr() for S in Ss])
    v_arr = PArr(*[v.data_ptr() for v in vs])
    x_arr = PArr(*[x.data_ptr() for x in xs])
    n_arr = I64Arr(*[d[0] for d in dims])
    m_arr = I64Arr(*[d[1] for d in dims])
    l_arr = I64Arr(*[d[2] for d in dims])
    lam_arr = (ctypes.c_double * k)(*[float(a) for a in lams])
    opt = _options(gram_prec, sweeps, shift_policy, x_fp64, final_resid, centered)
    opt.tol = float(tol)
    if exact_apply:
        opt.flags |= DFISHER_EXACT_APPLY
    infos = (Info * k)()
    st = _lib().dfisher_solve_uneven(ctx.ptr, k, s_arr, n_arr, m_arr, l_arr, v_arr, lam_arr, x_arr, ctypes.byref(opt),
                                     _stream(stream), infos)
    if st == DFISHER_E_NOT_SPD:
        # every problem's record is written: the error carries them (and the x's), so that the
        # caller can tell which problem failed to factor
        err = DfisherError(st, "dfisher_solve_uneven")
        err.infos = [i.as_dict() for i in infos]
        err.xs = xs
        raise err
    if st != DFISHER_E_NOT_CONVERGED:
        _check(st, "dfisher_solve_uneven")
    out = [i.as_dict() for i in infos]
    for d in out:
        d["converged"] = st == DFISHER_OK   # the status covers every problem of the call
    return xs, out
