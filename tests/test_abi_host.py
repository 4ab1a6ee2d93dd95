"""Host-side checks of the C ABI that need no GPU: the library loads, exports every entry point
declared in include/dfisher.h, rejects invalid arguments before touching a device, and reports
a missing device as DFISHER_E_DEVICE."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    with open(os.path.join(ROOT, "include", "dfisher.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dfisher_[A-Za-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def dfl():
    import paper_2310_17556_amd as dfl
    return dfl


def test_header_declares_entry_points():
    names = _header_functions()
    for required in ["dfisher_ctx_create", "dfisher_ctx_destroy", "dfisher_gram", "dfisher_potrf",
                     "dfisher_gemv", "dfisher_trsv", "dfisher_apply", "dfisher_solve", "dfisher_factor_create",
                     "dfisher_factor_solve", "dfisher_factor_copy_L", "dfisher_factor_destroy",
                     "dfisher_solve_batched", "dfisher_solve_uneven", "dfisher_status_string",
                     "dfisher_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol(dfl):
    lib = ctypes.CDLL(dfl.LIB_PATH)
    for name in _header_functions():
        assert hasattr(lib, name), f"{name} declared in dfisher.h but not exported"


def test_binding_names_match_abi(dfl):
    for name in _header_functions():
        assert hasattr(dfl, name), f"binding lacks {name}"


def test_status_strings(dfl):
    for code in range(7):
        assert dfl.dfisher_status_string(code) != "unknown status"
    assert dfl.dfisher_status_string(99) == "unknown status"


FAKE_CTX = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first
FAKE_DEV = ctypes.c_void_p(0x2000)


def _opts(dfl, prec=0, sweeps=0, shift=1, x64=0, tol=0.0, final=0, flags=0):
    return dfl._Options(prec, sweeps, shift, x64, tol, final, flags)


def test_invalid_arguments_rejected_on_host(dfl):
    lib = dfl.lib
    E = dfl.DFISHER_E_INVALID_ARG
    P = FAKE_DEV
    st = ctypes.c_void_p(0)
    # null context
    assert lib.dfisher_gram(None, P, 4, 8, 8, 0, 0.0, P, st) == E
    # bad sizes and strides
    assert lib.dfisher_gram(FAKE_CTX, P, 0, 8, 8, 0, 0.0, P, st) == E
    assert lib.dfisher_gram(FAKE_CTX, P, 4, 0, 8, 0, 0.0, P, st) == E
    assert lib.dfisher_gram(FAKE_CTX, P, 4, 8, 7, 0, 0.0, P, st) == E
    assert lib.dfisher_gram(FAKE_CTX, None, 4, 8, 8, 0, 0.0, P, st) == E
    assert lib.dfisher_gram(FAKE_CTX, P, 4, 8, 8, 0, 0.0, None, st) == E
    assert lib.dfisher_gram(FAKE_CTX, P, 4, 8, 8, 7, 0.0, P, st) == E      # unknown precision
    assert lib.dfisher_gram(FAKE_CTX, P, 4, 8, 8, 0, -1.0, P, st) == E     # lambda < 0
    assert lib.dfisher_gram(FAKE_CTX, P, 4, 8, 8, 0, float("nan"), P, st) == E
    info = dfl.Info()
    for lam in [0.0, -1e-3, float("inf"), float("nan")]:
        assert lib.dfisher_solve(FAKE_CTX, P, 4, 8, 8, P, lam, P, None, st, ctypes.byref(info)) == E
    for o in [_opts(dfl, prec=5), _opts(dfl, sweeps=-2), _opts(dfl, sweeps=17), _opts(dfl, shift=3),
              _opts(dfl, x64=2), _opts(dfl, tol=-1e-9), _opts(dfl, tol=float("nan")), _opts(dfl, tol=float("inf")),
              _opts(dfl, final=2), _opts(dfl, flags=8), _opts(dfl, flags=-1)]:
        assert lib.dfisher_solve(FAKE_CTX, P, 4, 8, 8, P, 1.0, P, ctypes.byref(o), st, None) == E
    assert lib.dfisher_solve(FAKE_CTX, P, 4, 8, 8, None, 1.0, P, None, st, None) == E
    assert lib.dfisher_solve(FAKE_CTX, P, 4, 8, 8, P, 1.0, None, None, st, None) == E
    for lam in [0.0, -1e-3, float("inf"), float("nan")]:
        assert lib.dfisher_solve_rowspace(FAKE_CTX, P, 4, 8, 8, P, lam, P, None, st, None) == E
    assert lib.dfisher_solve_rowspace(FAKE_CTX, P, 4, 8, 8, None, 1.0, P, None, st, None) == E
    assert lib.dfisher_solve_rowspace(FAKE_CTX, P, 4, 8, 8, P, 1.0, None, None, st, None) == E
    assert lib.dfisher_solve_rowspace(FAKE_CTX, P, 4, 8, 7, P, 1.0, P, None, st, None) == E
    assert lib.dfisher_solve_rowspace(FAKE_CTX, P, 4, 8, 8, P, 1.0, P, ctypes.byref(_opts(dfl, prec=5)), st, None) == E
    i64 = ctypes.c_int64(0)
    assert lib.dfisher_potrf(FAKE_CTX, P, 0, ctypes.byref(i64), st) == E
    assert lib.dfisher_potrf(FAKE_CTX, P, 4, None, st) == E
    assert lib.dfisher_trsv(FAKE_CTX, P, 4, 2, P, P, st) == E
    assert lib.dfisher_trsv(FAKE_CTX, P, 0, 0, P, P, st) == E
    assert lib.dfisher_apply(FAKE_CTX, P, 4, 8, 8, P, P, 0.0, P, 0, st) == E
    assert lib.dfisher_apply(FAKE_CTX, P, 4, 8, 8, P, P, 1.0, P, 3, st) == E
    assert lib.dfisher_gemv(FAKE_CTX, P, 4, 8, 8, None, P, st) == E
    out = ctypes.c_void_p()
    assert lib.dfisher_factor_create(FAKE_CTX, P, 4, 8, 8, 0.0, None, st, ctypes.byref(out), None) == E
    assert lib.dfisher_factor_create(FAKE_CTX, P, 4, 8, 8, 1.0, None, st, None, None) == E
    assert lib.dfisher_factor_solve(None, P, 1, 8, P, 8, st, None) == E
    lams = (ctypes.c_double * 2)(1e-3, -1.0)
    assert lib.dfisher_solve_batched(FAKE_CTX, P, 4, 8, 8, lams, 2, P, 1, 8, P, 8, None, st, None) == E
    lams = (ctypes.c_double * 1)(1e-3)
    assert lib.dfisher_solve_batched(FAKE_CTX, P, 4, 8, 8, lams, 0, P, 1, 8, P, 8, None, st, None) == E
    assert lib.dfisher_solve_batched(FAKE_CTX, P, 4, 8, 8, lams, 1, P, 1, 7, P, 8, None, st, None) == E
    assert lib.dfisher_solve_uneven(FAKE_CTX, 0, None, None, None, None, None, None, None, None, st, None) == E
    # a tolerance is honoured by dfisher_solve only; the fixed-sweep entry points refuse it
    U = dfl.DFISHER_E_UNSUPPORTED
    otol = _opts(dfl, sweeps=2, tol=1e-9)
    assert lib.dfisher_solve_batched(FAKE_CTX, P, 4, 8, 8, lams, 1, P, 1, 8, P, 8, ctypes.byref(otol), st, None) == U
    assert lib.dfisher_factor_create(FAKE_CTX, P, 4, 8, 8, 1.0, ctypes.byref(otol), st, ctypes.byref(out), None) == U
    arrp = (ctypes.c_void_p * 1)(P.value)
    arr64 = (ctypes.c_int64 * 1)(8)
    arrn = (ctypes.c_int64 * 1)(4)
    # the uneven call honours a tolerance (measured on the device); a negative one is rejected
    oneg = _opts(dfl, sweeps=2, tol=-1e-9)
    assert lib.dfisher_solve_uneven(FAKE_CTX, 1, arrp, arrn, arr64, arr64, arrp, lams, arrp, ctypes.byref(oneg), st,
                                    None) == E
    # the final-residual measurement is offered by dfisher_solve and dfisher_solve_uneven only
    ofin = _opts(dfl, sweeps=1, final=1)
    assert lib.dfisher_solve_batched(FAKE_CTX, P, 4, 8, 8, lams, 1, P, 1, 8, P, 8, ctypes.byref(ofin), st, None) == U
    assert lib.dfisher_factor_create(FAKE_CTX, P, 4, 8, 8, 1.0, ctypes.byref(ofin), st, ctypes.byref(out), None) == U
    assert "NULL" in dfl.dfisher_last_error() or dfl.dfisher_last_error() != ""
    # enqueue-only (DFISHER_ASYNC) is honoured by the batched call only, and there without the
    # host-decided shift escalation
    oasync = _opts(dfl, sweeps=1, shift=0, flags=dfl.DFISHER_ASYNC)
    assert lib.dfisher_solve(FAKE_CTX, P, 4, 8, 8, P, 1.0, P, ctypes.byref(oasync), st, None) == U
    assert lib.dfisher_solve_rowspace(FAKE_CTX, P, 4, 8, 8, P, 1.0, P, ctypes.byref(oasync), st, None) == U
    assert lib.dfisher_solve_complex(FAKE_CTX, P, 4, 8, 8, P, 1.0, P, ctypes.byref(oasync), st, None) == U
    assert lib.dfisher_factor_create(FAKE_CTX, P, 4, 8, 8, 1.0, ctypes.byref(oasync), st, ctypes.byref(out), None) == U
    assert lib.dfisher_solve_uneven(FAKE_CTX, 1, arrp, arrn, arr64, arr64, arrp, lams, arrp, ctypes.byref(oasync), st,
                                    None) == U
    oasync_fail = _opts(dfl, sweeps=1, shift=1, flags=dfl.DFISHER_ASYNC)
    assert lib.dfisher_solve_batched(FAKE_CTX, P, 4, 8, 8, lams, 1, P, 1, 8, P, 8, ctypes.byref(oasync_fail), st,
                                     None) == U
    # context switches and the tuning table
    assert lib.dfisher_ctx_enable_graphs(None, 1) == E
    assert lib.dfisher_ctx_enable_autotune(None, 1) == E
    assert lib.dfisher_autotune_gram(None, P, 4, 8, 8, 1, st) == E
    assert lib.dfisher_autotune_gram(FAKE_CTX, P, 4, 8, 8, 7, st) == E
    assert lib.dfisher_autotune_gram(FAKE_CTX, P, 4, 8, 7, 1, st) == E
    assert lib.dfisher_ctx_save_tuning(None, b"/tmp/x") == E
    assert lib.dfisher_ctx_load_tuning(None, b"/tmp/x") == E
    assert lib.dfisher_ctx_load_tuning(FAKE_CTX, None) == E
    # a nonexistent file is rejected before the context is touched
    assert lib.dfisher_ctx_load_tuning(FAKE_CTX, b"/nonexistent/dir/tune.txt") == E


def test_context_on_missing_device(dfl):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    out = ctypes.c_void_p()
    assert dfl.lib.dfisher_ctx_create(0, ctypes.byref(out)) == dfl.DFISHER_E_DEVICE
    assert out.value is None
    assert dfl.lib.dfisher_ctx_create(-1, ctypes.byref(out)) == dfl.DFISHER_E_INVALID_ARG
    assert dfl.lib.dfisher_ctx_create(0, None) == dfl.DFISHER_E_INVALID_ARG
    with pytest.raises(dfl.DfisherError) as ei:
        dfl.dfisher_ctx_create(0)
    assert ei.value.status == dfl.DFISHER_E_DEVICE
    assert dfl.lib.dfisher_ctx_destroy(None) == dfl.DFISHER_OK


def test_auto_sweeps_rule(dfl):
    """DFISHER_SWEEPS_AUTO's count: c = C / (sqrt(a) (1 - 1/sqrt(a))^2), a = m / n, and the smallest k
    with c^(k+1) <= 1e-7 (C = 0.1 scaled FP8, 1e-4 split-BF16, 1e-5 FP32; a <= 4 uses (1/2)^2), plus
    3 (a < 150) or 2 (a < 600) for the scaled-FP8 Gram; at most 16."""
    def rule(prec, n, m):
        a = m / n
        C = {0: 1e-5, 1: 1e-4, 2: 0.1}[prec]
        gap = (1 - a ** -0.5) ** 2 if a > 4 else 0.25
        c = C / (max(a, 1.0) ** 0.5 * gap)
        if not c < 0.5:
            return 16
        k, e = 0, c
        while e > 1e-7 and k < 16:
            e *= c
            k += 1
        if prec == 2:   # outlier directions of the scaled-FP8 Gram converge after the bulk
            k += 3 if a < 150 else (2 if a < 600 else 0)
        return min(k, 16)
    for prec in (0, 1, 2):
        for n, m in [(4096, 4_000_000), (2048, 2_000_000), (300, 20000), (1241, 119782), (32, 1024),
                     (1000, 1000), (64, 100), (1, 777)]:
            assert dfl.dfisher_auto_sweeps(prec, n, m) == rule(prec, n, m), (prec, n, m)
    # the headline shape needs two sweeps of the scaled-FP8 Gram and one of the others
    assert dfl.dfisher_auto_sweeps(2, 4096, 4_000_000) == 2
    assert dfl.dfisher_auto_sweeps(1, 4096, 4_000_000) == 1
    assert dfl.dfisher_auto_sweeps(3, 10, 10) == -1 and dfl.dfisher_auto_sweeps(0, 0, 10) == -1
