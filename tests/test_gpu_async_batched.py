"""Enqueue-only batched solves (DFISHER_ASYNC) through the C ABI: nothing waits for the device, the
per-lambda records stay on the device, and the call can be captured into a graph and replayed.

* Eager: X bit for bit equal to the synchronising call's, and the device records equal to the host
  records that call returns (fixed and automatic sweeps, no shift and the up-front shift, one and
  two groups of 16 vectors per pass), and every pair within 1e-6 of Algorithm 1 run by the oracle.
* Captured: one call captured into a CUDA graph on a fresh context after one eager call of the
  same shapes, replayed three times with other device work and synchronisations between the
  replays; every replay's X and records equal the eager call's bit for bit.
* The capture fixes that context's workspace: a later call that needs more is refused with
  DFISHER_E_UNSUPPORTED, while calls of the captured shapes keep working.
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


def _new_ctx(dfl):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return dfl.dfisher_ctx_create(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = [
    # n, m, nlam, nrhs, prec, sweeps, policy
    (192, 40000, 3, 2, 2, 3, "none"),      # 6 vectors: one ragged group
    (128, 32768, 4, 9, 2, -1, "always"),   # 36 vectors: two-group passes, then a ragged group; automatic sweeps
    (96, 9001, 2, 5, 1, 1, "none"),        # split-BF16 Gram, unaligned row length
]


@pytest.mark.parametrize("n,m,nlam,nrhs,prec,sweeps,policy", CASES)
def test_async_equals_sync(dfl, oracle_mod, n, m, nlam, nrhs, prec, sweeps, policy):
    print(f"[async batched] n={n} m={m} nlam={nlam} nrhs={nrhs} prec={prec} sweeps={sweeps} {policy}", flush=True)
    ctx = _new_ctx(dfl)
    S = synth.make_S(n, m, synth.seed(61, n), "iid")
    V = synth.make_V(m, nrhs, synth.seed(61, n))
    lams = list(np.logspace(-6, -2, nlam))
    pol = dfl.DFISHER_SHIFT_ALWAYS if policy == "always" else dfl.DFISHER_SHIFT_NONE
    Sd, Vd = dev(S), dev(V)
    X0, inf0 = dfl.dfisher_solve_batched(ctx, Sd, lams, Vd, gram_prec=prec, sweeps=sweeps, shift_policy=pol,
                                         x_fp64=True)
    X1, dinf = dfl.dfisher_solve_batched(ctx, Sd, lams, Vd, gram_prec=prec, sweeps=sweeps, shift_policy=pol,
                                         x_fp64=True, enqueue_only=True)
    torch.cuda.synchronize()
    assert torch.equal(X0, X1)
    inf1 = dfl.batch_infos(dinf)
    assert inf1 == inf0, (inf1, inf0)
    for d in inf1:
        assert d["potrf_info"] == 0 and d["attempts"] == 1 and d["resid"] == -1.0
        assert (d["shift"] > 0.0) == (policy == "always")
    Xref = oracle_mod.solve_batched(S, lams, V)
    X = X1.cpu().numpy()
    for li in range(nlam):
        for r in range(nrhs):
            assert rel(X[li, r], Xref[li, r]) <= 1e-6, (li, r)
    ctx.close()


def test_async_graph_replay(dfl):
    n, m, nlam, nrhs = 160, 24000, 3, 6
    print(f"[async batched graph] n={n} m={m} nlam={nlam} nrhs={nrhs}", flush=True)
    ctx = _new_ctx(dfl)
    other = _new_ctx(dfl)
    S = synth.make_S(n, m, synth.seed(62, n), "iid")
    V = synth.make_V(m, nrhs, synth.seed(62, n))
    lams = [1e-5, 1e-3, 1e-1]
    Sd, Vd = dev(S), dev(V)
    kw = dict(gram_prec=2, sweeps=2, shift_policy=dfl.DFISHER_SHIFT_NONE)
    # the eager call sizes the workspace (no allocation may happen during the capture)
    Xref, infref = dfl.dfisher_solve_batched(ctx, Sd, lams, Vd, **kw)
    torch.cuda.synchronize()
    X = torch.empty_like(Xref)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        _, dinf = dfl.dfisher_solve_batched(ctx, Sd, lams, Vd, X=X, enqueue_only=True, **kw)
    torch.cuda.synchronize()
    S2 = synth.make_S(96, 5000, synth.seed(63, 96), "iid")
    V2 = synth.make_V(5000, 2, synth.seed(63, 96))
    for rep in range(3):
        X.fill_(float("nan"))
        dinf.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        print(f"    replay {rep}", flush=True)
        assert torch.equal(X, Xref), rep
        assert dfl.batch_infos(dinf) == infref, rep
        # other device work between replays, on another context
        dfl.dfisher_solve_batched(other, dev(S2), [1e-3], dev(V2), gram_prec=2, sweeps=1)
        torch.cuda.synchronize()
    # the captured context's workspace is fixed now: a larger call is refused, the captured shapes still run
    Sbig = dev(synth.make_S(2 * n, m, synth.seed(64, n), "iid"))
    with pytest.raises(dfl.DfisherError) as e:
        dfl.dfisher_solve_batched(ctx, Sbig, lams, Vd, **kw)
    assert e.value.status == dfl.DFISHER_E_UNSUPPORTED
    Xagain, _ = dfl.dfisher_solve_batched(ctx, Sd, lams, Vd, **kw)
    assert torch.equal(Xagain, Xref)
    del g
    ctx.close()
    other.close()
