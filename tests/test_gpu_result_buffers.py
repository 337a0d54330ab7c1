"""Result blocks of the caller (pdlpb_set_result_buffers) through the C ABI:
a batch solved with its x~ and y~ written straight into device tensors gives
the bits of the same batch written into the context's own blocks, through
every way of reading them (get_batch into the same tensors, into host
arrays, get, get_trace, the entry point that allocates nothing), with LPs
settled at submission, the shared start, the full-width start, and captured
graphs replayed over several batches; bad calls are refused."""
import gc
import weakref

import numpy as np
import pytest

from tests.gpu_common import cfg2_setup, make_ctx
from workloads import deltas, choose_vars, SET_LO, SET_HI

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2601_21990_amd.pdlpb as P
    return P


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


def _batches():
    inst, lp, eta, base, D = cfg2_setup()
    v = int(choose_vars(inst.n, 1, seed=9)[0])
    bad = deltas([SET_LO, SET_HI], [v, v], [float(inst.u[v]) + 1.0, float(inst.l[v]) - 1.0])
    return inst, eta, base, [np.concatenate([D[:20], bad, D[20:40]]), D[10:60], D]


def _solve(ctx, D, base):
    ctx.set_batch(D, x_warm=base.x, y_warm=base.y, w_warm=np.full(len(D), base.w))
    ctx.solve(tol=1e-4, max_iters=100000)


@pytest.mark.parametrize("shared", [1, -1])
def test_results_in_caller_tensors_equal_own_blocks(P, torch, shared):
    inst, eta, base, batches = _batches()
    dev = torch.device("cuda:0")
    cap = max(len(D) for D in batches)
    X = torch.full((cap, inst.n), float("nan"), dtype=torch.float64, device=dev)
    Y = torch.full((cap, inst.m), float("nan"), dtype=torch.float64, device=dev)
    with make_ctx(inst, eta, eval_every=32, shared_start=shared) as own, \
            make_ctx(inst, eta, eval_every=32, shared_start=shared) as ext:
        ext.set_result_buffers(X, Y, cap)
        for D in batches + batches[:1]:      # graphs replayed on later batches
            _solve(own, D, base)
            _solve(ext, D, base)
            ref = own.get_batch()
            B = len(D)
            # the solve wrote the tensors; get_batch into them copies nothing
            got_dev = ext.get_batch(X=X, Y=Y, mem=P.MEM_DEVICE)
            for key in ("status", "iters", "kkt", "obj"):
                assert np.array_equal(got_dev[key], ref[key], equal_nan=True), key
            assert np.array_equal(X[:B].cpu().numpy(), ref["X"])
            assert np.array_equal(Y[:B].cpu().numpy(), ref["Y"])
            # and every other read sees the same bits
            got = ext.get_batch()
            assert np.array_equal(got["X"], ref["X"]) and np.array_equal(got["Y"], ref["Y"])
            Xh, Yh = np.full((B, inst.n), np.nan), np.full((B, inst.m), np.nan)
            rc = P.lib.pdlpb_get_batch_noalloc(ext._h, Xh.ctypes.data, Yh.ctypes.data, None,
                                               None, None, None, P.MEM_HOST)
            assert rc == P.OK
            assert np.array_equal(Xh, ref["X"]) and np.array_equal(Yh, ref["Y"])
            for j in (0, 20, 21, B - 1):
                a, b = ext.get(j), own.get(j)
                assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["y"], b["y"])
                ta, tb = ext.get_trace(j), own.get_trace(j)
                assert np.array_equal(ta["x_iter"], tb["x_iter"])
                assert np.array_equal(ta["y_iter"], tb["y_iter"])
        settled = batches[0]
        _solve(ext, settled, base)
        st = ext.get_batch(want_x=False, want_y=False)["status"]
        assert st[20] == P.STATUS_INFEASIBLE_BOUNDS
        assert not X[20].abs().sum().item() and not Y[20].abs().sum().item()


def test_bad_calls_are_refused(P, torch):
    inst, eta, base, batches = _batches()
    dev = torch.device("cuda:0")
    X = torch.zeros((8, inst.n), dtype=torch.float64, device=dev)
    Y = torch.zeros((8, inst.m), dtype=torch.float64, device=dev)
    with make_ctx(inst, eta) as ctx:
        with pytest.raises(P.PdlpbError):
            ctx.set_result_buffers(X, None, 8)
        with pytest.raises(P.PdlpbError):
            ctx.set_result_buffers(X, Y, 0)
        # the binding checks what the library cannot see behind a pointer
        with pytest.raises(TypeError):
            ctx.set_result_buffers(X.float(), Y.float(), 8)
        with pytest.raises(TypeError):
            ctx.set_result_buffers(X.cpu().numpy(), Y.cpu().numpy(), 8)
        with pytest.raises(TypeError):
            ctx.set_result_buffers(X.t(), Y, 8)
        with pytest.raises(ValueError):
            ctx.set_result_buffers(X[:4], Y[:4], 8)
        # the context keeps the tensors alive while it writes into them
        Xt, Yt = X.clone(), Y.clone()
        wx = weakref.ref(Xt)
        ctx.set_result_buffers(Xt, Yt, 8)
        del Xt, Yt
        gc.collect()
        assert wx() is not None
        ctx.set_result_buffers()
        gc.collect()
        assert wx() is None
        ctx.set_result_buffers(X, Y, 8)
        with pytest.raises(P.PdlpbError) as e:
            ctx.set_batch(batches[1])               # 50 LPs > 8
        assert e.value.code == P.EINVAL
        ctx.set_batch(batches[1][:8])
        ctx.solve(tol=1e-4, max_iters=100000)
        ctx.set_result_buffers()                    # back to the context's own blocks
        with pytest.raises(P.PdlpbError) as e:
            ctx.get_batch()                         # the batch was dropped with the buffers
        assert e.value.code == P.ESTATE
        ctx.set_batch(batches[1])
        ctx.solve(tol=1e-4, max_iters=100000)
        assert np.all(np.isfinite(ctx.get_batch()["X"]))
    with make_ctx(inst, eta, precision=P.MIXED32) as ctx:
        with pytest.raises(P.PdlpbError):
            ctx.set_result_buffers(X, Y, 8)
    with make_ctx(inst, eta, scaling=1) as ctx:
        with pytest.raises(P.PdlpbError):
            ctx.set_result_buffers(X, Y, 8)


def _serve(P, ctx, D, tol, max_iters):
    ids = list(ctx.submit(D, P.WARM_NONE, tol, max_iters))
    want, got = set(ids), {}
    for _ in range(100000):
        if not want:
            break
        ctx.serve_launch()
        ctx.serve_wait()
        for i in ctx.poll():
            if i in want:
                got[i] = ctx.result(i)
                want.discard(i)
    assert not want
    return [got[i] for i in ids]


def test_batches_around_a_serving_session(P, torch):
    """One context with result tensors and the shared start solves a batch,
    serves a few requests, then solves the batch again.  The session writes
    its results into its own rows and leaves the tensors alone (its storage
    drops the batch's shared-start buffers and captured graphs); both batches
    give the bits of a fresh context, and the served LPs those of the same
    LPs solved as a batch."""
    inst, eta, base, batches = _batches()
    D = batches[1]
    B = len(D)
    served = D[:6]
    dev = torch.device("cuda:0")
    X = torch.full((B, inst.n), float("nan"), dtype=torch.float64, device=dev)
    Y = torch.full((B, inst.m), float("nan"), dtype=torch.float64, device=dev)
    with make_ctx(inst, eta, eval_every=32, shared_start=1) as fresh:
        _solve(fresh, D, base)
        ref = fresh.get_batch()
        fresh.set_batch(served)
        fresh.solve(tol=1e-5, max_iters=20000)
        ref_served = fresh.get_batch()
    with make_ctx(inst, eta, eval_every=32, shared_start=1) as ctx:
        ctx.set_result_buffers(X, Y, B)
        for rnd in range(2):
            _solve(ctx, D, base)
            got = ctx.get_batch(X=X, Y=Y, mem=P.MEM_DEVICE)
            for key in ("status", "iters", "kkt", "obj"):
                assert np.array_equal(got[key], ref[key]), (rnd, key)
            assert np.array_equal(X.cpu().numpy(), ref["X"]), rnd
            assert np.array_equal(Y.cpu().numpy(), ref["Y"]), rnd
            if rnd:
                break
            ctx.serve_begin(8)
            out = _serve(P, ctx, served, 1e-5, 20000)
            for j, g in enumerate(out):
                assert g["status"] == ref_served["status"][j] and g["iters"] == ref_served["iters"][j]
                assert np.array_equal(g["x"], ref_served["X"][j]), j
                assert np.array_equal(g["y"], ref_served["Y"][j]), j
            assert np.array_equal(X.cpu().numpy(), ref["X"])
            assert np.array_equal(Y.cpu().numpy(), ref["Y"])
