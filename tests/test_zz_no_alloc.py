"""pdlpb_get_batch_noalloc, the entry point for callers that cannot allocate,
against pdlpb_get_batch through the C ABI: the same results, bit for bit, on
two calls in a row (the second on a smaller batch), with no growth of the
context's device memory, for every context kind that stages host copies
(FP32 iterates, scaling, both) and for device destinations; a vector that
does not fit the fixed staging array is refused with an error."""
import ctypes as C

import numpy as np
import pytest

from workloads import make_cfg3, make_cfg2, obbt_deltas, choose_vars

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2601_21990_amd.pdlpb as P
    return P


def _ptr(a):
    return None if a is None else a.ctypes.data


def _get(P, fn, ctx, B, n, m, mem=0, X=None, Y=None):
    if mem == P.MEM_HOST:
        X = np.full((B, n), np.nan)
        Y = np.full((B, m), np.nan)
        px, py = _ptr(X), _ptr(Y)
    else:
        px, py = X.data_ptr(), Y.data_ptr()
    st = np.empty(B, dtype=np.int32)
    kkt = np.empty((B, 4))
    obj = np.empty(B)
    it = np.empty(B, dtype=np.int64)
    rc = fn(ctx._h, px, py, st.ctypes.data_as(C.POINTER(C.c_int32)),
            kkt.ctypes.data_as(C.POINTER(C.c_double)), obj.ctypes.data_as(C.POINTER(C.c_double)),
            it.ctypes.data_as(C.POINTER(C.c_int64)), mem)
    if mem != P.MEM_HOST:
        X, Y = X.cpu().numpy(), Y.cpu().numpy()
    return rc, dict(X=X, Y=Y, status=st, kkt=kkt, obj=obj, iters=it)


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("prec, scaling", [("fp32", 0), ("fp64", 1), ("fp32", 1)])
def test_noalloc_matches_get_batch(P, prec, scaling):
    """The 20000 x 50000 bound-tightening matrix: a batch of 96 LPs needs
    96 x 50000 staged doubles, more than the fixed array holds, so the copy
    runs in several chunks; then a batch of 8 on the same context."""
    inst = make_cfg3()
    n, m = inst.n, inst.m
    precision = P.MIXED32 if prec == "fp32" else P.FP64
    with P.Context.from_instance(inst, precision=precision, scaling=scaling) as ctx:
        for B in (96, 8):
            ctx.set_batch(obbt_deltas(choose_vars(n, B // 2, seed=B)))
            ctx.solve(tol=0.0, max_iters=65)
            before = ctx.device_bytes
            rc, got = _get(P, P.lib.pdlpb_get_batch_noalloc, ctx, B, n, m)
            assert rc == P.OK, P.lib.pdlpb_last_error(ctx._h)
            assert ctx.device_bytes == before
            rc, ref = _get(P, P.lib.pdlpb_get_batch, ctx, B, n, m)
            assert rc == P.OK
            assert np.all(np.isfinite(ref["X"])) and np.all(np.isfinite(ref["Y"]))
            _same(got, ref)


def test_noalloc_device_destination(P):
    import torch
    inst = make_cfg2(m=200, n=500)
    with P.Context.from_instance(inst, precision=P.MIXED32, scaling=1) as ctx:
        for B in (16, 4):
            ctx.set_batch(obbt_deltas(choose_vars(inst.n, B // 2, seed=B)))
            ctx.solve(tol=1e-4, max_iters=5000)
            X = torch.full((B, inst.n), float("nan"), dtype=torch.float64, device="cuda:0")
            Y = torch.full((B, inst.m), float("nan"), dtype=torch.float64, device="cuda:0")
            before = ctx.device_bytes
            rc, got = _get(P, P.lib.pdlpb_get_batch_noalloc, ctx, B, inst.n, inst.m,
                           mem=P.MEM_DEVICE, X=X, Y=Y)
            assert rc == P.OK and ctx.device_bytes == before
            rc, ref = _get(P, P.lib.pdlpb_get_batch, ctx, B, inst.n, inst.m)
            assert rc == P.OK
            _same(got, ref)


def test_noalloc_refuses_a_vector_beyond_the_array(P):
    """n one above what the array holds, no rows: a staged copy of x~ is
    refused with an error naming the limit; y (empty) and the scalars still
    come back, and the context keeps working."""
    n = P.NOALLOC_SCRATCH_BYTES // 8 + 1
    ctx = P.Context(0, n, np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0),
                    np.linspace(-1.0, 1.0, n), np.zeros(0), np.zeros(0, dtype=np.uint8),
                    np.zeros(n), np.ones(n), precision=P.MIXED32, step_size=0.5)
    with ctx:
        ctx.set_batch(P.deltas_array([P.BASE], [0], [0.0]))
        ctx.solve(tol=0.0, max_iters=3)
        rc, _ = _get(P, P.lib.pdlpb_get_batch_noalloc, ctx, 1, n, 0)
        assert rc == P.EINVAL
        assert b"staging array" in P.lib.pdlpb_last_error(ctx._h)
        st = np.empty(1, dtype=np.int32)
        rc = P.lib.pdlpb_get_batch_noalloc(ctx._h, None, None,
                                           st.ctypes.data_as(C.POINTER(C.c_int32)), None, None,
                                           None, P.MEM_HOST)
        assert rc == P.OK and st[0] == P.STATUS_ITERATION_LIMIT
