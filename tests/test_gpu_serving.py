"""Continuous batching through the C ABI: requests admitted into a running
batch give the same bits as solved alone (per-LP restart scope), finished LPs
free columns for queued ones, and result rows are admission-controlled."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_common import make_ctx
from workloads import make_cfg2, obbt_deltas, choose_vars, fsb_deltas, choose_fractional, deltas

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2601_21990_amd.pdlpb as P
    return P


@pytest.fixture(scope="module")
def base():
    inst = make_cfg2(m=200, n=500)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    root = O.solve(lp, O.Options(tol=1e-7, step_size=eta))
    return inst, lp, eta, root


def _serve_until_done(P, ctx, ids):
    want = set(ids)
    got = {}
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
    return got


def _requests(inst, root):
    r1 = obbt_deltas(choose_vars(inst.n, 6, seed=1))
    r2 = fsb_deltas(root.x, choose_fractional(root.x, 4, seed=2))
    r3 = obbt_deltas(choose_vars(inst.n, 5, seed=3))
    return r1, r2, r3


def test_serve_matches_batch_solve(P, base):
    inst, lp, eta, root = base
    r1, _, _ = _requests(inst, root)
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(r1)
        ctx.solve(tol=1e-5, max_iters=20000)
        ref = ctx.get_batch()
    with make_ctx(inst, eta) as ctx:
        ctx.serve_begin(64)
        ids = ctx.submit(r1, P.WARM_NONE, 1e-5, 20000)
        got = _serve_until_done(P, ctx, list(ids))
    for j, i in enumerate(ids):
        assert got[i]["status"] == ref["status"][j]
        assert got[i]["iters"] == ref["iters"][j]
        np.testing.assert_array_equal(got[i]["x"], ref["X"][j])
        np.testing.assert_array_equal(got[i]["y"], ref["Y"][j])


def test_request_same_alone_and_in_the_mix(P, base):
    """A request admitted while others run (and while later ones arrive) gets
    bitwise the same results as when it is served alone."""
    inst, lp, eta, root = base
    r1, r2, r3 = _requests(inst, root)
    with make_ctx(inst, eta) as ctx:
        ctx.set_base_warm(root.x, root.y, root.w)
        ctx.serve_begin(128)
        alone_ids = ctx.submit(r2, P.WARM_BASE, 1e-5, 20000)
        alone = _serve_until_done(P, ctx, list(alone_ids))
    with make_ctx(inst, eta) as ctx:
        ctx.set_base_warm(root.x, root.y, root.w)
        ctx.serve_begin(128)
        a = ctx.submit(r1, P.WARM_NONE, 1e-5, 20000)
        for _ in range(3):                      # r1 is running when r2 arrives
            ctx.serve_launch()
            ctx.serve_wait()
        mix_ids = ctx.submit(r2, P.WARM_BASE, 1e-5, 20000)
        ctx.serve_launch()
        ctx.serve_wait()
        c = ctx.submit(r3, P.WARM_NONE, 1e-5, 20000)
        got = _serve_until_done(P, ctx, list(a) + list(mix_ids) + list(c))
    for i_alone, i_mix in zip(alone_ids, mix_ids):
        assert got[i_mix]["status"] == alone[i_alone]["status"]
        assert got[i_mix]["iters"] == alone[i_alone]["iters"]
        np.testing.assert_array_equal(got[i_mix]["x"], alone[i_alone]["x"])
        np.testing.assert_array_equal(got[i_mix]["y"], alone[i_alone]["y"])


def test_admission_with_few_columns(P, base):
    """Eight columns for 19 LPs: queued LPs enter as others finish, and every
    result equals the one-batch solve."""
    inst, lp, eta, root = base
    r1, r2, r3 = _requests(inst, root)
    allreq = np.concatenate([r1, r2, r3])
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(allreq)
        ctx.solve(tol=1e-5, max_iters=20000)
        ref = ctx.get_batch()
    with make_ctx(inst, eta, max_batch=8) as ctx:
        ctx.serve_begin(64)
        ids = list(ctx.submit(allreq, P.WARM_NONE, 1e-5, 20000))
        got = _serve_until_done(P, ctx, ids)
    for j, i in enumerate(ids):
        assert got[i]["iters"] == ref["iters"][j]
        np.testing.assert_array_equal(got[i]["x"], ref["X"][j])


def test_result_rows_are_admission_controlled(P, base):
    inst, lp, eta, root = base
    r1, _, _ = _requests(inst, root)
    with make_ctx(inst, eta) as ctx:
        ctx.serve_begin(12)
        ids = ctx.submit(r1, P.WARM_NONE, 1e-4, 20000)           # 12 rows used
        with pytest.raises(P.PdlpbError) as e:
            ctx.submit(r1[:1], P.WARM_NONE, 1e-4, 20000)
        assert e.value.code == P.ENOMEM
        _serve_until_done(P, ctx, list(ids))
        ctx.release(ids[0])
        more = ctx.submit(r1[:1], P.WARM_NONE, 1e-4, 20000)
        assert len(more) == 1
        with pytest.raises(P.PdlpbError):
            ctx.result(ids[0])                                   # released
        # a malformed change settles at submission without iterating
        ctx.release(ids[1])
        bad = ctx.submit(deltas([1], [3], [np.nan]), P.WARM_NONE, 1e-4, 20000)
        assert ctx.result(bad[0])["status"] == P.STATUS_INVALID_INPUT
        assert bad[0] in ctx.poll()


def test_server_loop_overlaps_bases(P, base):
    """The Python loop over two bases completes every request and reports
    statuses for all LPs."""
    from paper_2601_21990_amd.serve import Server, Request
    inst, lp, eta, root = base
    r1, r2, r3 = _requests(inst, root)
    ctxs = []
    try:
        for _ in range(2):
            c = make_ctx(inst, eta)
            c.set_base_warm(root.x, root.y, root.w)
            c.serve_begin(64)
            ctxs.append(c)
        srv = Server(ctxs, warm=True)
        for k, r in enumerate([r1, r2, r3, r2]):
            srv.submit(Request(base=k % 2, deltas=r, arrival=0.0, tol=1e-4))
        srv.drain()
        assert len(srv.completed) == 4
        assert srv.lps_done == len(r1) + 2 * len(r2) + len(r3)
        for req in srv.completed:
            assert set(req.statuses.values()) <= {P.STATUS_OPTIMAL, P.STATUS_PRIMAL_INFEASIBLE}
    finally:
        for c in ctxs:
            c.close()


def test_objective_change_warm_base_starts_from_base_primal(P, base):
    """An objective change admitted with the base warm start begins at the
    base primal point with y = 0 and the default weight, i.e. exactly the
    batch solve warm-started per LP that way."""
    inst, lp, eta, root = base
    D = obbt_deltas(choose_vars(inst.n, 4, seed=7))
    B = len(D)
    with make_ctx(inst, eta) as ctx:
        # no weights given: each LP takes the default ||c_j|| / ||b||
        ctx.set_batch(D, x_warm=np.tile(root.x, B), y_warm=np.zeros(B * inst.m),
                      warm_mode=P.WARM_PER_LP)
        ctx.solve(tol=1e-5, max_iters=20000)
        ref = ctx.get_batch()
    with make_ctx(inst, eta) as ctx:
        ctx.set_base_warm(root.x, root.y, root.w)
        ctx.serve_begin(16)
        ids = ctx.submit(D, P.WARM_BASE, 1e-5, 20000)
        got = _serve_until_done(P, ctx, list(ids))
    for j, i in enumerate(ids):
        assert got[i]["status"] == ref["status"][j] == P.STATUS_OPTIMAL
        assert got[i]["iters"] == ref["iters"][j]
        np.testing.assert_array_equal(got[i]["x"], ref["X"][j])
        np.testing.assert_array_equal(got[i]["y"], ref["Y"][j])


def test_batch_after_serving_ends_the_session(P, base):
    inst, lp, eta, root = base
    r1, _, _ = _requests(inst, root)
    with make_ctx(inst, eta) as ctx:
        ctx.serve_begin(16)
        ctx.submit(r1[:2], P.WARM_NONE, 1e-4, 20000)
        ctx.set_batch(r1[:2])
        ctx.solve(tol=1e-4, max_iters=20000)
        assert np.all(ctx.get_batch(want_x=False, want_y=False)["status"] == P.STATUS_OPTIMAL)
        with pytest.raises(P.PdlpbError) as e:
            ctx.serve_launch()
        assert e.value.code == P.ESTATE
        ctx.serve_begin(16)                        # a new session works again
        ids = ctx.submit(r1[:2], P.WARM_NONE, 1e-4, 20000)
        got = _serve_until_done(P, ctx, list(ids))
        assert all(g["status"] == P.STATUS_OPTIMAL for g in got.values())


def test_serving_right_after_a_long_solve(P, base):
    """A solve of many blocks (its replays run ahead of the host) returns with
    nothing left running: a serving session opened at once on the same context
    gives the same bits as one on a fresh context."""
    inst, lp, eta, root = base
    r1, _, _ = _requests(inst, root)
    with make_ctx(inst, eta, eval_every=4) as ctx:
        ctx.serve_begin(16)
        ids = ctx.submit(r1, P.WARM_NONE, 1e-6, 20000)
        ref = _serve_until_done(P, ctx, list(ids))
    with make_ctx(inst, eta, eval_every=4) as ctx:
        ctx.set_batch(r1)
        ctx.solve(tol=1e-9, max_iters=2000)     # hundreds of blocks of 4 iterations
        st = ctx.get_batch(want_x=False, want_y=False)
        assert np.all(st["iters"] > 4 * 8)
        ctx.serve_begin(16)
        ids2 = ctx.submit(r1, P.WARM_NONE, 1e-6, 20000)
        got = _serve_until_done(P, ctx, list(ids2))
    for i, i2 in zip(ids, ids2):
        assert got[i2]["iters"] == ref[i]["iters"]
        np.testing.assert_array_equal(got[i2]["x"], ref[i]["x"])
        np.testing.assert_array_equal(got[i2]["y"], ref[i]["y"])


def test_serve_matches_batch_solve_mixed32(P, base):
    """The same property with FP32 iterates and FP64 sums: an LP served through
    admission carries the bits it has when its request is solved as a batch."""
    inst, lp, eta, root = base
    r1, _, r3 = _requests(inst, root)
    with make_ctx(inst, eta, precision=P.MIXED32) as ctx:
        ctx.set_batch(r3)
        ctx.solve(tol=1e-4, max_iters=20000)
        ref = ctx.get_batch()
    with make_ctx(inst, eta, precision=P.MIXED32) as ctx:
        ctx.serve_begin(32)
        ctx.submit(r1, P.WARM_NONE, 1e-4, 20000)        # running when r3 arrives
        ctx.serve_launch()
        ctx.serve_wait()
        ids = ctx.submit(r3, P.WARM_NONE, 1e-4, 20000)
        got = _serve_until_done(P, ctx, list(ids))
    for j, i in enumerate(ids):
        assert got[i]["status"] == ref["status"][j]
        assert got[i]["iters"] == ref["iters"][j]
        np.testing.assert_array_equal(got[i]["x"], ref["X"][j])
        np.testing.assert_array_equal(got[i]["y"], ref["Y"][j])


def test_lps_stopping_at_admission_leave_with_the_first_block(P):
    """Strong branching from the root of the 2000 x 5000 family at a tolerance
    that about half of the branches meet at z~ = T(z^0): after the first
    block every LP that stopped at its first evaluation is reported, the
    running count is the LPs still iterating, and every result equals the
    same LPs solved as a batch, bit for bit (the admission's compaction moves
    running LPs into the freed columns before the block's iterations)."""
    from tests.gpu_common import cfg2_setup
    inst, lp, eta, root, D = cfg2_setup()
    tol = 1e-3
    with make_ctx(inst, eta, eval_every=16) as ctx:
        ctx.set_batch(D, x_warm=root.x, y_warm=root.y, w_warm=np.full(len(D), root.w))
        ctx.solve(tol=tol, max_iters=20000)
        ref = ctx.get_batch()
    first = int(np.sum(ref["iters"] == 1))
    assert len(D) // 4 < first < 3 * len(D) // 4
    with make_ctx(inst, eta, eval_every=16) as ctx:
        ctx.set_base_warm(root.x, root.y, root.w)
        ctx.serve_begin(128)
        ids = list(ctx.submit(D, P.WARM_BASE, tol, 20000))
        ctx.serve_launch()
        running, _ = ctx.serve_wait()
        done = set(ctx.poll())
        # the LPs that stopped at t = 0 and those that stopped within the block
        stopped_by_16 = {ids[j] for j in range(len(D)) if ref["iters"][j] <= 17}
        assert {ids[j] for j in range(len(D)) if ref["iters"][j] == 1} <= done
        assert done == stopped_by_16
        assert running == len(D) - len(done)
        got = _serve_until_done(P, ctx, [i for i in ids if i not in done])
        for i in done:
            got[i] = ctx.result(i)
    for j, i in enumerate(ids):
        assert got[i]["status"] == ref["status"][j]
        assert got[i]["iters"] == ref["iters"][j]
        np.testing.assert_array_equal(got[i]["x"], ref["X"][j])
        np.testing.assert_array_equal(got[i]["y"], ref["Y"][j])
