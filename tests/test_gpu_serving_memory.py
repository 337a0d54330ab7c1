"""Serving storage that follows the admitted work, through the C ABI: the
footprint a context reports before a submission is the device memory it holds
after the launch that admits it; growing the storage while LPs run keeps
their iterates (their results equal a solve alone, bit for bit); trimming an
idle session gives the memory back; and the request loop under a
device-memory budget admits requests whole, in arrival order, never above the
budget, with the results of an unbounded loop."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_common import make_ctx
from workloads import make_cfg2, obbt_deltas, choose_vars, fsb_deltas, choose_fractional

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


def _drain(ctx, ids, want_xy=True):
    want, got = set(ids), {}
    for _ in range(100000):
        if not want:
            break
        ctx.serve_launch()
        ctx.serve_wait()
        for i in ctx.poll():
            if i in want:
                got[i] = ctx.result(i, want_x=want_xy, want_y=want_xy)
                want.discard(i)
    assert not want
    return got


def _alone(P, inst, eta, D, tol, K):
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(D)
        ctx.solve(tol=tol, max_iters=K)
        return ctx.get_batch()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_footprint_is_what_the_launch_allocates(P, base, prec):
    inst, lp, eta, root = base
    precision = P.MIXED32 if prec == "fp32" else P.FP64
    with make_ctx(inst, eta, precision=precision, max_batch=256) as ctx:
        ctx.serve_begin(512)
        idle = ctx.device_bytes
        assert ctx.serve_footprint(0) == idle
        for count in (3, 40, 150):
            want = ctx.serve_footprint(count)
            assert want >= ctx.device_bytes
            D = obbt_deltas(choose_vars(inst.n, (count + 1) // 2, seed=count))[:count]
            ids = ctx.submit(D, P.WARM_NONE, 1e-4, 20000)
            assert ctx.serve_footprint(0) == want       # submitted, not yet admitted
            ctx.serve_launch()
            ctx.serve_wait()
            assert ctx.device_bytes == want
            got = _drain(ctx, list(ids), want_xy=False)
            for i in ids:
                ctx.release(i)
            assert all(r["status"] == P.STATUS_OPTIMAL for r in got.values())
        grown = ctx.device_bytes
        ctx.serve_trim()                                # idle: back to one column and one row
        assert ctx.device_bytes == idle < grown
        assert ctx.serve_footprint(0) == idle


def test_growth_keeps_running_lps(P, base):
    """Three LPs run one block in storage for four columns; then 60 more
    arrive and the next launch moves the running ones into storage for 64
    columns; every LP's result equals its solve alone, bit for bit."""
    inst, lp, eta, root = base
    first = obbt_deltas(choose_vars(inst.n, 2, seed=11))[:3]
    more = fsb_deltas(root.x, choose_fractional(root.x, 30, seed=12))
    tol, K = 1e-5, 20000
    with make_ctx(inst, eta) as ctx:
        ctx.serve_begin(128)
        ids1 = list(ctx.submit(first, P.WARM_NONE, tol, K))
        ctx.serve_launch()
        ctx.serve_wait()
        small = ctx.device_bytes
        ids2 = list(ctx.submit(more, P.WARM_NONE, tol, K))
        got = _drain(ctx, ids1 + ids2)
        assert ctx.device_bytes > small
    ref1 = _alone(P, inst, eta, first, tol, K)
    ref2 = _alone(P, inst, eta, more, tol, K)
    for ids, ref in ((ids1, ref1), (ids2, ref2)):
        for j, i in enumerate(ids):
            assert got[i]["status"] == ref["status"][j]
            assert got[i]["iters"] == ref["iters"][j]
            np.testing.assert_array_equal(got[i]["x"], ref["X"][j])
            np.testing.assert_array_equal(got[i]["y"], ref["Y"][j])


def test_budgeted_loop_matches_unbounded(P, base):
    """Two bases, requests of 8..48 LPs, a budget a little above the bases'
    idle footprint plus the largest request: requests wait for memory, none is
    admitted above the budget, and every LP's result equals the unbounded
    loop's."""
    from paper_2601_21990_amd.serve import Server, Request
    inst, lp, eta, root = base
    rng = np.random.default_rng(7)
    reqs = []
    for k in range(10):
        size = int(rng.integers(4, 25)) * 2
        if k % 2:
            d = fsb_deltas(root.x, choose_fractional(root.x, size // 2, seed=100 + k))
        else:
            d = obbt_deltas(choose_vars(inst.n, size // 2, seed=100 + k))
        reqs.append((k % 2, d))

    def run(budget_of):
        ctxs = []
        for _ in range(2):
            c = make_ctx(inst, eta, max_batch=128)
            c.set_base_warm(root.x, root.y, root.w)
            c.serve_begin(256)
            ctxs.append(c)
        budget = budget_of(ctxs)
        srv = Server(ctxs, warm=True, budget_bytes=budget)
        tagged = []
        for b, d in reqs:
            r = Request(base=b, deltas=d, arrival=0.0, tol=1e-4, max_iters=20000)
            srv.submit(r)
            tagged.append(r)
        srv.drain()
        out = [tuple([d[i] for i in sorted(d)] for d in (r.statuses, r.iters, r.objs))
               for r in tagged]
        stats = (srv.peak_bytes, srv.blocked_on_budget, budget)
        for c in ctxs:
            c.close()
        return out, stats

    free, _ = run(lambda ctxs: None)

    def tight(ctxs):
        idle = sum(c.serve_footprint(0) for c in ctxs)
        biggest = max(ctxs[b].serve_footprint(len(d)) - ctxs[b].serve_footprint(0)
                      for b, d in reqs)
        return idle + biggest + biggest // 2

    capped, (peak, blocked, budget) = run(tight)
    assert peak <= budget and blocked > 0
    assert free == capped
