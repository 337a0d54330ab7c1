"""Served LPs against the FP64 oracle, through the C ABI.

Continuous batching admits LPs into a running batch: an admitted LP makes its
first iteration (an evaluation) at admission and then follows the per-LP
schedule of Section 4 from its own first iteration.  Under the per-LP restart
scope its trajectory is therefore the oracle's one-LP-at-a-time trajectory
started the same way:
  * bound changes (SET_LO / SET_HI, strong branching, Section 5.1) with the
    base warm start begin at the base x projected onto the LP's box, the base
    y and the base primal weight;
  * objective changes (OBJ_UNIT, bound tightening, Section 5.2) with the base
    warm start begin at the base x, y = 0 and the default weight
    ||c_j|| / ||b||;
  * cold LPs begin at the projection of 0 with y = 0 and the default weight.
Tolerances are those of the batch parity tests: after a fixed iteration count
the returned point agrees to 1e-9 relative per LP and per coordinate, with
identical statuses and counts; converged runs stop at the same iteration with
points within 1e-8 and the KKT measures within 1e-7.
"""
import numpy as np
import pytest

import oracle as O
from tests.gpu_common import (ITER_RTOL, KKT_ATOL, OBJ_RTOL, make_ctx, lp_for, rel_err,
                              assert_iterates_match)
from workloads import (make_cfg2, make_cfg4, obbt_deltas, choose_vars, fsb_deltas,
                       choose_fractional, OBJ_UNIT, seed_for)

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
    assert root.status == O.OPTIMAL
    return inst, lp, eta, root


def oracle_served(lp, eta, root, d, warm, tol, max_iters, C):
    """The oracle run an LP served with `warm` (True: the base warm start) must reproduce."""
    lpj = lp_for(lp, d)
    opt = O.Options(tol=tol, max_iters=max_iters, step_size=eta, eval_every=C)
    if not warm:
        return O.solve(lpj, opt)
    if int(d["kind"]) == OBJ_UNIT:
        return O.solve(lpj, opt, x_init=root.x, y_init=np.zeros(lp.m), w_init=None)
    return O.solve(lpj, opt, x_init=root.x, y_init=root.y, w_init=root.w)


def serve_all(ctx, ids):
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
    return got


def compare(g, o, rtol, what):
    assert g["status"] == o.status, (what, g["status"], o.status)
    assert g["iters"] == o.iters, (what, g["iters"], o.iters)
    assert_iterates_match((("x~", g["x"], o.x), ("y~", g["y"], o.y)), rtol, what)
    ref = (o.kkt.gap, o.kkt.primal, o.kkt.dual, o.kkt.rel)
    for name, a, b in zip(("gap", "primal", "dual", "max"), g["kkt"], ref):
        assert abs(a - b) <= KKT_ATOL, (what, name, a, b)
    assert abs(g["obj"] - o.kkt.obj) <= OBJ_RTOL * (1 + abs(o.kkt.obj)), (what, g["obj"], o.kkt.obj)


def _requests(inst, root):
    cold = obbt_deltas(choose_vars(inst.n, 3, seed=11))                         # 6 LPs, cold
    bounds = fsb_deltas(root.x, choose_fractional(root.x, 4, seed=12))         # 8 LPs, warm
    objs = obbt_deltas(choose_vars(inst.n, 3, seed=13))                         # 6 LPs, warm
    return cold, bounds, objs


def _serve_mid_stream(P, inst, eta, root, tol, max_iters, C):
    """A cold request runs for two blocks before a bound-change and an
    objective-change request (both with the base warm start) arrive; a
    second cold request arrives one block later."""
    cold, bounds, objs = _requests(inst, root)
    with make_ctx(inst, eta, eval_every=C) as ctx:
        ctx.set_base_warm(root.x, root.y, root.w)
        ctx.serve_begin(128)
        a = list(ctx.submit(cold, P.WARM_NONE, tol, max_iters))
        for _ in range(2):
            ctx.serve_launch()
            ctx.serve_wait()
        b = list(ctx.submit(bounds, P.WARM_BASE, tol, max_iters))
        c = list(ctx.submit(objs, P.WARM_BASE, tol, max_iters))
        ctx.serve_launch()
        ctx.serve_wait()
        d = list(ctx.submit(cold[:2], P.WARM_NONE, tol, max_iters))
        got = serve_all(ctx, a + b + c + d)
    return [(got[i], dl, False) for i, dl in zip(a, cold)] + \
        [(got[i], dl, True) for i, dl in zip(b, bounds)] + \
        [(got[i], dl, True) for i, dl in zip(c, objs)] + \
        [(got[i], dl, False) for i, dl in zip(d, cold[:2])]


@pytest.mark.parametrize("C,K", [(16, 1), (16, 40), (64, 200), (16, 700)])
def test_served_mid_stream_fixed_iterations_match_oracle(P, base, C, K):
    inst, lp, eta, root = base
    served = _serve_mid_stream(P, inst, eta, root, 0.0, K, C)
    for j, (g, d, warm) in enumerate(served):
        o = oracle_served(lp, eta, root, d, warm, 0.0, K, C)
        assert g["status"] == P.STATUS_ITERATION_LIMIT
        compare(g, o, ITER_RTOL, f"C={C} K={K} LP {j} warm={warm} kind={int(d['kind'])}")


@pytest.mark.parametrize("C", [16, 64])
def test_served_mid_stream_converged_match_oracle(P, base, C):
    inst, lp, eta, root = base
    served = _serve_mid_stream(P, inst, eta, root, 1e-6, 20000, C)
    for j, (g, d, warm) in enumerate(served):
        o = oracle_served(lp, eta, root, d, warm, 1e-6, 20000, C)
        compare(g, o, 1e-8, f"C={C} LP {j} warm={warm} kind={int(d['kind'])}")
        if o.status == O.OPTIMAL:
            assert g["kkt"][3] <= 1e-6


def test_result_and_release_before_the_lp_stops(P, base):
    """A queued or running LP reports RUNNING without touching its result row,
    and its row cannot be released until it has stopped."""
    inst, lp, eta, root = base
    cold, _, _ = _requests(inst, root)
    with make_ctx(inst, eta) as ctx:
        ctx.serve_begin(16)
        ids = list(ctx.submit(cold, P.WARM_NONE, 1e-6, 20000))
        r = ctx.result(ids[0])                               # queued
        assert r["status"] == P.STATUS_RUNNING and r["iters"] == 0 and np.isnan(r["obj"])
        with pytest.raises(P.PdlpbError) as e:
            ctx.release(ids[0])
        assert e.value.code == P.ESTATE
        ctx.serve_launch()
        ctx.serve_wait()
        done = set(ctx.poll())
        running = [i for i in ids if i not in done]
        assert running                                       # 1e-6 takes more than one block
        assert ctx.result(running[0])["status"] == P.STATUS_RUNNING
        with pytest.raises(P.PdlpbError) as e:
            ctx.release(running[0])
        assert e.value.code == P.ESTATE
        rest = serve_all(ctx, running)
        for i in ids:
            if i in rest:
                assert rest[i]["status"] == P.STATUS_OPTIMAL
            ctx.release(i)                                   # stopped: allowed
        with pytest.raises(P.PdlpbError):
            ctx.release(ids[0])                              # already released


# ---------------------------------------------------------------------------
# uneven batches over several bases through the serving loop
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def mixed_bases():
    """The three smallest bases of the mixed family (m = 1000, 1931, 3728;
    n = 2.5 m; 4..12 N(0,1) nonzeros per column), each with its oracle root
    solution as the resident warm start."""
    out = []
    for i in range(3):
        inst = make_cfg4(i)
        lp = O.from_instance(inst)
        eta = O.step_size(lp.A)
        root = O.solve(lp, O.Options(tol=1e-6, step_size=eta))
        assert root.status == O.OPTIMAL
        out.append((inst, lp, eta, root))
    return out


def _mixed_requests(mixed_bases):
    """Per base: one bound-change request and one objective-change request of
    uneven sizes (6, 10 / 4, 8 / 2, 12 LPs)."""
    sizes = [(6, 10), (4, 8), (2, 12)]
    reqs = []
    for b, ((inst, lp, eta, root), (nb, no)) in enumerate(zip(mixed_bases, sizes)):
        vb = choose_fractional(root.x, nb // 2, seed_for(4, 500 + b))
        vo = choose_vars(inst.n, no // 2, seed_for(4, 600 + b))
        reqs.append((b, fsb_deltas(root.x, vb)))
        reqs.append((b, obbt_deltas(vo)))
    return reqs


def _serve_mixed(P, mixed_bases, reqs, tol, max_iters, C, precision):
    from paper_2601_21990_amd.serve import Server, Request
    ctxs = []
    try:
        for inst, lp, eta, root in mixed_bases:
            c = make_ctx(inst, eta, eval_every=C, precision=precision, max_batch=16)
            c.set_base_warm(root.x, root.y, root.w)
            c.serve_begin(64)
            ctxs.append(c)
        srv = Server(ctxs, warm=True, keep_results=True)
        tagged = []
        for b, d in reqs:
            r = Request(base=b, deltas=d, arrival=0.0, tol=tol, max_iters=max_iters)
            srv.submit(r)
            tagged.append(r)
        srv.drain()
        return [(r.base, d, srv.results[(r.base, i)]) for r in tagged
                for i, d in zip(r.ids, r.deltas)]
    finally:
        for c in ctxs:
            c.close()


def test_mixed_bases_through_server_converged_match_oracle(P, mixed_bases):
    """42 LPs over three bases, 16 columns per base (so LPs queue and enter as
    others finish), FP64, evaluation every 16 iterations: each LP stops at the
    oracle's iteration with the oracle's point."""
    reqs = _mixed_requests(mixed_bases)
    served = _serve_mixed(P, mixed_bases, reqs, 1e-4, 20000, 16, P.FP64)
    assert len(served) == 42
    for j, (b, d, g) in enumerate(served):
        inst, lp, eta, root = mixed_bases[b]
        o = oracle_served(lp, eta, root, d, True, 1e-4, 20000, 16)
        compare(g, o, 1e-8, f"base {b} LP {j} kind={int(d['kind'])}")


def test_mixed_bases_through_server_mixed32_within_rounding_growth(P, mixed_bases):
    """The same stream with FP32 iterates and FP64 sums after K = 16
    iterations: within 4 (K + 1) u of the FP64 oracle (the bound of the
    batch's mixed-precision parity test), same statuses and counts."""
    K = 16
    reqs = _mixed_requests(mixed_bases)
    served = _serve_mixed(P, mixed_bases, reqs, 0.0, K, 16, P.MIXED32)
    bound = 4 * (K + 1) * 2.0 ** -24
    for j, (b, d, g) in enumerate(served):
        inst, lp, eta, root = mixed_bases[b]
        o = oracle_served(lp, eta, root, d, True, 0.0, K, 16)
        assert (g["status"], g["iters"]) == (o.status, o.iters), (b, j)
        errs = (rel_err(g["x"], o.x), rel_err(g["y"], o.y))
        assert max(errs) <= bound, (b, j, errs, bound)
