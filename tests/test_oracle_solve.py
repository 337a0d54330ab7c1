"""End-to-end pins of the reference solver: the converged objective against
exact optima (vertex enumeration, box closed form, hand-solved LPs, HiGHS),
KKT and complementary-slackness invariants at every returned point, the
strong-branching / bound-tightening semantics of Section 5, statuses, the
batched restart scope, and the Halpern rate bound with and without restarts."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from tests.lp_exact import vertex_enum, box_closed_form, highs
from workloads import (make_tiny, make_cfg1, make_cfg2, choose_fractional, fsb_deltas,
                       obbt_deltas, choose_vars)

INF = np.inf


def _check_invariants(lp, res, tol):
    """At a returned point: x~ in the box and y~ in the barrier cone exactly;
    the two nonnegative parts of the duality gap are small, which bounds the
    complementary-slackness violation."""
    x, y = res.x, res.y
    assert np.all(x >= lp.xl) and np.all(x <= lp.xu)
    np.testing.assert_array_equal(O.proj_barrier_cone(y, lp.l, lp.u), y)
    r = O.reduced_cost(lp, y)
    ax = lp.A @ x
    # gap = (phi(y) - y'Ax) + (phi(r) - r'x) + (c + A'y + r)'x, first two parts >= 0 when Ax, x feasible
    part_y = O.support(y, lp.l, lp.u) - float(y @ O.proj_box(ax, lp.l, lp.u))
    part_r = O.support(r, lp.xl, lp.xu) - float(r @ x)
    assert part_y >= -1e-9 * (1 + abs(part_y)) and part_r >= -1e-9 * (1 + abs(part_r))
    scale = 1 + abs(res.kkt.obj) + abs(res.kkt.dual_obj)
    assert part_r <= 10 * tol * scale
    # complementary slackness per coordinate: r_j > 0 only where x_j sits near its upper bound, etc.
    big = np.abs(r) > 1e-3
    dist = np.where(r > 0, lp.xu - x, x - lp.xl)
    assert np.all(np.abs(r[big]) * dist[big] <= 10 * tol * scale + 1e-9)


@pytest.mark.parametrize("seed", range(8))
def test_converges_to_vertex_enumeration_optimum(seed):
    inst = make_tiny(seed, m=3, n=5, senses="ELG", box=(0.0, 4.0))
    lp = O.from_instance(inst)
    best, _ = vertex_enum(lp.A.toarray(), lp.l, lp.u, lp.xl, lp.xu, lp.c)
    res = O.solve(lp, O.Options(tol=1e-9, max_iters=400000))
    assert res.status == O.OPTIMAL
    assert abs(res.obj - best) <= 1e-7 * (1 + abs(best))
    _check_invariants(lp, res, 1e-9)


def test_textbook_lps_solved():
    with open(os.path.join(os.path.dirname(__file__), "golden", "textbook_lps.json")) as f:
        data = json.load(f)["lps"]
    for d in data:
        A = np.array(d["A"])
        csr = sp.csr_matrix(A)
        lp = O.from_arrays(A.shape[0], A.shape[1], csr.indptr, csr.indices, csr.data, d["c"],
                           d["b"], np.frombuffer(d["sense"].encode(), dtype=np.uint8),
                           d["l"], d["u"])
        res = O.solve(lp, O.Options(tol=1e-10, max_iters=200000))
        assert res.status == O.OPTIMAL, d["name"]
        assert abs(res.obj - d["obj"]) <= 1e-8 * (1 + abs(d["obj"])), d["name"]
        np.testing.assert_allclose(res.x, d["x"], atol=1e-6)


@pytest.mark.parametrize("seed", range(3))
def test_box_only_closed_form(seed):
    """All rows free (l = -inf, u = +inf): y = 0 and each x_j sits at the bound
    selected by the sign of c_j."""
    rng = np.random.default_rng(seed)
    m, n = 6, 12
    A = sp.random(m, n, density=0.5, random_state=seed, data_rvs=rng.standard_normal).tocsr()
    xl = rng.uniform(-3, 0, n)
    xu = xl + rng.uniform(0.1, 4, n)
    c = rng.standard_normal(n)
    lp = O.LP(A=A, c=c, l=np.full(m, -INF), u=np.full(m, INF), xl=xl, xu=xu, b=np.ones(m))
    res = O.solve(lp, O.Options(tol=1e-12, max_iters=100000))
    obj, x = box_closed_form(c, xl, xu)
    assert res.status == O.OPTIMAL
    assert math.isclose(res.obj, obj, rel_tol=1e-10, abs_tol=1e-10)
    np.testing.assert_allclose(res.x, x, atol=1e-9)
    np.testing.assert_array_equal(res.y, 0.0)


def test_zero_matrix_closed_form():
    n = 8
    rng = np.random.default_rng(4)
    c = rng.standard_normal(n)
    lp = O.LP(A=sp.csr_matrix((3, n)), c=c, l=np.zeros(3), u=np.zeros(3),
              xl=np.zeros(n), xu=np.full(n, 2.0), b=np.zeros(3))
    res = O.solve(lp, O.Options(tol=1e-12, max_iters=10000))
    assert res.status == O.OPTIMAL
    assert math.isclose(res.obj, box_closed_form(c, lp.xl, lp.xu)[0], rel_tol=1e-12)


def test_cfg1_matches_highs():
    lp = O.from_instance(make_cfg1())
    res = O.solve(lp, O.Options(tol=1e-8))
    obj, _, _ = highs(lp)
    assert res.status == O.OPTIMAL
    assert abs(res.obj - obj) <= 1e-6 * (1 + abs(obj))
    _check_invariants(lp, res, 1e-8)


def test_cfg2_shape_matches_highs_at_1e4():
    """A 200 x 500 member of the strong-branching family at the throughput
    tolerance: two 1e-4-optimal points bracket the optimum by the gap test."""
    lp = O.from_instance(make_cfg2(m=200, n=500))
    res = O.solve(lp, O.Options(tol=1e-4))
    obj, _, _ = highs(lp)
    assert res.status == O.OPTIMAL
    assert abs(res.obj - obj) <= 4e-4 * (1 + abs(obj))
    _check_invariants(lp, res, 1e-4)


def test_strong_branching_batch_semantics():
    """Each branch restricts the base LP (Section 5.1), so its optimum is no
    better than the base optimum; both children are checked against HiGHS."""
    lp = O.from_instance(make_cfg2(m=200, n=500))
    base = O.solve(lp, O.Options(tol=1e-8))
    vars_ = choose_fractional(base.x, 3, seed=7)
    D = fsb_deltas(base.x, vars_)
    assert list(D["kind"]) == [O.SET_LO] * 3 + [O.SET_HI] * 3
    for d in D:
        lpj = O.apply_delta(lp, int(d["kind"]), int(d["var"]), float(d["value"]))
        r = O.solve(lpj, O.Options(tol=1e-7), x_init=base.x, y_init=base.y, w_init=base.w)
        obj, _, _ = highs(lpj)
        assert r.status == O.OPTIMAL
        assert abs(r.obj - obj) <= 1e-5 * (1 + abs(obj))
        assert obj >= base.obj - 1e-6 * (1 + abs(base.obj))


def test_bound_tightening_semantics():
    """min x_j <= x0_j <= max x_j for the feasible witness x0 (Section 5.2)."""
    inst = make_cfg2(m=100, n=250)
    lp = O.from_instance(inst)
    vars_ = choose_vars(lp.n, 3, seed=5)
    D = obbt_deltas(vars_)
    res = [O.solve(O.apply_delta(lp, int(d["kind"]), int(d["var"]), float(d["value"])),
                   O.Options(tol=1e-7)) for d in D]
    for i, j in enumerate(vars_):
        lo = res[i].obj            # min x_j
        hi = -res[i + 3].obj       # max x_j = -min(-x_j)
        assert lp.xl[j] - 1e-6 <= lo <= inst.x0[j] + 1e-4 * (1 + abs(lo))
        assert inst.x0[j] - 1e-4 * (1 + abs(hi)) <= hi <= lp.xu[j] + 1e-6


def test_statuses():
    lp = O.from_instance(make_cfg1())
    # crossing bounds after a delta: closed form, never iterated
    bad = O.apply_delta(lp, O.SET_LO, 3, 11.0)
    r = O.solve(bad)
    assert r.status == O.INFEASIBLE_BOUNDS and r.iters == 0
    # exact iteration limit
    for K in (1, 2, 63, 64, 65, 130):
        r = O.solve(lp, O.Options(tol=0.0, max_iters=K))
        assert r.status == O.ITERATION_LIMIT and r.iters == K
    # NaN data is caught at the first evaluation
    lpn = O.LP(A=lp.A, c=lp.c.copy(), l=lp.l, u=lp.u, xl=lp.xl, xu=lp.xu, b=lp.b)
    lpn.c[5] = np.nan
    r = O.solve(lpn)
    assert r.status == O.NUMERICAL_ERROR and r.iters == 1


def test_restart_resets_iterate_to_tilde():
    """After a restart the next iteration starts from the anchor z~ (a restart
    leaves x inside the box); the Halpern iterate returned at a limit is the
    reflected-average of the last step."""
    lp = O.from_instance(make_cfg1())
    # the stopping tests precede the restart test: a limit at t = 64 wins
    assert O.solve(lp, O.Options(tol=0.0, max_iters=65)).restarts == []
    r1 = O.solve(lp, O.Options(tol=0.0, max_iters=66))
    assert r1.restarts == [64]
    # at the limit t=65 (k=0 after the restart), the Halpern weight is 1/2:
    # z^1 = (2 z~ - z) / 2 + z0 / 2 with z = z0 = anchor  ->  z~
    np.testing.assert_allclose(r1.x_iter, r1.x, atol=1e-14)


def test_batch_avg_single_lp_equals_solve():
    lp = O.from_instance(make_cfg1())
    a = O.solve(lp, O.Options(tol=1e-6))
    b = O.solve_batch_avg([lp], O.Options(tol=1e-6))[0]
    assert a.status == b.status and a.iters == b.iters and a.restarts == b.restarts
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.y, b.y)


def test_batch_avg_converges_each_lp():
    lp = O.from_instance(make_cfg2(m=100, n=250))
    lps = [O.apply_delta(lp, O.OBJ_UNIT, j, s) for j in (3, 17) for s in (1.0, -1.0)]
    res = O.solve_batch_avg(lps, O.Options(tol=1e-6))
    for lpj, r in zip(lps, res):
        obj, _, _ = highs(lpj)
        assert r.status == O.OPTIMAL
        assert abs(r.obj - obj) <= 2e-5 * (1 + abs(obj))
    # all LPs restart together
    longest = max(res, key=lambda r: r.iters)
    for r in res:
        assert set(r.restarts) == {t for t in longest.restarts if t < r.iters - 1}


# ---------------------------------------------------------------------------
# Worst-case rate of the Halpern iteration: with anchor weight 1/(k+2) and a
# nonexpansive map R, ||z^k - R z^k|| <= 2 ||z^0 - z*|| / (k+1) for every fixed
# point z* (Lieder, Optim. Lett. 2021).  Here R = 2T - I, nonexpansive in the
# metric M of the residual because T is firmly nonexpansive there, so the
# residual r(z^k) = ||T z^k - z^k||_M is at most ||z^0 - z*||_M / (k+1).  The
# bound holds along the oracle's own iterate trajectory once restarts, the
# stopping test and the infeasibility tests are switched off.
# ---------------------------------------------------------------------------

def _no_restarts(K, eta):
    return O.Options(tol=0.0, max_iters=K, beta_s=0.0, beta_n=0.0, beta_a=1e12,
                     infeas_tol=0.0, step_size=eta)


def _rate_setup(inst, seed):
    """eta, w, a start z^0 (zero, or random in the box and the barrier cone)
    and ||z^0 - z*||_M with z* the oracle's point converged to 1e-12."""
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    w = O.initial_primal_weight(lp)
    ref = O.solve(lp, O.Options(tol=1e-12, max_iters=400000, step_size=eta))
    assert ref.status == O.OPTIMAL
    if seed is None:
        x0, y0 = O.proj_box(np.zeros(lp.n), lp.xl, lp.xu), np.zeros(lp.m)
    else:
        rng = np.random.default_rng(seed)
        x0 = O.proj_box(rng.uniform(-1.0, 4.0, lp.n), lp.xl, lp.xu)
        y0 = O.proj_barrier_cone(rng.normal(size=lp.m), lp.l, lp.u)
    dist = O.fixed_point_residual(lp, x0, y0, ref.x, ref.y, w, eta)
    return lp, eta, w, x0, y0, dist


@pytest.mark.parametrize("start", [None, 101])
@pytest.mark.parametrize("inst", [make_tiny(s, m=4, n=7, senses="ELG", box=(0.0, 3.0))
                                  for s in range(3)] + [make_cfg1()],
                         ids=["tiny0", "tiny1", "tiny2", "cfg1"])
def test_halpern_rate_bound_along_the_trajectory(inst, start):
    lp, eta, w, x0, y0, dist = _rate_setup(inst, start)
    for K in (1, 2, 3, 5, 10, 30, 100, 300, 1000, 3000):
        res = O.solve(lp, _no_restarts(K, eta), x_init=x0, y_init=y0, w_init=w)
        assert res.iters == K and not res.restarts
        xt, yt = O.pdhg_operator(lp, res.x_iter, res.y_iter, eta / w, eta * w)
        r = O.fixed_point_residual(lp, res.x_iter, res.y_iter, xt, yt, w, eta)
        assert r <= dist / (K + 1) * (1 + 1e-6) + 1e-12, (K, r, dist / (K + 1))


def _worst_ratio(lp, eta, w, x0, y0, dist, update, K=3000):
    """max over k of r(z^k) (k+1) / ||z^0 - z*||_M for an iteration given by `update`."""
    x, y = x0.copy(), y0.copy()
    worst = 0.0
    for k in range(K):
        xt, yt = O.pdhg_operator(lp, x, y, eta / w, eta * w)
        worst = max(worst, O.fixed_point_residual(lp, x, y, xt, yt, w, eta) * (k + 1) / dist)
        x, y = update(k, x, y, xt, yt, x0, y0)
    return worst


def _halpern(k, z, z0):
    return (k + 1) / (k + 2) * z + z0 / (k + 2)


# plausible mistakes in the iteration, each planted in a copy of it built from
# the oracle's operator: the bound is violated, so the check above has teeth
_MISTAKES = {
    "not reflected": lambda k, x, y, xt, yt, x0, y0: (_halpern(k, xt, x0), _halpern(k, yt, y0)),
    "dual not reflected": lambda k, x, y, xt, yt, x0, y0: (_halpern(k, 2 * xt - x, x0),
                                                           _halpern(k, yt, y0)),
    "dual anchor sign": lambda k, x, y, xt, yt, x0, y0: (_halpern(k, 2 * xt - x, x0),
                                                         _halpern(k, 2 * yt - y, -y0)),
    "no anchor": lambda k, x, y, xt, yt, x0, y0: (2 * xt - x, 2 * yt - y),
    "anchor at z^k": lambda k, x, y, xt, yt, x0, y0: (_halpern(k, 2 * xt - x, x),
                                                      _halpern(k, 2 * yt - y, y)),
}


@pytest.mark.parametrize("mistake", sorted(_MISTAKES))
@pytest.mark.parametrize("seed", [1, 2])
def test_halpern_rate_bound_catches_planted_mistakes(seed, mistake):
    inst = make_tiny(seed, m=4, n=7, senses="ELG", box=(0.0, 3.0))
    args = _rate_setup(inst, 100 + seed)
    good = _worst_ratio(*args, lambda k, x, y, xt, yt, x0, y0: (_halpern(k, 2 * xt - x, x0),
                                                                _halpern(k, 2 * yt - y, y0)))
    assert good <= 1.0
    assert _worst_ratio(*args, _MISTAKES[mistake]) > 1.05


# ---------------------------------------------------------------------------
# Restarted trajectories (Section 4, Restarts).  With theta = 0 the smoothed
# weight equals the old one, so T and the metric M stay the same across
# restarts, and with z* a fixed point three facts follow from T being firmly
# nonexpansive in M:
#   (i)   every cycle starts no farther from z* than the first one does
#         (||T z - z*|| <= ||z - z*||, and a Halpern iterate is a convex
#         combination of R z^k and its anchor, both inside that ball);
#   (ii)  a new cycle's first residual is at most the residual that fired the
#         restart (||T(T z) - T z|| <= ||T z - z||);
#   (iii) inside each cycle the Halpern bound above holds from that cycle's
#         own start.
# Checked on cycles whose start is farther from z* than 1e-7 of the first,
# above the accuracy of the converged reference point and of rounding.
# ---------------------------------------------------------------------------

def _restart_opts(K, eta, C):
    return O.Options(tol=0.0, max_iters=K, eval_every=C, theta=0.0, infeas_tol=0.0, step_size=eta)


def _residual(lp, eta, w, x, y):
    xt, yt = O.pdhg_operator(lp, x, y, eta / w, eta * w)
    return O.fixed_point_residual(lp, x, y, xt, yt, w, eta)


def _oracle_cycles(lp, eta, w, x0, y0, K, run, js=(1, 2, 3, 5, 8, 13, 21, 34, 55)):
    """Cycles of one LP's restarted run of K iterations, read from shorter runs
    of the same solve (`run(max_iters)` returns that LP's result):
    max_iters = t + 1 returns T(z^t), which is the next cycle's start when t
    fired a restart, and max_iters = t returns z^t."""
    ts = run(K).restarts
    cycles = []
    for n, b in enumerate([0] + [t + 1 for t in ts]):
        if n == 0:
            start = (x0, y0)
        else:
            r = run(b)
            assert r.restarts == ts[:n - 1]
            start = (r.x, r.y)
        end = ts[n] if n < len(ts) else K - 1
        samples = [(0, _residual(lp, eta, w, *start))]
        for j in js:
            if b + j <= end:
                r = run(b + j)
                samples.append((j, _residual(lp, eta, w, r.x_iter, r.y_iter)))
        trig = None
        if n < len(ts):
            r = run(ts[n])
            trig = _residual(lp, eta, w, r.x_iter, r.y_iter)
        cycles.append(dict(start=start, trig=trig, samples=samples))
    return cycles


def _restart_ratios(lp, eta, w, ref, cycles, floor=1e-7):
    """Worst ratios of (i), (ii), (iii) over the cycles above the floor (each
    at most 1 when the facts hold) and the number of cycles checked."""
    dist = lambda z: O.fixed_point_residual(lp, z[0], z[1], ref.x, ref.y, w, eta)
    d0 = dist(cycles[0]["start"])
    out = {"start": 0.0, "first residual": 0.0, "rate": 0.0}
    checked = 0
    for n, c in enumerate(cycles):
        dn = dist(c["start"])
        if dn < floor * d0:
            break
        checked += 1
        out["start"] = max(out["start"], dn / d0)
        if n:
            out["first residual"] = max(out["first residual"],
                                        c["samples"][0][1] / cycles[n - 1]["trig"])
        for j, r in c["samples"]:
            out["rate"] = max(out["rate"], r * (j + 1) / dn)
    return out, checked


def _setup_with_star(inst, seed):
    lp, eta, w, x0, y0, _ = _rate_setup(inst, seed)
    ref = O.solve(lp, O.Options(tol=1e-12, max_iters=400000, step_size=eta))
    return lp, eta, w, x0, y0, ref


@pytest.mark.parametrize("C", [16, 64])
@pytest.mark.parametrize("start", [None, 101])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_restarted_trajectory_bounds(seed, start, C):
    inst = make_tiny(seed, m=4, n=7, senses="ELG", box=(0.0, 3.0))
    lp, eta, w, x0, y0, ref = _setup_with_star(inst, start)
    run = lambda KK: O.solve(lp, _restart_opts(KK, eta, C), x_init=x0, y_init=y0, w_init=w)
    cycles = _oracle_cycles(lp, eta, w, x0, y0, 1000, run)
    ratios, checked = _restart_ratios(lp, eta, w, ref, cycles)
    assert checked >= 4, checked
    for name, v in ratios.items():
        assert v <= 1.0 + 1e-6, (name, v)


@pytest.mark.parametrize("C", [16, 64])
def test_restarted_trajectory_bounds_batch_average(C):
    """The same facts for every LP of a batch under the batch-average scope,
    where the mean residual decides when all LPs restart together."""
    import functools
    lps = [O.from_instance(make_tiny(s, m=4, n=7, senses="ELG", box=(0.0, 3.0))) for s in range(3)]
    eta = min(O.step_size(lp.A) for lp in lps)
    ws = [O.initial_primal_weight(lp) for lp in lps]
    rng = np.random.default_rng(5)
    x0s = [O.proj_box(rng.uniform(-1.0, 4.0, lp.n), lp.xl, lp.xu) for lp in lps]
    y0s = [O.proj_barrier_cone(rng.normal(size=lp.m), lp.l, lp.u) for lp in lps]
    runs = functools.lru_cache(maxsize=None)(
        lambda KK: O.solve_batch_avg(lps, _restart_opts(KK, eta, C), x0s, y0s, ws))
    for j, lp in enumerate(lps):
        ref = O.solve(lp, O.Options(tol=1e-12, max_iters=400000, step_size=eta))
        assert ref.status == O.OPTIMAL
        cycles = _oracle_cycles(lp, eta, ws[j], x0s[j], y0s[j], 1000, lambda KK: runs(KK)[j])
        ratios, checked = _restart_ratios(lp, eta, ws[j], ref, cycles)
        assert checked >= 3, (j, checked)
        for name, v in ratios.items():
            assert v <= 1.0 + 1e-6, (j, name, v)


def _restarted_copy(lp, eta, w, x0, y0, C, K, mistake=None):
    """A copy of the restarted iteration built from the oracle's operator,
    residual and restart test, with a mistake planted in the restart."""
    x, y, xa, ya = x0, y0, x0, y0
    k, r0, r_prev = 0, None, None
    cycles = [dict(start=(x, y), trig=None, samples=[])]
    restarts = []
    for t in range(K):
        xt, yt = O.pdhg_operator(lp, x, y, eta / w, eta * w)
        full = t % C == 0
        r = O.fixed_point_residual(lp, x, y, xt, yt, w, eta)
        cycles[-1]["samples"].append((k if mistake != "k not reset" else len(cycles[-1]["samples"]), r))
        if k == 0:
            r0 = r
        elif full and O.restart_due(r, r0, r_prev, k, t, 0.2, 0.8, 0.36):
            cycles[-1]["trig"] = r
            restarts.append(t)
            if mistake == "restart to the anchor":
                x, y = xa, ya
            elif mistake == "anchor kept":
                x, y = xt, yt
            else:
                x, y, xa, ya = xt, yt, xt, yt
            cycles.append(dict(start=(x, y), trig=None, samples=[]))
            k = k + 1 if mistake == "k not reset" else 0
            r_prev = None
            continue
        if full or k == 0:
            r_prev = r
        x = (k + 1) / (k + 2) * (2 * xt - x) + xa / (k + 2)
        y = (k + 1) / (k + 2) * (2 * yt - y) + ya / (k + 2)
        k += 1
    return cycles, restarts


@pytest.mark.parametrize("seed", [0, 1])
def test_restarted_trajectory_bounds_catch_planted_mistakes(seed):
    inst = make_tiny(seed, m=4, n=7, senses="ELG", box=(0.0, 3.0))
    lp, eta, w, x0, y0, ref = _setup_with_star(inst, 100 + seed)
    K, C = 1500, 16
    cycles, restarts = _restarted_copy(lp, eta, w, x0, y0, C, K)
    # the copy restarts where the oracle does, and meets the bounds
    assert restarts == O.solve(lp, _restart_opts(K, eta, C), x_init=x0, y_init=y0,
                               w_init=w).restarts
    ratios, _ = _restart_ratios(lp, eta, w, ref, cycles)
    assert max(ratios.values()) <= 1.0 + 1e-6, ratios
    for mistake in ("restart to the anchor", "anchor kept", "k not reset"):
        cycles, _ = _restarted_copy(lp, eta, w, x0, y0, C, K, mistake)
        ratios, _ = _restart_ratios(lp, eta, w, ref, cycles)
        assert max(ratios.values()) > 1.5, (mistake, ratios)
