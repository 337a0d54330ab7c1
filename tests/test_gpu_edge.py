"""Degenerate shapes through the C ABI against the oracle: no rows at all,
only free rows (the box-only closed form), empty rows and columns, a matrix
without nonzeros, one-variable LPs, the widest batch, and free and half-bounded
variables in an LP of several tiles."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from tests.gpu_common import rel_err, elem_err, ITER_RTOL
from workloads import deltas, BASE, SET_LO, SET_HI, OBJ_UNIT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2601_21990_amd.pdlpb as P
    return P


def _ctx(P, A, b, sense, c, l, u, **kw):
    A = sp.csr_matrix(A)
    return P.Context(A.shape[0], A.shape[1], A.indptr.astype(np.int64), A.indices.astype(np.int32),
                     A.data, c, b, np.frombuffer(sense.encode(), dtype=np.uint8), l, u, **kw)


def _oracle_lp(A, b, sense, c, l, u):
    A = sp.csr_matrix(A)
    return O.from_arrays(A.shape[0], A.shape[1], A.indptr, A.indices, A.data, c, b,
                         np.frombuffer(sense.encode(), dtype=np.uint8), l, u)


CASES = {
    "no_rows": (np.zeros((0, 3)), np.zeros(0), "", [1.0, -2.0, 0.5], [0.0, -1.0, 2.0],
                [4.0, 3.0, 5.0]),
    "free_rows": ([[1.0, 2.0, 0.0], [0.0, 1.0, -1.0]], [3.0, 1.0], "NN", [1.0, -2.0, 0.5],
                  [0.0, -1.0, 2.0], [4.0, 3.0, 5.0]),
    "empty_row_and_column": ([[1.0, 0.0, 1.0, 0.0], [0.0, 0.0, 0.0, 0.0], [2.0, 0.0, -1.0, 0.0]],
                             [2.0, 0.0, 1.0], "ELG", [1.0, 3.0, 1.0, -1.0],
                             [0.0, 0.0, 0.0, 0.0], [5.0, 5.0, 5.0, 2.0]),
    "no_nonzeros": (np.zeros((2, 3)), [0.0, 1.0], "EL", [2.0, -1.0, 0.0], [0.0, 0.0, -1.0],
                    [1.0, 1.0, 1.0]),
    "one_variable": ([[2.0]], [3.0], "L", [-1.0], [0.0], [10.0]),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("K", [1, 50])
def test_degenerate_shapes_match_oracle(P, name, K):
    """Fixed iteration counts below the first full evaluation after t = 0: these
    LPs reach their optima exactly, and with tol = 0 the rounding of a full
    evaluation's sums (zero or not) would decide where each side stops."""
    A, b, sense, c, l, u = CASES[name]
    lp = _oracle_lp(A, b, sense, c, l, u)
    eta = O.step_size(lp.A)
    n = lp.n
    D = deltas([BASE, SET_LO, SET_HI, OBJ_UNIT], [0, n - 1, 0, n - 1], [0.0, 0.5, 0.5, -1.0])
    with _ctx(P, A, b, sense, c, l, u, step_size=eta) as ctx:
        ctx.set_batch(D)
        ctx.solve(tol=0.0, max_iters=K)
        got = [ctx.get(j) for j in range(len(D))]
    for j, d in enumerate(D):
        lpj = O.apply_delta(lp, int(d["kind"]), int(d["var"]), float(d["value"]))
        r = O.solve(lpj, O.Options(tol=0.0, max_iters=K, step_size=eta))
        assert got[j]["status"] == r.status and got[j]["iters"] == r.iters, (name, j)
        assert rel_err(got[j]["x"], r.x) <= ITER_RTOL, (name, j)
        assert elem_err(got[j]["x"], r.x) <= ITER_RTOL, (name, j)
        if lp.m:
            assert rel_err(got[j]["y"], r.y) <= ITER_RTOL, (name, j)
            assert elem_err(got[j]["y"], r.y) <= ITER_RTOL, (name, j)


def test_box_only_closed_form(P):
    """Free rows only: each x_j ends at the bound its cost sign selects and y = 0."""
    A, b, sense, c, l, u = CASES["free_rows"]
    with _ctx(P, A, b, sense, c, l, u) as ctx:
        ctx.set_batch(deltas([BASE], [0], [0.0]))
        ctx.solve(tol=1e-10, max_iters=10000)
        r = ctx.get(0)
    c, l, u = map(np.asarray, (c, l, u))
    want = np.where(c > 0, l, np.where(c < 0, u, np.clip(0.0, l, u)))
    assert r["status"] == P.STATUS_OPTIMAL
    np.testing.assert_allclose(r["x"], want, atol=1e-9)
    np.testing.assert_array_equal(r["y"], np.zeros(2))
    assert r["obj"] == pytest.approx(float(c @ want), abs=1e-9)


def test_maximum_batch_width(P):
    """B = 4096, the largest batch a context accepts by default: 128 distinct
    bound-tightening LPs, each placed 32 times at scattered positions.  Every
    copy of an LP carries the same bits (its arithmetic does not depend on
    its slot or on the batch), a sample matches the oracle's trajectory over a
    full evaluation, and one LP more is rejected."""
    from tests.gpu_common import make_ctx, lp_for, assert_trajectory_match
    from workloads import make_cfg2, obbt_deltas, choose_vars
    inst = make_cfg2(m=200, n=500)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    U = obbt_deltas(choose_vars(inst.n, 64, seed=7))          # 128 distinct LPs
    perm = np.random.default_rng(7).permutation(4096)
    D = np.tile(U, 32)[perm]                                    # copy c of LP u at perm^-1
    K = 65
    with make_ctx(inst, eta) as ctx:
        assert ctx.options.max_batch == 4096
        ctx.set_batch(D)
        ctx.solve(tol=0.0, max_iters=K)
        out = ctx.get_batch()
        sample = {}
        for u in (0, 63, 64, 127):
            j = int(np.nonzero(perm % 128 == u)[0][0])
            sample[u] = (ctx.get(j), ctx.get_trace(j))
        with pytest.raises(P.PdlpbError) as e:
            ctx.set_batch(np.tile(U, 33)[:4097])
        assert e.value.code == P.EINVAL
    assert np.all(out["iters"] == K)
    src = perm % 128
    for u in range(128):
        rows = np.nonzero(src == u)[0]
        assert rows.size == 32
        for q in ("X", "Y"):
            assert np.array_equal(out[q][rows], np.broadcast_to(out[q][rows[0]], out[q][rows].shape))
    for u, (res, tr) in sample.items():
        ores = O.solve(lp_for(lp, U[u]), O.Options(tol=0.0, max_iters=K, step_size=eta))
        assert_trajectory_match(res, tr, ores, what=f"LP {u}")


@pytest.mark.parametrize("K", [1, 65, 300])
def test_infinite_bounds_several_tiles(P, K):
    """Free, lower-only and upper-only variables in a 200 x 500 LP (several row
    tiles, nine LPs for a ragged slot tile): the projections, reduced costs and
    support functions at infinite bounds give the oracle's iterates, statuses
    and restart iterations after K iterations."""
    import dataclasses
    from tests.gpu_common import lp_for, oracle_run, assert_trajectory_match
    from workloads import make_cfg2
    inst = make_cfg2(m=200, n=500)
    kind = np.random.default_rng(7).integers(0, 4, size=inst.n)   # box, free, [l, inf), (-inf, u]
    l, u = inst.l.copy(), inst.u.copy()
    l[kind == 1], u[kind == 1] = -np.inf, np.inf
    u[kind == 2] = np.inf
    l[kind == 3] = -np.inf
    inst = dataclasses.replace(inst, l=l, u=u)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    free, lower, upper = (int(np.flatnonzero(kind == k)[0]) for k in (1, 2, 3))
    D = deltas([BASE, SET_LO, SET_HI, SET_HI, SET_LO, OBJ_UNIT, OBJ_UNIT, SET_LO, SET_HI],
               [0, free, free, lower, upper, free, lower, lower, upper],
               [0.0, -1.0, 2.0, 5.0, 3.0, 1.0, -1.0, 1.0, 8.0])
    with P.Context.from_instance(inst, step_size=float(eta)) as ctx:
        ctx.set_batch(D)
        ctx.solve(tol=0.0, max_iters=K)
        got = [(ctx.get(j), ctx.get_trace(j)) for j in range(len(D))]
    for j, d in enumerate(D):
        ores = oracle_run(lp_for(lp, d), eta, 0.0, K)
        assert_trajectory_match(*got[j], ores, what=f"LP {j} K={K}")
