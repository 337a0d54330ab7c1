"""Parity at the largest size, in the launch configuration the benchmark
times: A 200000 x 500000 (4 N(0,1) nonzeros per column), FP64, B = 512
bound-tightening LPs, default options (the tile autotuner times its candidate
shapes on the first block of iterations, as in the benchmark), 65 iterations
(one full evaluation with its restart tests).  The oracle recomputes a sample of the
LPs one at a time with its own step size; every LP of the batch must also be
finite and still running or stopped with a valid status."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_common import make_ctx, lp_for, assert_trajectory_match
from workloads import make_cfg5, obbt_deltas, choose_vars

pytestmark = pytest.mark.gpu

K = 65


@pytest.fixture(scope="module")
def P():
    import paper_2601_21990_amd.pdlpb as P
    return P


def test_largest_size_sampled_lps_match_oracle(P):
    inst = make_cfg5()
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    D = obbt_deltas(choose_vars(inst.n, 256, seed=512))
    with make_ctx(inst, eta) as ctx:
        ctx.set_batch(D)
        ctx.solve(tol=0.0, max_iters=K)
        st = ctx.get_batch(want_x=False, want_y=False)
        sample = [0, 255, 256, 511]
        res = {j: (ctx.get(j), ctx.get_trace(j)) for j in sample}
    assert np.all(st["iters"] == K) and np.all(st["status"] == P.STATUS_ITERATION_LIMIT)
    assert np.all(np.isfinite(st["kkt"]))
    for j in sample:
        ores = O.solve(lp_for(lp, D[j]), O.Options(tol=0.0, max_iters=K, step_size=eta))
        assert_trajectory_match(*res[j], ores, what=f"LP {j}")
