"""Helpers shared by the GPU parity tests: build a library context and the
matching reference LPs from one seeded instance, and compare results."""
from __future__ import annotations

import functools

import numpy as np

import oracle as O
from workloads import make_cfg2, choose_fractional, fsb_deltas, seed_for

ITER_RTOL = 1e-9          # relative error on iterates after a fixed iteration count (FP64)
# The KKT measures of eq:stopping are ratios of norms of the iterates; iterates
# within ITER_RTOL move them by at most ITER_RTOL times norm ratios such as
# ||A|| ||x|| / (1 + ||Ax||), which stay below 100 on these workloads.
KKT_ATOL = 1e-7
# |c'x_gpu - c'x_ref| <= ||c|| ||x|| ITER_RTOL, and ||c|| ||x|| / (1 + |c'x|)
# stays below 1000 on these workloads
OBJ_RTOL = 1e-6


def rel_err(a, b) -> float:
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1.0))


def elem_scale(b, floor="one"):
    """Per-coordinate scale of the reference vector b: max(|b_i|, 1), or with
    floor="rms" max(|b_i|, rms(b), 1).  Rounding moves a coordinate in
    proportion to the magnitudes mixed into it (its row's terms, the norms in
    the primal weight), not to its own value, so after many iterations on a
    vector whose entries are typically far above 1 a coordinate near zero
    carries the absolute error of its neighbours."""
    b = np.asarray(b, dtype=np.float64)
    s = np.maximum(np.abs(b), 1.0)
    if floor == "rms" and b.size:
        s = np.maximum(s, float(np.sqrt(np.mean(b * b))))
    return s


def elem_err(a, b, floor="one") -> float:
    """Largest coordinate error, each relative to its own reference value:
    max_i |a_i - b_i| / max(|b_i|, 1) (see elem_scale for floor="rms").  The
    norm-relative error can hide one wrong coordinate of a long vector; this
    cannot."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    if a.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b) / elem_scale(b, floor)))


def assert_iterates_match(pairs, rtol=ITER_RTOL, what="", floor="one"):
    """Every (gpu, reference) vector pair agrees per LP in norm and per coordinate."""
    worst = 0.0
    for name, g, o in pairs:
        en, ee = rel_err(g, o), elem_err(g, o, floor)
        if not (en <= rtol and ee <= rtol):
            g64, o64 = np.asarray(g, dtype=np.float64), np.asarray(o, dtype=np.float64)
            i = int(np.argmax(np.abs(g64 - o64) / elem_scale(o64, floor)))
            rms = float(np.sqrt(np.mean(o64 * o64)))
            raise AssertionError((what, name, en, ee, f"worst coordinate {i}: gpu {g64[i]!r} "
                                  f"ref {o64[i]!r}, rms of ref {rms:.6g}"))
        worst = max(worst, en, ee)
    return worst


def lp_for(base_lp, delta):
    return O.apply_delta(base_lp, int(delta["kind"]), int(delta["var"]), float(delta["value"]))


def make_ctx(inst, eta=None, **kw):
    import paper_2601_21990_amd.pdlpb as P
    opts = {}
    if eta is not None:
        opts["step_size"] = float(eta)
    opts.update(kw)
    return P.Context.from_instance(inst, **opts)


@functools.lru_cache(maxsize=None)
def cfg2_setup(m=2000, n=5000, p=32):
    """Strong-branching batch: base LP solved by the reference solver to 1e-6,
    2p bound changes on fractional variables, warm start from the base."""
    inst = make_cfg2(m=m, n=n)
    lp = O.from_instance(inst)
    eta = O.step_size(lp.A)
    base = O.solve(lp, O.Options(tol=1e-6, step_size=eta))
    vars_ = choose_fractional(base.x, p, seed_for(2, 0))
    D = fsb_deltas(base.x, vars_)
    return inst, lp, eta, base, D


def oracle_run(lp, eta, tol, max_iters, x0=None, y0=None, w0=None, **kw):
    return O.solve(lp, O.Options(tol=tol, max_iters=max_iters, step_size=eta, **kw),
                   x_init=x0, y_init=y0, w_init=w0)


def assert_trajectory_match(gpu_res, gpu_trace, ores, rtol=ITER_RTOL, what="", floor="one"):
    assert gpu_res["status"] == ores.status, (what, gpu_res["status"], ores.status)
    assert gpu_res["iters"] == ores.iters, (what, gpu_res["iters"], ores.iters)
    assert gpu_trace["restart_log"] == ores.restarts[:64], (what, gpu_trace["restart_log"],
                                                            ores.restarts)
    ex = rel_err(gpu_res["x"], ores.x)
    ey = rel_err(gpu_res["y"], ores.y)
    assert ex <= rtol and ey <= rtol, (what, ex, ey)
    # per coordinate as well: z~ (the returned point)
    assert_iterates_match((("x~", gpu_res["x"], ores.x), ("y~", gpu_res["y"], ores.y)), rtol, what,
                          floor)
    if ores.kkt is not None and "kkt" in gpu_res:
        ref = (ores.kkt.gap, ores.kkt.primal, ores.kkt.dual, ores.kkt.rel)
        for name, a, b in zip(("gap", "primal", "dual", "max"), gpu_res["kkt"], ref):
            if np.isfinite(b):
                assert abs(a - b) <= KKT_ATOL, (what, name, a, b)
            else:
                assert a == b or (np.isnan(a) and np.isnan(b)), (what, name, a, b)
        assert abs(gpu_res["obj"] - ores.kkt.obj) <= OBJ_RTOL * (1 + abs(ores.kkt.obj)), \
            (what, "obj", gpu_res["obj"], ores.kkt.obj)
    if ores.x_iter is not None:
        # the Halpern iterate z^{k+1}, in norm and per coordinate
        assert_iterates_match((("x_iter", gpu_trace["x_iter"], ores.x_iter),
                               ("y_iter", gpu_trace["y_iter"], ores.y_iter)), rtol, what, floor)
    return max(ex, ey)
