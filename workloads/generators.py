"""Seeded synthetic LP instances and batch specifications.

This module only *builds inputs*: sparse matrices, right-hand sides, row
senses, costs, variable boxes, and the per-LP change lists ("deltas") that
turn one base LP into a batch.  It performs none of the solver's arithmetic,
so both the FP64 reference solver and the GPU library may consume the same
bytes.

Instance shapes follow the workloads of the batched-PDHG paper
(arXiv 2601.21990): strong branching changes one variable bound per LP
(Section 5.1, full strong branching) and bound tightening replaces the
objective by +-e_j (Section 5.2, optimisation-based bound tightening).  The
paper measures on instance families that are not available here; these
random families stand in for them (sizes in ``CONFIGS``).

Every generator draws from ``numpy.random.default_rng`` (PCG64) seeded with
``seed_for(cfg, rep)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List

import numpy as np

# Delta kinds.  Values are part of the C ABI (pdlpb_delta.kind).
BASE = 0       # the base LP unchanged
SET_LO = 1     # lower bound of variable `var` becomes `value` (branch up)
SET_HI = 2     # upper bound of variable `var` becomes `value` (branch down)
OBJ_UNIT = 3   # objective becomes value * e_var (bound tightening: +1 min, -1 max)

DELTA_DTYPE = np.dtype([("kind", "<i4"), ("var", "<i4"), ("value", "<f8")])

SEED_BASE = 2601021990


def seed_for(cfg: int, rep: int = 0) -> int:
    return SEED_BASE + 1000 * cfg + rep


@dataclass
class LPInstance:
    """One base LP  min c'x  s.t. rows of A x against b by `sense`, l <= x <= u.

    A is CSR with sorted column indices inside each row.  `sense` holds one
    byte per row: b'E' (= b), b'L' (<= b) or b'G' (>= b).  `x0` is the
    feasibility witness the instance was built from.
    """
    m: int
    n: int
    row_ptr: np.ndarray   # int64, m+1
    col_idx: np.ndarray   # int32, nnz
    val: np.ndarray       # float64, nnz
    c: np.ndarray         # float64, n
    b: np.ndarray         # float64, m
    sense: np.ndarray     # uint8 (ASCII), m
    l: np.ndarray         # float64, n  (variable lower bounds)
    u: np.ndarray         # float64, n  (variable upper bounds)
    x0: np.ndarray        # float64, n  (witness)
    name: str = ""
    meta: Dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        A = np.zeros((self.m, self.n))
        for i in range(self.m):
            s, e = self.row_ptr[i], self.row_ptr[i + 1]
            A[i, self.col_idx[s:e]] = self.val[s:e]
        return A


def _coo_to_csr(m: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, cols.astype(np.int32), vals.astype(np.float64)


def _k_per_column(rng, m: int, n: int, k) -> tuple:
    """Exactly k[j] nonzeros in column j at distinct uniform rows."""
    ks = np.broadcast_to(np.asarray(k), (n,)).astype(np.int64)
    kmax = int(ks.max())
    if kmax > m:
        raise ValueError("more nonzeros per column than rows")
    used = np.arange(kmax)[None, :] < ks[:, None]          # n x kmax
    draw = rng.integers(0, m, size=(n, kmax))
    bad = np.arange(n)
    while bad.size:
        # columns whose used entries repeat a row are redrawn whole
        sub = np.where(used[bad], draw[bad], -1 - np.arange(kmax)[None, :])
        sub.sort(axis=1)
        dup = np.any(sub[:, 1:] == sub[:, :-1], axis=1)
        bad = bad[dup]
        if bad.size:
            draw[bad] = rng.integers(0, m, size=(bad.size, kmax))
    cols = np.repeat(np.arange(n, dtype=np.int64), ks)
    rows = draw[used]
    return rows.astype(np.int64), cols


def _finish(rng, name, m, n, rows, cols, vals, x0, senses, lo, hi, meta=None) -> LPInstance:
    row_ptr, col_idx, val = _coo_to_csr(m, rows, cols, vals)
    # row activity of the witness: the instance is feasible by construction
    ax0 = np.zeros(m)
    np.add.at(ax0, rows, vals * x0[cols])
    slack = rng.uniform(0.0, 1.0, size=m)
    b = ax0.copy()
    b[senses == ord("L")] += slack[senses == ord("L")]
    b[senses == ord("G")] -= slack[senses == ord("G")]
    c = rng.standard_normal(n)
    return LPInstance(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, val=val, c=c, b=b,
                      sense=senses.astype(np.uint8), l=np.full(n, float(lo)),
                      u=np.full(n, float(hi)), x0=x0, name=name, meta=meta or {})


def make_tiny(seed: int, m: int = 3, n: int = 5, density: float = 0.6,
              senses: str = "ELG", box=(0.0, 4.0)) -> LPInstance:
    """Small random LP for brute-force checks (vertex enumeration)."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    rows, cols = np.nonzero(mask)
    vals = rng.standard_normal(rows.size)
    x0 = rng.uniform(box[0], box[1], size=n)
    sv = np.array([ord(senses[i % len(senses)]) for i in range(m)], dtype=np.uint8)
    return _finish(rng, f"tiny{seed}", m, n, rows.astype(np.int64), cols.astype(np.int64),
                   vals, x0, sv, box[0], box[1])


def make_cfg1(rep: int = 0) -> LPInstance:
    """50x100, 5% Bernoulli mask, N(0,1) values, all equality rows, box [0,10]."""
    rng = np.random.default_rng(seed_for(1, rep))
    m, n = 50, 100
    mask = rng.random((m, n)) < 0.05
    rows, cols = np.nonzero(mask)
    vals = rng.standard_normal(rows.size)
    x0 = rng.uniform(0.0, 10.0, size=n)
    senses = np.full(m, ord("E"), dtype=np.uint8)
    return _finish(rng, "cfg1", m, n, rows.astype(np.int64), cols.astype(np.int64), vals,
                   x0, senses, 0.0, 10.0)


def make_cfg2(rep: int = 0, m: int = 2000, n: int = 5000) -> LPInstance:
    """2000x5000, 5 nonzeros per column N(0,1); 1000 E rows then 1000 L rows; box [0,10]."""
    rng = np.random.default_rng(seed_for(2, rep))
    rows, cols = _k_per_column(rng, m, n, 5)
    vals = rng.standard_normal(rows.size)
    x0 = rng.uniform(0.0, 10.0, size=n)
    senses = np.full(m, ord("L"), dtype=np.uint8)
    senses[: m // 2] = ord("E")
    return _finish(rng, "cfg2", m, n, rows, cols, vals, x0, senses, 0.0, 10.0)


def make_cfg3(rep: int = 0, m: int = 20000, n: int = 50000) -> LPInstance:
    """20000x50000, 8 nonzeros per column U[-1,1], senses uniform over E/L/G; box [0,5]."""
    rng = np.random.default_rng(seed_for(3, rep))
    rows, cols = _k_per_column(rng, m, n, 8)
    vals = rng.uniform(-1.0, 1.0, size=rows.size)
    x0 = rng.uniform(0.0, 5.0, size=n)
    senses = np.array([ord("E"), ord("L"), ord("G")], dtype=np.uint8)[rng.integers(0, 3, m)]
    return _finish(rng, "cfg3", m, n, rows, cols, vals, x0, senses, 0.0, 5.0)


def cfg4_sizes() -> List[int]:
    return [int(round(10 ** (3 + 2 * i / 7))) for i in range(8)]


def make_cfg4(i: int, rep: int = 0) -> LPInstance:
    """Base matrix i of the mixed family: m = round(10^(3+2i/7)), n = 2.5 m,
    4..12 nonzeros per column N(0,1), senses uniform, box [0,10]."""
    rng = np.random.default_rng(seed_for(4, 100 * rep + i))
    m = cfg4_sizes()[i]
    n = int(round(2.5 * m))
    k = rng.integers(4, 13, size=n)
    rows, cols = _k_per_column(rng, m, n, k)
    vals = rng.standard_normal(rows.size)
    x0 = rng.uniform(1.0, 9.0, size=n)
    senses = np.array([ord("E"), ord("L"), ord("G")], dtype=np.uint8)[rng.integers(0, 3, m)]
    return _finish(rng, f"cfg4_{i}", m, n, rows, cols, vals, x0, senses, 0.0, 10.0)


def make_cfg5(base: int = 0, m: int = 200000, n: int = 500000) -> LPInstance:
    """200k x 500k, 4 nonzeros per column N(0,1), senses uniform, box [0,10]."""
    rng = np.random.default_rng(seed_for(5, base))
    rows, cols = _k_per_column(rng, m, n, 4)
    vals = rng.standard_normal(rows.size)
    x0 = rng.uniform(1.0, 9.0, size=n)
    senses = np.array([ord("E"), ord("L"), ord("G")], dtype=np.uint8)[rng.integers(0, 3, m)]
    return _finish(rng, f"cfg5_{base}", m, n, rows, cols, vals, x0, senses, 0.0, 10.0)


def make_setcover(rep: int = 0, m: int = 2000, n: int = 4000, k: int = 8) -> LPInstance:
    """Set-covering LP relaxation: min c'x, every row covered (sum over its
    columns >= 1), 0 <= x <= 1.  Each row holds k distinct random columns with
    coefficient 1; costs c ~ U{1..100}.  x = 1 is feasible."""
    rng = np.random.default_rng(seed_for(8, rep))
    cols = np.stack([rng.choice(n, size=k, replace=False) for _ in range(m)]).ravel()
    rows = np.repeat(np.arange(m), k)
    row_ptr, col_idx, val = _coo_to_csr(m, rows.astype(np.int64), cols.astype(np.int64),
                                        np.ones(m * k))
    c = rng.integers(1, 101, size=n).astype(np.float64)
    return LPInstance(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, val=val, c=c,
                      b=np.ones(m), sense=np.full(m, ord("G"), dtype=np.uint8),
                      l=np.zeros(n), u=np.ones(n), x0=np.ones(n), name="setcover")


def make_facility(rep: int = 0, F: int = 100, C: int = 1000, k: int = 10) -> LPInstance:
    """Capacitated facility-location LP relaxation on random points in the unit
    square: facilities i with opening cost f_i ~ U[50, 150] (variables y_i,
    first F columns), customers j with demand d_j ~ U[5, 35] served by their k
    nearest facilities (variables x_ij, cost = distance * 100 * d_j).  Rows:
    sum_i x_ij = 1 for every customer (E); x_ij - y_i <= 0 for every pair (L);
    sum_j d_j x_ij - s_i y_i <= 0 for every facility (L), with s_i = U[1.05, 2]
    times the load the even split below puts on i.  Bounds [0, 1].  Opening
    every facility and splitting each customer evenly over its k facilities is
    feasible."""
    rng = np.random.default_rng(seed_for(9, rep))
    fp = rng.random((F, 2))
    cp = rng.random((C, 2))
    dist = np.linalg.norm(cp[:, None, :] - fp[None, :, :], axis=2)
    near = np.argsort(dist, axis=1)[:, :k]                  # C x k facility indices
    dem = rng.uniform(5.0, 35.0, size=C)
    n = F + C * k
    m = C + C * k + F
    pair = np.arange(C * k)
    xcol = F + pair                                          # column of x_ij
    cust = np.repeat(np.arange(C), k)
    fac = near.ravel()
    load = np.bincount(fac, weights=dem[cust] / k, minlength=F)
    cap = np.where(load > 0, load * rng.uniform(1.05, 2.0, size=F), 1.0)
    rows = np.concatenate([cust, C + pair, C + pair, C + C * k + fac, C + C * k + np.arange(F)])
    cols = np.concatenate([xcol, xcol, fac, xcol, np.arange(F)])
    vals = np.concatenate([np.ones(C * k), np.ones(C * k), -np.ones(C * k), dem[cust], -cap])
    row_ptr, col_idx, val = _coo_to_csr(m, rows.astype(np.int64), cols.astype(np.int64), vals)
    c = np.concatenate([rng.uniform(50.0, 150.0, size=F), 100.0 * dist[cust, fac] * dem[cust]])
    b = np.concatenate([np.ones(C), np.zeros(C * k + F)])
    sense = np.concatenate([np.full(C, ord("E")), np.full(C * k + F, ord("L"))]).astype(np.uint8)
    x0 = np.concatenate([np.ones(F), np.full(C * k, 1.0 / k)])
    return LPInstance(m=m, n=n, row_ptr=row_ptr, col_idx=col_idx, val=val, c=c, b=b,
                      sense=sense, l=np.zeros(n), u=np.ones(n), x0=x0, name="facility")


def make_badly_scaled(rep: int = 0, m: int = 200, n: int = 500) -> LPInstance:
    """The 2000 x 5000 family at a smaller size with rows multiplied by
    10^U[-3, 3] (their right-hand sides with them) and objective entries by
    10^U[-2, 2]: the same feasible set, entries spread over twelve decades."""
    inst = make_cfg2(rep, m=m, n=n)
    rng = np.random.default_rng(seed_for(7, rep))
    rs = 10.0 ** rng.uniform(-3.0, 3.0, size=m)
    cs = 10.0 ** rng.uniform(-2.0, 2.0, size=n)
    rows = np.repeat(np.arange(m), np.diff(inst.row_ptr))
    return LPInstance(m=m, n=n, row_ptr=inst.row_ptr, col_idx=inst.col_idx,
                      val=inst.val * rs[rows], c=inst.c * cs, b=inst.b * rs, sense=inst.sense,
                      l=inst.l, u=inst.u, x0=inst.x0, name="badly_scaled")


def make_packing(rep: int = 0, m: int = 200, n: int = 500, k: int = 5,
                 box=(0.0, 10.0)) -> LPInstance:
    """Packing rows with a finite box: k nonzeros per column drawn U[0.5, 1.5],
    all rows <=, witness x0 ~ U[0, 2].  Row capacities sit well below what the
    box allows, so maximising a variable meets its rows before its upper bound
    (bound tightening moves bounds on this family)."""
    rng = np.random.default_rng(seed_for(6, rep))
    rows, cols = _k_per_column(rng, m, n, k)
    vals = rng.uniform(0.5, 1.5, size=rows.size)
    x0 = rng.uniform(0.0, 2.0, size=n)
    senses = np.full(m, ord("L"), dtype=np.uint8)
    return _finish(rng, "packing", m, n, rows, cols, vals, x0, senses, box[0], box[1])


# ---------------------------------------------------------------------------
# batch specifications
# ---------------------------------------------------------------------------

def deltas(kinds, vars_, values) -> np.ndarray:
    d = np.zeros(len(kinds), dtype=DELTA_DTYPE)
    d["kind"] = kinds
    d["var"] = vars_
    d["value"] = values
    return d


def choose_fractional(x_rel: np.ndarray, p: int, seed: int,
                      lo: float = 0.1, hi: float = 0.9) -> np.ndarray:
    """Pick p distinct variables whose fractional part lies in [lo, hi]."""
    frac = x_rel - np.floor(x_rel)
    cand = np.nonzero((frac >= lo) & (frac <= hi))[0]
    if cand.size < p:
        raise ValueError(f"only {cand.size} fractional candidates, need {p}")
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(cand, size=p, replace=False)).astype(np.int32)


def fsb_deltas(x_rel: np.ndarray, vars_: np.ndarray) -> np.ndarray:
    """Full strong branching batch of 2p LPs: column i raises the lower bound of
    vars_[i] to ceil(x_rel), column p+i lowers its upper bound to floor(x_rel)
    (Section 5.1)."""
    p = len(vars_)
    xv = x_rel[vars_]
    kinds = np.concatenate([np.full(p, SET_LO), np.full(p, SET_HI)])
    values = np.concatenate([np.ceil(xv), np.floor(xv)])
    return deltas(kinds, np.concatenate([vars_, vars_]), values)


def obbt_deltas(vars_: np.ndarray) -> np.ndarray:
    """Bound tightening batch of 2p LPs: column i minimises x_{vars_[i]},
    column p+i maximises it, i.e. minimises -x (Section 5.2)."""
    p = len(vars_)
    kinds = np.full(2 * p, OBJ_UNIT)
    values = np.concatenate([np.ones(p), -np.ones(p)])
    return deltas(kinds, np.concatenate([vars_, vars_]), values)


def choose_vars(n: int, p: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=p, replace=False)).astype(np.int32)


def lp_to_npz(lp: LPInstance, path: str, **extra) -> None:
    np.savez(path, m=lp.m, n=lp.n, row_ptr=lp.row_ptr, col_idx=lp.col_idx, val=lp.val,
             c=lp.c, b=lp.b, sense=lp.sense, l=lp.l, u=lp.u, x0=lp.x0, **extra)


def lp_from_npz(path: str) -> LPInstance:
    z = np.load(path, allow_pickle=False)
    return LPInstance(m=int(z["m"]), n=int(z["n"]), row_ptr=z["row_ptr"], col_idx=z["col_idx"],
                      val=z["val"], c=z["c"], b=z["b"], sense=z["sense"], l=z["l"], u=z["u"],
                      x0=z["x0"])
