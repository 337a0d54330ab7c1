"""Continuous-batching request loop over resident base LPs.

Each base LP (constraint matrix, bounds, objective and a warm start) lives in
its own library context on the GPU.  A request is a strong-branching or
bound-tightening batch on one base: a list of per-LP changes.  Requests are
queued in the library as they arrive; every round the loop launches one block
of iterations on every context that has work (admitting queued LPs into
columns freed by finished ones), then waits for all of them, so the blocks of
different bases run concurrently on the device.  A request completes when all
of its LPs have stopped; its latency is completion time minus arrival time.

Admission by memory footprint: a context holds `max_batch` LP columns and
`result_capacity` result rows, both allocated when serving begins; LPs beyond
the free columns wait in the library's FIFO queue, and a request whose LPs do
not fit the free result rows waits in this loop until rows are released.  The
requests of one base enter the library in arrival order: one that does not fit
holds back the later ones of its base, so a large request is not overtaken
indefinitely by small ones.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import pdlpb as P


@dataclass
class Request:
    base: int
    deltas: np.ndarray
    arrival: float
    tol: float = 1e-4
    max_iters: int = 100000
    ids: List[int] = field(default_factory=list)
    pending: int = 0
    submitted: Optional[float] = None
    done: Optional[float] = None
    statuses: Dict[int, int] = field(default_factory=dict)
    iters: Dict[int, int] = field(default_factory=dict)
    objs: Dict[int, float] = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Server:
    def __init__(self, contexts: List[P.Context], warm: bool = True, keep_results: bool = False):
        self.ctx = contexts
        self.warm = warm
        self.keep_results = keep_results
        self.waiting: List[Request] = []            # not yet in the library (result rows full)
        self.by_id: List[Dict[int, Request]] = [dict() for _ in contexts]
        self.results: Dict[tuple, dict] = {}
        self.completed: List[Request] = []
        self.lps_done = 0

    def submit(self, req: Request) -> None:
        self.waiting.append(req)
        self._admit_waiting()

    def _admit_waiting(self) -> None:
        still = []
        blocked = set()           # bases whose oldest waiting request did not fit
        for req in self.waiting:
            if req.base in blocked:
                still.append(req)
                continue
            ctx = self.ctx[req.base]
            try:
                ids = ctx.submit(req.deltas, P.WARM_BASE if self.warm else P.WARM_NONE,
                                 req.tol, req.max_iters)
            except P.PdlpbError as e:
                if e.code != P.ENOMEM:
                    raise
                blocked.add(req.base)
                still.append(req)
                continue
            req.ids = list(ids)
            req.pending = len(req.ids)
            req.submitted = time.perf_counter()
            for i in req.ids:
                self.by_id[req.base][i] = req
        self.waiting = still

    def busy(self) -> bool:
        return bool(self.waiting) or any(self.by_id)

    def step(self) -> List[Request]:
        """One round: launch a block on every context with work, wait for all,
        collect stopped LPs.  Returns the requests completed in this round."""
        active = [k for k, c in enumerate(self.ctx) if self.by_id[k]]
        for k in active:
            self.ctx[k].serve_launch()
        for k in active:
            self.ctx[k].serve_wait()
        now = time.perf_counter()
        finished = []
        for k in active:
            for i in self.ctx[k].poll():
                req = self.by_id[k].pop(i, None)
                if req is None:
                    continue
                r = self.ctx[k].result(i, want_x=self.keep_results, want_y=self.keep_results)
                req.statuses[i] = r["status"]
                req.iters[i] = r["iters"]
                req.objs[i] = r["obj"]
                if self.keep_results:
                    self.results[(k, i)] = r
                self.ctx[k].release(i)
                self.lps_done += 1
                req.pending -= 1
                if req.pending == 0:
                    req.done = now
                    finished.append(req)
        self.completed.extend(finished)
        if self.waiting:
            self._admit_waiting()
        return finished

    def drain(self, max_rounds: int = 1_000_000) -> None:
        for _ in range(max_rounds):
            if not self.busy():
                return
            self.step()
        raise RuntimeError("serving loop did not drain")


def percentile(values, q) -> float:
    return float(np.percentile(np.asarray(values, dtype=np.float64), q)) if values else float("nan")
