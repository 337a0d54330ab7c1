"""Continuous-batching request loop over resident base LPs.

Each base LP (constraint matrix, bounds, objective and a warm start) lives in
its own library context on the GPU.  A request is a strong-branching or
bound-tightening batch on one base: a list of per-LP changes.

Admission by device-memory footprint: the loop holds one budget of device
bytes for all contexts.  Requests wait in one FIFO queue in arrival order; the
request at its head is handed to its context (pdlpb_submit) only when the
bytes every context will hold afterwards -- each context's
pdlpb_serve_footprint, which counts its matrix, its storage grown for every LP
it runs or holds queued, and for this context the request's LPs too -- fit the
budget.  When they do not, contexts with nothing to run are trimmed first
(pdlpb_serve_trim); if the head still does not fit, it and everything behind it
wait until finished requests give memory back.  The library also refuses a
request whose LPs do not fit the context's free result rows; such a request
waits at the head in the same way.

Per-context completion: every context with work has one block of C iterations
in flight on its own stream.  The loop finds the contexts whose block has
finished (pdlpb_serve_ready, which never blocks), collects their stopped LPs,
admits waiting requests and launches the next block on those contexts at once,
while the blocks of the other contexts keep running.  A request completes when
all of its LPs have stopped; its latency is completion time minus arrival time.
"""
from __future__ import annotations

import time
from collections import deque
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

    @property
    def wait(self) -> float:
        """Time spent queued before the library accepted the request."""
        return self.submitted - self.arrival


class Server:
    def __init__(self, contexts: List[P.Context], warm: bool = True, keep_results: bool = False,
                 budget_bytes: Optional[int] = None):
        self.ctx = contexts
        self.warm = warm
        self.keep_results = keep_results
        self.budget = budget_bytes
        self.fifo: deque = deque()                  # requests not yet in the library, arrival order
        self.by_id: List[Dict[int, Request]] = [dict() for _ in contexts]
        self.launched = [False] * len(contexts)
        self.results: Dict[tuple, dict] = {}
        self.completed: List[Request] = []
        self.lps_done = 0
        self.peak_bytes = 0                         # largest footprint admitted against the budget
        self.blocked_on_budget = 0                  # admissions deferred because the budget was full
        self.trims = 0

    # ---- admission ------------------------------------------------------------
    def submit(self, req: Request) -> None:
        self.fifo.append(req)
        self._admit()

    def _footprint_with(self, base: int, extra: int) -> int:
        total = 0
        for k, c in enumerate(self.ctx):
            total += c.serve_footprint(extra if k == base else 0)
        return total

    def _trim_idle(self) -> bool:
        """Shrink the storage of contexts with no block in flight; True if any
        shrank."""
        shrank = False
        for k, c in enumerate(self.ctx):
            if self.launched[k]:
                continue
            before = c.device_bytes
            c.serve_trim()
            if c.device_bytes < before:
                shrank = True
                self.trims += 1
        return shrank

    def _fits(self, req: Request) -> bool:
        if self.budget is None:
            return True
        need = self._footprint_with(req.base, len(req.deltas))
        if need > self.budget and self._trim_idle():
            need = self._footprint_with(req.base, len(req.deltas))
        if need > self.budget:
            return False
        self.peak_bytes = max(self.peak_bytes, need)
        return True

    def _admit(self) -> None:
        while self.fifo:
            req = self.fifo[0]
            if not self._fits(req):
                self.blocked_on_budget += 1
                return
            ctx = self.ctx[req.base]
            try:
                ids = ctx.submit(req.deltas, P.WARM_BASE if self.warm else P.WARM_NONE,
                                 req.tol, req.max_iters)
            except P.PdlpbError as e:
                if e.code != P.ENOMEM:
                    raise
                return                              # result rows full: wait at the head
            self.fifo.popleft()
            req.ids = list(ids)
            req.pending = len(req.ids)
            req.submitted = time.perf_counter()
            for i in req.ids:
                self.by_id[req.base][i] = req

    # ---- the loop ---------------------------------------------------------------
    def busy(self) -> bool:
        return bool(self.fifo) or any(self.by_id)

    def _launch_idle(self) -> None:
        for k, c in enumerate(self.ctx):
            if not self.launched[k] and self.by_id[k]:
                c.serve_launch()
                self.launched[k] = True

    def _collect(self, k: int, now: float) -> List[Request]:
        c = self.ctx[k]
        c.serve_wait()
        self.launched[k] = False
        finished = []
        for i in c.poll():
            req = self.by_id[k].pop(i, None)
            if req is None:
                continue
            r = c.result(i, want_x=self.keep_results, want_y=self.keep_results)
            req.statuses[i] = r["status"]
            req.iters[i] = r["iters"]
            req.objs[i] = r["obj"]
            if self.keep_results:
                self.results[(k, i)] = r
            c.release(i)
            self.lps_done += 1
            req.pending -= 1
            if req.pending == 0:
                req.done = now
                finished.append(req)
        return finished

    def step(self, poll_s: float = 20e-6) -> List[Request]:
        """Launch a block on every context that has work and none in flight,
        then wait until at least one context's block has finished; collect
        the stopped LPs of every finished context, admit waiting requests and
        relaunch those contexts.  Returns the requests completed."""
        finished = []
        # (a context whose LPs all settled at submission launches nothing and
        # is ready at once; its LPs come back through the same poll)
        self._launch_idle()
        flying = [k for k in range(len(self.ctx)) if self.launched[k]]
        if flying:
            while True:
                ready = [k for k in flying if self.ctx[k].serve_ready()]
                if ready:
                    break
                time.sleep(poll_s)
            now = time.perf_counter()
            for k in ready:
                finished += self._collect(k, now)
        self.completed.extend(finished)
        self._admit()
        self._launch_idle()
        return finished

    def drain(self, max_rounds: int = 10_000_000) -> None:
        for _ in range(max_rounds):
            if not self.busy():
                return
            self.step()
        raise RuntimeError("serving loop did not drain")


def percentile(values, q) -> float:
    return float(np.percentile(np.asarray(values, dtype=np.float64), q)) if values else float("nan")
