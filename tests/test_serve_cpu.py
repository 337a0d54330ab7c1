"""The continuous-batching request loop (paper_2601_21990_amd/serve.py) on the
host, against a stand-in for a library context: every LP of a request is
collected once with its status, iterations and objective; a request completes
when its last LP has stopped; only contexts with work launch blocks; requests
that do not fit the free result rows wait and enter in arrival order per base;
errors other than a full context propagate; a loop that cannot drain says so."""
import numpy as np
import pytest

import paper_2601_21990_amd.pdlpb as P
from paper_2601_21990_amd.serve import Server, Request, percentile
from workloads.generators import DELTA_DTYPE


class FakeContext:
    """Holds `rows` result rows; an LP stops `blocks` launches after it was
    admitted (the number is its delta's value); ids count up from 0."""

    def __init__(self, rows=8, fail=None):
        self.rows = rows
        self.used = 0
        self.next_id = 0
        self.running = {}          # id -> launches left
        self.stopped = []
        self.launches = 0
        self.submits = []
        self.fail = fail

    def submit(self, deltas, warm, tol, max_iters):
        if self.fail is not None:
            raise P.PdlpbError(self.fail, "refused")
        if self.used + len(deltas) > self.rows:
            raise P.PdlpbError(P.ENOMEM, "result rows full")
        self.used += len(deltas)
        ids = list(range(self.next_id, self.next_id + len(deltas)))
        self.next_id += len(deltas)
        for i, d in zip(ids, deltas):
            self.running[i] = int(d["value"])
        self.submits.append((len(deltas), warm, tol, max_iters))
        return np.array(ids, dtype=np.int32)

    def serve_launch(self):
        self.launches += 1
        for i in list(self.running):
            self.running[i] -= 1
            if self.running[i] <= 0:
                del self.running[i]
                self.stopped.append(i)

    def serve_wait(self):
        pass

    def poll(self):
        out, self.stopped = self.stopped, []
        return out

    def result(self, i, want_x=False, want_y=False):
        return {"status": P.STATUS_OPTIMAL, "iters": 100 + i, "obj": -float(i)}

    def release(self, i):
        self.used -= 1


def _req(base, blocks, arrival=0.0):
    d = np.zeros(len(blocks), dtype=DELTA_DTYPE)
    d["kind"] = P.SET_LO
    d["var"] = np.arange(len(blocks))
    d["value"] = blocks
    return Request(base=base, deltas=d, arrival=arrival, tol=1e-4, max_iters=500)


def test_every_lp_is_collected_and_requests_complete_last_lp_first():
    ctx = FakeContext(rows=16)
    srv = Server([ctx], warm=True)
    a, b = _req(0, [1, 3, 2]), _req(0, [1])
    srv.submit(a)
    srv.submit(b)
    done = srv.step()                        # after one block: b's LP and a's first LP stop
    assert done == [b] and a.pending == 2
    srv.drain()
    assert srv.completed == [b, a] and not srv.busy()
    assert sorted(a.statuses) == a.ids and all(s == P.STATUS_OPTIMAL for s in a.statuses.values())
    assert a.iters == {i: 100 + i for i in a.ids} and a.objs == {i: -float(i) for i in a.ids}
    assert srv.lps_done == 4 and ctx.used == 0
    assert ctx.launches == 3                 # a's slowest LP stops after three blocks
    assert ctx.submits[0] == (3, P.WARM_BASE, 1e-4, 500)
    assert a.done >= a.submitted and a.latency >= 0.0


def test_only_contexts_with_work_launch():
    c0, c1 = FakeContext(), FakeContext()
    srv = Server([c0, c1], warm=False)
    srv.submit(_req(1, [2]))
    srv.drain()
    assert c0.launches == 0 and c1.launches == 2
    assert c1.submits[0][1] == P.WARM_NONE


def test_full_context_queues_requests_in_arrival_order_per_base():
    ctx = FakeContext(rows=4)
    srv = Server([ctx])
    big, large, small = _req(0, [2, 2, 2]), _req(0, [1, 1, 1, 1]), _req(0, [1])
    for r in (big, large, small):
        srv.submit(r)
    # big fits (3 of 4 rows); large does not, and small, behind it, waits as well
    assert srv.waiting == [large, small] and big.ids and not small.ids
    srv.step()
    assert srv.waiting == [large, small]     # big still holds its rows
    srv.step()                               # big stops and releases its rows
    assert srv.waiting == [small] and large.ids
    srv.drain()
    order = [r for r in srv.completed]
    assert order == [big, large, small]


def test_other_submit_errors_propagate():
    srv = Server([FakeContext(fail=P.EINVAL)])
    with pytest.raises(P.PdlpbError) as e:
        srv.submit(_req(0, [1]))
    assert e.value.code == P.EINVAL


def test_a_loop_that_cannot_drain_says_so():
    srv = Server([FakeContext(rows=2)])
    srv.submit(_req(0, [10 ** 6]))
    with pytest.raises(RuntimeError):
        srv.drain(max_rounds=5)


def test_percentile_of_latencies():
    assert percentile([1.0, 2.0, 3.0, 4.0], 50) == pytest.approx(2.5)
    assert np.isnan(percentile([], 99))
