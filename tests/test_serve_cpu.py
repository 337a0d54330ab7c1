"""The continuous-batching request loop (paper_2601_21990_amd/serve.py) on the
host, against a stand-in for a library context: every LP of a request is
collected once with its status, iterations and objective; a request completes
when its last LP has stopped; only contexts with work launch blocks; requests
wait in one arrival-order queue while their LPs do not fit the free result rows
or the device-memory budget; a context whose block is still running does not
hold up the others; errors other than a full context propagate; a loop that
cannot drain says so."""
import numpy as np
import pytest

import paper_2601_21990_amd.pdlpb as P
from paper_2601_21990_amd.serve import Server, Request, percentile
from workloads.generators import DELTA_DTYPE


class FakeContext:
    """Holds `rows` result rows; an LP stops `blocks` launches after it was
    admitted (the number is its delta's value); ids count up from 0."""

    def __init__(self, rows=8, fail=None, base_bytes=1000, lp_bytes=100, slow=0):
        self.rows = rows
        self.base_bytes = base_bytes
        self.lp_bytes = lp_bytes
        self.slow = slow           # polls a launched block stays unfinished
        self.busy_polls = 0
        self.trims = 0
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

        self.busy_polls = self.slow

    def serve_ready(self):
        if self.busy_polls > 0:
            self.busy_polls -= 1
            return False
        return True

    def serve_wait(self):
        pass

    def serve_footprint(self, extra=0):
        return self.base_bytes + self.lp_bytes * (self.used + extra)

    def serve_trim(self):
        self.trims += 1

    @property
    def device_bytes(self):
        return self.serve_footprint(0)

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


def test_full_context_queues_requests_in_arrival_order():
    ctx = FakeContext(rows=4)
    srv = Server([ctx])
    big, large, small = _req(0, [2, 2, 2]), _req(0, [1, 1, 1, 1]), _req(0, [1])
    for r in (big, large, small):
        srv.submit(r)
    # big fits (3 of 4 rows); large does not, and small, behind it, waits as well
    assert list(srv.fifo) == [large, small] and big.ids and not small.ids
    srv.step()
    assert list(srv.fifo) == [large, small]  # big still holds its rows
    srv.step()                               # big stops and releases its rows
    assert list(srv.fifo) == [small] and large.ids
    srv.drain()
    order = [r for r in srv.completed]
    assert order == [big, large, small]


def test_admission_by_device_memory_budget_across_bases():
    """Two contexts of 1000 bytes each and 100 bytes per LP under a budget of
    2500 bytes: a 4-LP request (footprint 2400 with both bases) is admitted;
    a 2-LP request on the other base would need 2600, so it waits, although its
    base is idle, until the first request's LPs are released."""
    c0, c1 = FakeContext(rows=8), FakeContext(rows=8)
    srv = Server([c0, c1], budget_bytes=2500)
    a, b = _req(0, [2, 2, 2, 2]), _req(1, [1, 1])
    srv.submit(a)
    srv.submit(b)
    assert a.ids and not b.ids and list(srv.fifo) == [b]
    assert srv.blocked_on_budget >= 1 and c1.trims >= 1     # idle contexts were trimmed first
    srv.step()
    assert not b.ids                                        # a still runs
    srv.step()                                              # a's LPs stop and are released
    assert b.ids and not srv.fifo
    srv.drain()
    assert srv.completed == [a, b]
    assert srv.peak_bytes <= 2500
    assert b.wait > 0.0 and a.wait >= 0.0


def test_a_running_block_does_not_hold_up_other_contexts():
    """Context 0's block stays unfinished for many polls; context 1's requests
    complete and new ones are admitted and launched meanwhile."""
    slow, fast = FakeContext(slow=10 ** 9), FakeContext()
    srv = Server([slow, fast])
    s0 = _req(0, [1])
    srv.submit(s0)
    done = []
    for k in range(3):
        r = _req(1, [1])
        srv.submit(r)
        done += srv.step(poll_s=0.0)
    assert len(done) == 3 and all(r.base == 1 for r in done)
    assert slow.launches == 1 and fast.launches == 3 and not s0.done
    slow.busy_polls = 0
    slow.slow = 0
    srv.drain()
    assert s0.done is not None


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
