"""Serving scheduler against a fake executor (CPU): admission by budget and slots, oversize
rejection, FIFO order, injected launch and completion failures, queue timeouts."""
import pytest
import torch

from paper_2412_08265_amd import ops
from paper_2412_08265_amd.serve import QueueTimeout, Rejected, Request, Result, Scheduler


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Footprint = particle count; a batch finishes when the test releases it (or at once)."""

    def __init__(self, lanes=1, auto=True, fail_launch=(), fail_collect=(), refuse=()):
        self.lanes = lanes
        self.auto = auto
        self.fail_launch, self.fail_collect, self.refuse = set(fail_launch), set(fail_collect), \
            set(refuse)
        self.batches = []             # rids of every launched batch, in launch order
        self.inflight_fp = 0
        self.max_inflight_fp = 0
        self.released = set()

    def check(self, req):
        if req.rid in self.refuse:
            raise ValueError("unsupported request")

    def footprint(self, req):
        return req.n

    def launch(self, reqs):
        rids = [r.rid for r in reqs]
        if any(r in self.fail_launch for r in rids):
            raise RuntimeError(f"launch failed for batch {rids}")
        h = {"id": len(self.batches), "rids": rids, "fp": sum(r.n for r in reqs)}
        self.batches.append(rids)
        self.inflight_fp += h["fp"]
        self.max_inflight_fp = max(self.max_inflight_fp, self.inflight_fp)
        return h

    def done(self, h):
        return self.auto or h["id"] in self.released

    def collect(self, h):
        self.inflight_fp -= h["fp"]
        if any(r in self.fail_collect for r in h["rids"]):
            raise RuntimeError(f"device error in batch {h['rids']}")
        return [Result(r, torch.full((1,), float(r))) for r in h["rids"]]


def req(rid, n=10):
    obs = ops.Observation((0.0, 0.0, 0.0), 4, 4, 1.0, 5000.0, 1.0, 8)
    return Request(torch.zeros((9, n)), obs, rid)


def test_results_reach_their_own_future_in_fifo_batches():
    ex = FakeExecutor(lanes=1, auto=False)
    s = Scheduler(ex, budget_bytes=10_000, max_slots=3)
    futs = [s.submit(req(i)) for i in range(8)]
    s.poll()                                   # first batch: head of the queue, 3 slots
    assert ex.batches == [[0, 1, 2]]
    s.poll()                                   # lane busy: nothing else launches
    assert len(ex.batches) == 1
    while s.busy():
        ex.released.add(len(ex.batches) - 1)
        s.poll()
    assert ex.batches == [[0, 1, 2], [3, 4, 5], [6, 7]]
    for i, f in enumerate(futs):
        r = f.result(timeout=0)
        assert r.rid == i and float(r.cube[0]) == i


def test_budget_bounds_memory_in_flight():
    ex = FakeExecutor(lanes=4, auto=False)
    s = Scheduler(ex, budget_bytes=100, max_slots=8)
    futs = [s.submit(req(i, n=40)) for i in range(6)]
    s.poll()
    assert ex.batches == [[0, 1]]              # a third request would exceed the budget
    assert s.used == 80
    while s.busy():
        ex.released.update(range(len(ex.batches)))
        s.poll()
        assert s.used <= 100 and ex.inflight_fp <= 100
    assert ex.max_inflight_fp <= 100 and s.peak_used == 80
    assert all(f.result(timeout=0).rid == i for i, f in enumerate(futs))


def test_head_of_queue_is_not_overtaken():
    ex = FakeExecutor(lanes=2, auto=False)
    s = Scheduler(ex, budget_bytes=100, max_slots=8)
    s.submit(req(0, n=70))
    s.poll()
    s.submit(req(1, n=60))                     # does not fit beside request 0
    s.submit(req(2, n=10))                     # would fit, but must not pass request 1
    s.poll()
    assert ex.batches == [[0]]
    ex.released.add(0)
    s.poll()
    assert ex.batches == [[0], [1, 2]]


def test_oversize_and_unsupported_requests_are_rejected_at_submit():
    ex = FakeExecutor(refuse={3})
    s = Scheduler(ex, budget_bytes=50)
    big = s.submit(req(1, n=51))
    bad = s.submit(req(3, n=5))
    ok = s.submit(req(2, n=50))
    assert isinstance(big.exception(timeout=0), Rejected)
    assert isinstance(bad.exception(timeout=0), Rejected)
    s.drain()
    assert ok.result(timeout=0).rid == 2
    assert ex.batches == [[2]]


@pytest.mark.parametrize("where", ["launch", "collect"])
def test_failed_batch_is_rerun_one_request_at_a_time(where):
    kw = {"fail_launch": {2}} if where == "launch" else {"fail_collect": {2}}
    ex = FakeExecutor(lanes=1, **kw)
    s = Scheduler(ex, budget_bytes=10_000, max_slots=4)
    futs = [s.submit(req(i)) for i in range(6)]
    s.drain()
    for i, f in enumerate(futs):
        if i == 2:
            assert isinstance(f.exception(timeout=0), RuntimeError)
        else:
            assert f.result(timeout=0).rid == i
    # the failing batch [0..3] was split into solo runs, then the rest batched again
    solo = [[0], [1], [2], [3]] if where == "collect" else [[0], [1], [3]]
    first = [[0, 1, 2, 3]] if where == "collect" else []
    assert ex.batches == first + solo + [[4, 5]]
    assert s.used == 0 and not s.busy()


def test_queue_timeout_expires_waiting_requests_only():
    clk = Clock()
    ex = FakeExecutor(lanes=1, auto=False)
    s = Scheduler(ex, budget_bytes=10_000, max_slots=1, queue_timeout_s=1.0, clock=clk)
    f0 = s.submit(req(0))
    s.poll()                                   # request 0 runs (and never times out)
    f1 = s.submit(req(1))
    clk.t = 0.5
    f2 = s.submit(req(2))
    clk.t = 1.2                                # request 1 waited 1.2 s, request 2 0.7 s
    s.poll()
    assert isinstance(f1.exception(timeout=0), QueueTimeout)
    assert not f2.done() and not f0.done()
    ex.released.add(0)
    s.poll()
    ex.released.add(1)
    s.poll()
    assert f0.result(timeout=0).rid == 0 and f2.result(timeout=0).rid == 2


def test_max_slots_validation():
    with pytest.raises(ValueError):
        Scheduler(FakeExecutor(), budget_bytes=1, max_slots=0)
