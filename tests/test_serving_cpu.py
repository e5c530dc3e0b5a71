"""The serving loop's admission and continuous batching, on the CPU: a fake
executor runs the FP64 oracle, each batch finishing after a fixed number of
polls (so later arrivals queue behind batches in flight)."""
import numpy as np

import oracle
import siggen
from paper_1706_02740_amd.serve import Request, Server, run_trace


class FakePlan:
    def __init__(self, N, s):
        self.N, self.s = N, s
        self.op = oracle.make_plan(N, s)


class FakeExecutor:
    def __init__(self, slots=2, polls=3):
        self.slots, self.polls = slots, polls
        self.busy = [None] * slots
        self.launched = []

    def free_slot(self):
        return next((i for i, b in enumerate(self.busy) if b is None), None)

    def launch(self, batch):
        i = self.free_slot()
        self.busy[i] = [self.polls]
        self.launched.append([r.rid for r in batch])
        return (i, batch)

    def done(self, h):
        c = self.busy[h[0]]
        c[0] -= 1
        return c[0] <= 0

    def finish(self, h, batch):
        for r in batch:
            w, c = oracle.sft(r.plan.op, r.f)
            r.result = (w, c, len(w))
        self.busy[h[0]] = None


class Tick:
    """A clock that advances by one unit per reading."""
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1.0
        return self.t


def make_requests(count, nbytes):
    plans = {}
    out = []
    for i, rq in enumerate(siggen.serving_requests(0, count, rate_hz=0.5, min_log2=10, max_log2=12)):
        N, s = rq["N"], min(rq["s"], 16)
        if (N, s) not in plans:
            plans[(N, s)] = FakePlan(N, s)
        sg = siggen.sparse_signal(N, s, seed=rq["seed"], snr_db=rq["snr_db"])
        out.append(Request(rid=i, plan=plans[(N, s)], f=sg.f32, arrival=rq["t"], nbytes=nbytes))
    return out


def test_continuous_batching_results_equal_alone():
    reqs = make_requests(12, nbytes=10)
    ex = FakeExecutor(slots=2, polls=4)
    srv = Server(ex, budget_bytes=60, max_batch=4, clock=Tick())
    run_trace(srv, reqs, t0=0.0)
    assert len(srv.completed) == 12 and not srv.rejected
    assert srv.max_held <= 60 and srv.max_inflight == 2       # two batches overlapped
    assert max(len(b) for b in ex.launched) > 1               # later arrivals were batched
    assert sorted(i for b in ex.launched for i in b) == list(range(12))
    for r in srv.completed:                                   # alone == in the mix
        w, c = oracle.sft(r.plan.op, r.f)
        assert np.array_equal(np.asarray(r.result[0]), w) and np.array_equal(np.asarray(r.result[1]), c)
        assert r.done >= r.start >= r.arrival


def test_admission_by_footprint():
    reqs = make_requests(6, nbytes=25)
    reqs[2].nbytes = 1000                                     # larger than the budget: rejected
    ex = FakeExecutor(slots=2, polls=2)
    srv = Server(ex, budget_bytes=50, max_batch=8, clock=Tick())
    run_trace(srv, reqs, t0=0.0)
    assert [r.rid for r in srv.rejected] == [2] and srv.rejected[0].error
    assert len(srv.completed) == 5
    assert srv.max_held <= 50
    assert all(len(b) <= 2 for b in ex.launched)              # at most two 25-byte requests fit


def test_slot_budget_bounds_each_batch():
    """With the slots' workspaces sized up front (slot_budget = budget /
    slots), no batch holds more than one slot's bytes, and a request larger
    than a slot is rejected."""
    reqs = make_requests(8, nbytes=20)
    reqs[3].nbytes = 45                                       # fits the budget, not a slot
    ex = FakeExecutor(slots=2, polls=2)
    srv = Server(ex, budget_bytes=80, max_batch=8, clock=Tick(), slot_budget=40)
    run_trace(srv, reqs, t0=0.0)
    assert [r.rid for r in srv.rejected] == [3]
    assert len(srv.completed) == 7 and srv.max_held <= 80
    sizes = {r.rid: r.nbytes for r in reqs}
    assert all(sum(sizes[i] for i in b) <= 40 for b in ex.launched)
