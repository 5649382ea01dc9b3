"""Host logic of the serving form (admission by footprint, continuous batching),
driven with stand-in contexts so that it runs without a GPU."""
import numpy as np
import pytest

from paper_1503_08462_amd.serving import Server


class FakeCtx:
    """Converges after `need` corrections; records its life cycle."""
    log = []

    def __init__(self, p, opts):
        self.q, self.need, self.fp, self.name = p["q"], p["need"], p["fp"], p["name"]
        self.steps = 0
        self.bound = self.closed = False

    def footprint(self):
        return self.fp

    def bind(self, stream=None):
        self.bound = True
        self.stream = stream
        FakeCtx.log.append(("bind", self.name))

    def init(self, mode):
        assert self.bound

    def correct(self, steps):
        self.steps = min(self.need, self.steps + steps)

    def progress(self):
        return {"theta": np.arange(1.0, self.q + 3), "rho": np.zeros(self.q + 2), "steps": self.steps,
                "converged": self.steps >= self.need}

    def close(self):
        self.closed = True
        FakeCtx.log.append(("close", self.name))


def make_server(budget, **kw):
    tick = iter(range(10 ** 6))
    batches = []

    def batch(cs, steps):
        batches.append([c.name for c in cs])
        for c in cs:
            c.correct(steps)
    srv = Server(budget, context_factory=FakeCtx, batch_fn=batch, stream_factory=lambda: object(),
                 clock=lambda: float(next(tick)), **kw)
    return srv, batches


def prob(name, fp, need, q=2):
    return {"name": name, "fp": fp, "need": need, "q": q}


def test_admission_respects_budget_and_arrival_order():
    FakeCtx.log = []
    srv, batches = make_server(100, steps_per_round=1)
    for name, fp, need in [("a", 60, 3), ("b", 50, 1), ("c", 30, 2), ("d", 40, 1)]:
        srv.submit(prob(name, fp, need))
    res = srv.run()
    assert sorted(res) == [0, 1, 2, 3]
    # b cannot join a (60 + 50 > 100); c and d wait behind b (first come, first served)
    assert batches[0] == ["a"]
    assert all(r["converged"] for r in res.values())
    assert srv.peak_in_use <= 100 and srv.in_use == 0
    binds = [n for k, n in FakeCtx.log if k == "bind"]
    assert binds == ["a", "b", "c", "d"]


def test_requests_join_and_leave_at_round_boundaries():
    FakeCtx.log = []
    srv, batches = make_server(100, steps_per_round=2)
    srv.submit(prob("long", 50, 8))
    srv.submit(prob("short", 40, 2))
    srv.submit(prob("late", 40, 2))  # fits once "short" has left
    srv.run()
    assert batches[0] == ["long", "short"]
    assert batches[1] == ["long", "late"]  # joined while "long" keeps running
    assert srv.finished[0].result["steps"] == 8
    lat = srv.latency()
    assert lat["count"] == 3 and lat["p50_s"] <= lat["p99_s"]


def test_oversized_request_is_rejected_and_closed():
    srv, _ = make_server(10)
    with pytest.raises(ValueError):
        srv.submit(prob("huge", 11, 1))
    assert srv.queue == []


def test_step_limit_ends_a_request_unconverged():
    srv, _ = make_server(100, steps_per_round=3)
    rid = srv.submit(prob("slow", 10, 100), max_steps=6)
    res = srv.run()
    assert res[rid]["steps"] == 6 and not res[rid]["converged"]
    assert res[rid]["lam"].shape == (2,)


def test_active_limit_caps_concurrency_and_keeps_order():
    FakeCtx.log = []
    srv, batches = make_server(1000, steps_per_round=1, max_active=2)
    for name, need in [("a", 3), ("b", 1), ("c", 2), ("d", 1)]:
        srv.submit(prob(name, 10, need))
    res = srv.run()
    assert all(len(b) <= 2 for b in batches)
    assert batches[0] == ["a", "b"]
    assert batches[1] == ["a", "c"]  # c joins when b leaves
    binds = [n for k, n in FakeCtx.log if k == "bind"]
    assert binds == ["a", "b", "c", "d"]
    assert all(r["converged"] for r in res.values())


def test_requests_admitted_in_one_round_start_together():
    """A custom start hook receives, once per round, the requests admitted in
    that round (already bound), before their first corrections."""
    starts = []

    def init_fn(cs):
        assert all(c.bound for c in cs)
        starts.append([c.name for c in cs])
    srv, batches = make_server(60, steps_per_round=1, init_fn=init_fn)
    for name, fp, need in (("a", 20, 3), ("b", 20, 1), ("c", 20, 1), ("d", 30, 1)):
        srv.submit(prob(name, fp, need))
    srv.run()
    assert starts[0] == ["a", "b", "c"]  # d does not fit until b and c leave
    assert starts[1] == ["d"]
    assert batches[0] == ["a", "b", "c"]


class WideningCtx(FakeCtx):
    """Stalls until its block is widened once: the first progress report after
    `stall` corrections says the width was raised and the footprint doubled
    (the context unbound, its iterate gone); after the next bind and start it
    converges after `need` corrections."""

    def __init__(self, p, opts):
        super().__init__(p, opts)
        self.stall, self.wide, self.inits = p.get("stall", 10 ** 9), False, 0

    def init(self, mode):
        assert self.bound
        self.inits += 1
        self.steps = 0

    def correct(self, steps):
        self.steps += steps

    def progress(self):
        pr = super().progress()
        if not self.wide and self.stall < 10 ** 9:
            pr["converged"] = False
            if self.steps >= self.stall:
                self.wide, self.bound, self.fp = True, False, 2 * self.fp
                pr["widened"], pr["bound"] = True, False
        return pr


def test_widened_request_goes_back_to_the_head_of_the_queue():
    tick = iter(range(10 ** 6))
    srv = Server(100, context_factory=WideningCtx, batch_fn=lambda cs, n: [c.correct(n) for c in cs],
                 stream_factory=lambda: object(), clock=lambda: float(next(tick)), steps_per_round=2)
    a = srv.submit(dict(prob("a", 30, need=4), stall=4))
    b = srv.submit(prob("b", 60, need=20), max_steps=100)
    srv.round()  # both admitted (90 of 100)
    assert srv.in_use == 90 and len(srv.active) == 2
    srv.round()  # a widens: releases 30 and waits at the head of the queue with 60
    assert [r.id for r in srv.queue] == [a] and srv.queue[0].footprint == 60 and srv.in_use == 60
    res = srv.run()
    assert res[a]["converged"] and res[a]["widened"] == 1 and res[b]["converged"]
    assert srv.finished[a].ctx.inits == 2 and srv.peak_in_use <= 100


def test_widened_request_beyond_the_budget_finishes_unconverged():
    tick = iter(range(10 ** 6))
    srv = Server(100, context_factory=WideningCtx, batch_fn=lambda cs, n: [c.correct(n) for c in cs],
                 stream_factory=lambda: object(), clock=lambda: float(next(tick)), steps_per_round=2)
    a = srv.submit(dict(prob("a", 70, need=4), stall=2))
    res = srv.run()
    assert not res[a]["converged"] and res[a]["widened"] == 1 and srv.in_use == 0


def test_async_admission_finishes_every_request_within_budget():
    """Binding and starting admitted requests on the worker thread: every
    request still finishes converged, the budget holds, no request runs a
    round before it is bound, and streams go back to a free list for reuse."""
    FakeCtx.log = []
    srv, batches = make_server(100, steps_per_round=2, async_admit=True)
    needs = [3, 5, 2, 7, 4, 6, 1, 8]
    for k, need in enumerate(needs):
        srv.submit(prob("r%d" % k, 30 + 5 * (k % 3), need))
    while srv.round():
        assert srv.in_use <= 100
        for names in batches[-1:]:
            for n in names:
                assert ("bind", n) in FakeCtx.log
    srv.close()
    res = srv.results()
    assert len(res) == len(needs) and all(r["converged"] for r in res.values())
    assert srv.peak_in_use <= 100
    assert not srv.binding and not srv.active and not srv.queue
    assert len(srv._free_streams) >= 1
