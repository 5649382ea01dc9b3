"""Serving form of the solver: many eigenproblems of uneven size on one GPU.

Requests are set up on the host when they are submitted (the AMG hierarchy,
Section 2), admitted to the device in arrival order while their device
footprint fits the memory budget, and then advanced together: every
scheduling round enqueues a few correction steps (Algorithm 3.1) for each
active request on its own stream from a small pool, so the streaming kernels
of different requests overlap on the device, and by default solves the small
eigenproblems (3.3) of all of them in shared launches.  Requests join at a
round boundary (after their Algorithm 3.2 start) and leave as soon as their
convergence test holds or their step limit is reached, which frees their
memory for the next arrivals (continuous batching).  A request whose block
the library widens (its block ended inside a cluster of eigenvalues) goes back
to the head of the queue with its larger footprint.  Latency is measured from
submission (or the given arrival time) to completion.

The scheduler only orders host calls into the library; every step of a solve
runs in the library's kernels.
"""
import concurrent.futures as _cf
import time

import numpy as np

from . import INIT_NESTED, Context, correct_batch_joint, defaults


def _default_init(contexts):
    for c in contexts:
        c.init(INIT_NESTED)


class Request:
    __slots__ = ("id", "ctx", "q", "tol", "max_steps", "footprint", "arrival", "admitted", "done", "stream",
                 "result", "widened")

    def __init__(self, rid, ctx, q, tol, max_steps, arrival):
        self.id, self.ctx, self.q, self.tol, self.max_steps = rid, ctx, q, tol, max_steps
        self.footprint = ctx.footprint()
        self.arrival = arrival
        self.admitted = self.done = None
        self.stream = None
        self.result = None
        self.widened = 0


class Server:
    """Admission by footprint, continuous batching at step boundaries.

    budget_bytes:     device memory the admitted requests may hold together
    n_streams:        stream pool; request k of a round uses stream k mod n_streams
    max_active:       at most this many requests on the device at once (None: only
                      the budget limits admission); fewer concurrent requests
                      finish sooner each, which lowers the latency percentiles
    steps_per_round:  corrections enqueued per request between convergence checks
    context_factory:  (problem dict, opts) -> context; the default builds a
                      library Context (tests pass stand-ins)
    batch_fn:         (contexts, steps) -> None; the default is
                      correct_batch_joint (each context on its own stream, the
                      small eigenproblems of all of them in shared launches)
    init_fn:          (contexts) -> None, the nested start of the requests
                      admitted in one round; the default is each context's own
                      init on its stream (init_batch_joint, which solves the
                      small problems of the starts together, holds the new
                      requests in step with each other and measured slower)
    keep_contexts:    a finished request gives back its device workspace but
                      its context stays open (the caller may submit it again,
                      e.g. for another measured pass over the same requests)
    async_admit:      bind and start admitted requests on worker threads
                      (workspace, upload of the hierarchy, Algorithm 3.2 start)
                      while this thread keeps enqueueing the active requests'
                      rounds; each admitted request then gets a stream of its
                      own (a bind waits for its stream).  A request joins the
                      rounds once its start is enqueued.
    admit_workers:    worker threads of the asynchronous admission
    """

    def __init__(self, budget_bytes, n_streams=4, steps_per_round=2, opts=None, context_factory=None,
                 batch_fn=None, stream_factory=None, clock=time.perf_counter, max_active=None, init_fn=None,
                 keep_contexts=False, async_admit=False, admit_workers=8):
        if budget_bytes <= 0 or n_streams < 1 or steps_per_round < 1 or (max_active is not None and max_active < 1):
            raise ValueError("budget, stream count, steps per round and active limit must be positive")
        self.max_active = max_active
        self.keep_contexts = keep_contexts
        self.budget = int(budget_bytes)
        self.steps_per_round = int(steps_per_round)
        self.opts = opts
        self.clock = clock
        self._make = context_factory or (lambda p, o: Context(p["rowptr"], p["col"], p["A"], p["M"], p["q"], o))
        self._batch = batch_fn or (lambda cs, steps: correct_batch_joint(cs, steps))
        self._init = init_fn or _default_init
        if stream_factory is None:
            def stream_factory():
                import torch
                return torch.cuda.Stream()  # default priority
        self._stream_factory = stream_factory
        self.streams = [stream_factory() for _ in range(n_streams)]
        self.async_admit = bool(async_admit) and init_fn is None
        self._binder = _cf.ThreadPoolExecutor(max_workers=max(1, int(admit_workers))) if self.async_admit else None
        self._free_streams = []  # per-request streams of the asynchronous admission, for reuse
        self.binding = []        # (request, future) being bound and started
        self.queue = []       # submitted, waiting for memory, in arrival order
        self.active = []      # on the device
        self.finished = {}    # id -> Request
        self.in_use = 0       # bytes held by active requests
        self.peak_in_use = 0
        self.rounds = 0
        # host seconds spent admitting (bind, upload, start), enqueueing the
        # rounds' steps, and waiting for and reading the progress reports
        self.host_s = {"admit": 0.0, "enqueue": 0.0, "retire": 0.0}
        self._next_id = 0
        self._next_stream = 0

    # ------------------------------------------------------------- requests
    def submit(self, problem, tol=1e-8, max_steps=200, opts=None, arrival=None):
        """Host setup now; returns the request id.  A request larger than the
        whole budget is rejected (ValueError) rather than queued forever."""
        base = opts if opts is not None else (self.opts if self.opts is not None else defaults())
        o = type(base).from_buffer_copy(base) if hasattr(type(base), "from_buffer_copy") else base
        if hasattr(o, "tol"):
            o.tol = tol  # the device-side convergence test of each step
        ctx = self._make(problem, o)
        rid = self._next_id
        self._next_id += 1
        req = Request(rid, ctx, int(problem["q"]), tol, max_steps, self.clock() if arrival is None else arrival)
        if req.footprint > self.budget:
            ctx.close()
            raise ValueError("request %d needs %d bytes, more than the budget of %d" % (rid, req.footprint,
                                                                                        self.budget))
        self.queue.append(req)
        return rid

    def _bind_start(self, req):
        req.ctx.bind(stream=req.stream)
        self._init([req.ctx])

    def _admit_async(self):
        ready = [b for b in self.binding if b[1].done()]
        if not self.active and self.binding and not ready:
            ready = [self.binding[0]]  # nothing to run meanwhile: wait for the oldest
        for req, fut in ready:
            fut.result()
            req.admitted = self.clock()
            self.active.append(req)
        self.binding = [b for b in self.binding if b not in ready]
        while (self.queue and self.in_use + self.queue[0].footprint <= self.budget
               and (self.max_active is None or len(self.active) + len(self.binding) < self.max_active)):
            req = self.queue.pop(0)
            req.stream = self._free_streams.pop() if self._free_streams else self._stream_factory()
            self.in_use += req.footprint
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            self.binding.append((req, self._binder.submit(self._bind_start, req)))

    def _release_stream(self, req):
        if self.async_admit and req.stream is not None:
            self._free_streams.append(req.stream)
        req.stream = None

    def _admit(self):
        if self.async_admit:
            self._admit_async()
            return
        new = []
        while (self.queue and self.in_use + self.queue[0].footprint <= self.budget
               and (self.max_active is None or len(self.active) + len(new) < self.max_active)):
            req = self.queue.pop(0)
            req.stream = self.streams[self._next_stream % len(self.streams)]
            self._next_stream += 1
            req.ctx.bind(stream=req.stream)
            self.in_use += req.footprint
            self.peak_in_use = max(self.peak_in_use, self.in_use)
            new.append(req)
        if new:
            self._init([r.ctx for r in new])
            now = self.clock()
            for req in new:
                req.admitted = now
            self.active.extend(new)

    def _retire(self):
        still, again = [], []
        for req in self.active:
            pr = req.ctx.progress()
            if pr.get("widened"):
                # the library raised the block width (the block ended inside a
                # cluster): the iterate is gone; start again in place, or wait
                # for memory at the head of the queue with the larger footprint
                if pr.get("bound"):
                    self._init([req.ctx])
                    still.append(req)
                else:
                    self.in_use -= req.footprint
                    if hasattr(req.ctx, "workspace"):
                        req.ctx.workspace = None
                    self._release_stream(req)
                    req.footprint = req.ctx.footprint()
                    req.widened += 1
                    if req.footprint <= self.budget:
                        again.append(req)
                        continue
                    # the wider block can never be admitted: finish unconverged
                    req.done = self.clock()
                    req.result = {"lam": np.asarray(pr["theta"][:req.q]).copy(),
                                  "rho": np.asarray(pr["rho"][:req.q]).copy(), "steps": pr["steps"],
                                  "converged": False, "latency_s": req.done - req.arrival,
                                  "widened": req.widened}
                    req.ctx.close()
                    self.finished[req.id] = req
                continue
            if pr["converged"] or pr["steps"] >= req.max_steps:
                req.done = self.clock()
                req.result = {"lam": np.asarray(pr["theta"][:req.q]).copy(), "rho": np.asarray(pr["rho"][:req.q]).copy(),
                              "steps": pr["steps"], "converged": bool(pr["converged"]),
                              "latency_s": req.done - req.arrival, "widened": req.widened}
                if not self.keep_contexts:
                    req.ctx.close()
                if hasattr(req.ctx, "workspace"):
                    req.ctx.workspace = None  # back to the allocator for the next admissions
                self._release_stream(req)
                self.in_use -= req.footprint
                self.finished[req.id] = req
            else:
                still.append(req)
        self.active = still
        self.queue[:0] = again

    def round(self):
        """One scheduling round; returns the number of requests still pending."""
        t0 = self.clock()
        self._admit()
        t1 = self.clock()
        self.host_s["admit"] += t1 - t0
        if not self.active and self.queue and not self.binding:  # cannot happen while every request fits the budget
            raise RuntimeError("no request can be admitted")
        if self.active:
            self._batch([r.ctx for r in self.active], self.steps_per_round)
            self.rounds += 1
            t2 = self.clock()
            self.host_s["enqueue"] += t2 - t1
            self._retire()
            self.host_s["retire"] += self.clock() - t2
        return len(self.queue) + len(self.active) + len(self.binding)

    def run(self):
        while self.round():
            pass
        return self.results()

    def close(self):
        """Stop the admission worker (asynchronous admission)."""
        if self._binder is not None:
            self._binder.shutdown(wait=True)
            self._binder = None

    # -------------------------------------------------------------- reports
    def results(self):
        return {rid: r.result for rid, r in sorted(self.finished.items())}

    def latency(self):
        lat = np.array([r.result["latency_s"] for r in self.finished.values()])
        if lat.size == 0:
            return {"p50_s": None, "p99_s": None, "count": 0}
        return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)), "count": int(lat.size)}
