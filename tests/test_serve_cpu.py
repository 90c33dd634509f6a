"""Scheduler logic of the continuous-batching server, on the CPU with a
simulated engine (memory budget, device time proportional to the work)."""
import numpy as np

from paper_2212_11878_amd import inputs
from paper_2212_11878_amd.serve import Server


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


class SimEngine:
    """Bookkeeping twin of the library: budget in bytes (64 B per particle),
    slots, per-box step counters; a step costs particles / rate seconds."""

    def __init__(self, clock, budget_bytes, rate=5e10, max_slots=64):
        self.clock, self.budget, self.rate, self.max_slots = clock, budget_bytes, rate, max_slots
        self.used = 0
        self.boxes = {}
        self.admitted = []

    def admit(self, req):
        need = 64 * req["n"]
        if self.used + need > self.budget or len(self.boxes) >= self.max_slots:
            return None
        slot = min(set(range(self.max_slots)) - set(self.boxes))
        self.boxes[slot] = dict(req=req, step=0)
        self.used += need
        self.admitted.append(req["seed"])
        return slot

    def step(self, n):
        work = 0
        for b in self.boxes.values():
            k = min(n, b["req"]["steps"] - b["step"])
            b["step"] += k
            work += k * b["req"]["n"]
        self.clock.t += work / self.rate

    def observe(self, slot):
        b = self.boxes[slot]
        return dict(step=b["step"], T=1.0, vacf=np.ones(3), status=0)

    def release(self, slot):
        self.used -= 64 * self.boxes.pop(slot)["req"]["n"]
        assert self.used >= 0


def test_every_request_completes_with_its_step_count():
    clock = SimClock()
    reqs = inputs.served_requests(rate_hz=20, window_s=5, seed=5)
    eng = SimEngine(clock, budget_bytes=4 << 30)
    summary, done = Server(eng, chunk_steps=50, clock=clock, sleep=clock.sleep).run(reqs)
    assert summary["completed"] == len(reqs) == summary["offered"]
    assert summary["unfinished"] == 0
    for d in done:
        assert d["step"] == d["req"]["steps"]
        assert d["latency"] >= d["queued"] >= 0
    assert eng.used == 0 and not eng.boxes


def test_budget_limits_concurrency_and_queues_the_rest():
    clock = SimClock()
    reqs = inputs.served_requests(rate_hz=200, window_s=1, seed=7)
    big = max(r["n"] for r in reqs)
    eng = SimEngine(clock, budget_bytes=64 * big * 3)
    summary, done = Server(eng, chunk_steps=100, clock=clock, sleep=clock.sleep).run(reqs)
    assert summary["completed"] == len(reqs)
    assert summary["max_live"] <= 3 * big / min(r["n"] for r in reqs) + 1
    # first come, first served: admission order is arrival order
    arrival_order = [r["seed"] for r in sorted(reqs, key=lambda r: r["arrival"])]
    assert eng.admitted == arrival_order
    # queueing shows up in the latency tail
    assert summary["p99_latency_s"] >= summary["p50_latency_s"] > 0


def test_overload_is_reported_not_hidden():
    """Offered work above the engine's rate: the wall clock stops the run and
    the unfinished requests are counted."""
    clock = SimClock()
    reqs = inputs.served_requests(rate_hz=200, window_s=2, seed=9)
    eng = SimEngine(clock, budget_bytes=1 << 34, rate=1e10)
    summary, done = Server(eng, chunk_steps=50, clock=clock, sleep=clock.sleep).run(reqs, max_wall_s=3.0)
    assert summary["unfinished"] > 0
    assert summary["completed"] + summary["unfinished"] + summary["rejected"] == summary["offered"]


def test_request_larger_than_the_budget_is_rejected():
    """A request that cannot fit even an empty engine is rejected at once;
    the others are still served and the server terminates."""
    clock = SimClock()
    reqs = inputs.served_requests(rate_hz=50, window_s=1, seed=11)
    reqs[len(reqs) // 2]["n"] = 10 ** 9           # 64 GB at 64 B per particle
    eng = SimEngine(clock, budget_bytes=1 << 30)
    summary, done = Server(eng, chunk_steps=50, clock=clock, sleep=clock.sleep).run(reqs)
    assert summary["rejected"] == 1
    assert summary["completed"] == len(reqs) - 1 and summary["unfinished"] == 0
    assert all(d["req"]["n"] != 10 ** 9 for d in done)
