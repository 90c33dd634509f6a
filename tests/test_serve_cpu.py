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


def _by_seed(done):
    return {d["req"]["seed"]: d for d in done}


def test_cancel_live_request_releases_its_box_and_spares_the_rest():
    """A request cancelled while its box is live is released at once (its
    memory returns to the budget) after fewer than its steps; every other
    request still completes with its full step count."""
    clock = SimClock()
    reqs = inputs.served_requests(rate_hz=20, window_s=2, seed=13)
    eng = SimEngine(clock, budget_bytes=4 << 30)
    victim = reqs[3]
    srv = Server(eng, chunk_steps=50, clock=clock, sleep=clock.sleep)

    steps_seen = []
    real_step = eng.step

    def step(n):   # cancel once the victim's box has run a few chunks
        real_step(n)
        live = [b for b in eng.boxes.values() if b["req"]["seed"] == victim["seed"]]
        if live:
            steps_seen.append(live[0]["step"])
            if live[0]["step"] >= 100:
                srv.cancel(victim["seed"])
    eng.step = step
    summary, done = srv.run(reqs)
    got = _by_seed(done)
    assert summary["cancelled"] == 1 and summary["completed"] == len(reqs) - 1
    assert summary["completed"] + summary["cancelled"] + summary["rejected"] + summary["unfinished"] == len(reqs)
    c = got[victim["seed"]]
    assert c["status"] == "cancelled" and 100 <= c["step"] < victim["steps"]
    assert max(steps_seen) < victim["steps"]
    for r in reqs:
        if r is not victim:
            assert got[r["seed"]]["status"] == 0 and got[r["seed"]]["step"] == r["steps"]
    assert eng.used == 0 and not eng.boxes


def test_cancel_queued_and_not_yet_arrived_requests():
    """Cancelled while queued behind the budget, or before it arrives, a
    request is never admitted."""
    clock = SimClock()
    reqs = inputs.served_requests(rate_hz=200, window_s=0.5, seed=17)
    big = max(r["n"] for r in reqs)
    eng = SimEngine(clock, budget_bytes=64 * big)        # room for one box at a time
    queued, future = reqs[2], reqs[-1]
    queued["cancel_at"] = queued["arrival"] + 1e-6
    srv = Server(eng, chunk_steps=50, clock=clock, sleep=clock.sleep)
    srv.cancel(future["seed"])                            # before run(): applies when reached
    summary, done = srv.run(reqs)
    got = _by_seed(done)
    assert summary["cancelled"] == 2 and summary["completed"] == len(reqs) - 2
    for r in (queued, future):
        assert got[r["seed"]]["status"] == "cancelled" and got[r["seed"]]["step"] == 0
        assert r["seed"] not in eng.admitted
    assert eng.used == 0


def test_cancel_of_unknown_or_finished_request_is_ignored():
    clock = SimClock()
    reqs = inputs.served_requests(rate_hz=20, window_s=1, seed=19)
    eng = SimEngine(clock, budget_bytes=4 << 30)
    srv = Server(eng, chunk_steps=50, clock=clock, sleep=clock.sleep)
    srv.cancel(-12345)
    summary, done = srv.run(reqs)
    assert summary["cancelled"] == 0 and summary["completed"] == len(reqs)
    assert not srv._cancel


def test_cancel_from_another_thread():
    """Server.cancel called from a second thread while run() serves on the
    real clock."""
    import threading
    import time

    class SlowEngine(SimEngine):
        def step(self, n):
            super().step(n)
            time.sleep(0.002)

    clock = SimClock()
    reqs = inputs.served_requests(rate_hz=50, window_s=0.1, seed=23, steps=(2000, 2000))
    for r in reqs:
        r["arrival"] = 0.0
    eng = SlowEngine(clock, budget_bytes=4 << 30)
    srv = Server(eng, chunk_steps=10)
    t = threading.Timer(0.02, srv.cancel, args=(reqs[0]["seed"],))
    t.start()
    summary, done = srv.run(reqs)
    t.join()
    got = _by_seed(done)[reqs[0]["seed"]]
    assert got["status"] == "cancelled" and 0 < got["step"] < 2000
    assert summary["completed"] == len(reqs) - 1


def test_one_at_a_time_server():
    """max_live=1 serves the same requests one box at a time, in arrival
    order, with the same per-request step counts."""
    clock = SimClock()
    reqs = inputs.served_requests(rate_hz=50, window_s=1, seed=29)
    eng = SimEngine(clock, budget_bytes=4 << 30)
    summary, done = Server(eng, chunk_steps=50, clock=clock, sleep=clock.sleep, max_live=1).run(reqs)
    assert summary["max_live"] == 1 and summary["completed"] == len(reqs)
    assert eng.admitted == [r["seed"] for r in sorted(reqs, key=lambda r: r["arrival"])]
    assert all(d["step"] == d["req"]["steps"] for d in done)
