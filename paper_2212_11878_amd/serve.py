"""Continuous-batching server for ensembles of SRD boxes.

Requests (one periodic box each: edge, density, dt, alpha, steps, seed)
arrive over time.  The server admits a request as soon as the device-memory
budget and a slot allow it, keeps every admitted box resident on the GPU, and
advances all of them together: each mpcd_step call is one batched launch
sequence over every live box, so new arrivals join the running batch while
others are mid-flight.  Each round queues one chunk of steps (the call
returns at once), admits arrivals while the chunk runs, then observes
(temperature and velocity autocorrelation) and releases the boxes that
reached their step count, freeing memory for the queue; a box that finishes
inside a chunk idles on the device until then.  Latency is completion time
minus arrival time.

A request can be cancelled at any point (`Server.cancel`, from any thread,
or a `cancel_at` time in the request): not yet arrived or still queued, it is
dropped; live, its box is released at once, with steps of it still queued on
the device (the library frees its memory in stream order), and the other
boxes go on unchanged.  With `max_live=1` the same server runs the requests
one at a time, the baseline that batching is measured against.

The scheduler talks to an engine with four calls (admit / step / observe /
release).  `LibraryEngine` drives libmpcd through its C ABI; tests can plug
in another engine to exercise queueing and admission without a GPU.
"""
import collections
import math
import threading
import time

import numpy as np


class LibraryEngine:
    """Engine backed by libmpcd (one context, torch memory and stream)."""

    def __init__(self, hbm_budget, binning=None, use_graph=True, max_slots=4096, vacf_stride=10):
        from . import mpcd
        self.m = mpcd
        self.vacf_stride = vacf_stride
        self.ctx = mpcd.Context(binning=mpcd.MPCD_BIN_AUTO if binning is None else binning,
                                use_graph=use_graph, hbm_budget=hbm_budget, max_slots=max_slots)

    def admit(self, req):
        d = self.m.make_desc(req["L"], req["n"], dt=req["dt"], alpha_deg=req["alpha_deg"],
                             seed=req["seed"], n_steps=req["steps"], init="maxwell",
                             vacf_stride=self.vacf_stride)
        return self.ctx.try_admit(d)

    def step(self, n):
        self.ctx.step(n)

    def observe(self, slot):
        o = self.ctx.observe(slot)
        return dict(step=o["step"], T=o["T"], vacf=o["vacf"], status=o["status"])

    def release(self, slot):
        self.ctx.release(slot)

    def close(self):
        self.ctx.close()


def request_key(req):
    """A request's name for cancellation: its "id" if it has one, else its seed."""
    return req.get("id", req["seed"])


class Server:
    """Admission by memory budget, batched stepping, per-request latency,
    cancellation."""

    def __init__(self, engine, chunk_steps=50, clock=time.perf_counter, sleep=time.sleep, max_live=None):
        self.engine = engine
        self.chunk_steps = int(chunk_steps)
        self.clock = clock
        self.sleep = sleep
        self.max_live = max_live
        self._lock = threading.Lock()
        self._cancel = set()

    def cancel(self, key):
        """Ask for the request named `key` (see request_key) to be cancelled;
        safe from another thread while run() serves.  Takes effect at the
        next scheduling round; a key that matches no unfinished request is
        ignored."""
        with self._lock:
            self._cancel.add(key)


    def run(self, requests, max_wall_s=None, progress=None, progress_every_s=10.0):
        """Serve `requests` (dicts with arrival, L, n, dt, alpha_deg, steps,
        seed; optional id and cancel_at; times in seconds from the start).
        Returns a summary dict and the per-request results.  `progress`, if
        given, is called about every progress_every_s seconds with the
        counts so far."""
        pending = collections.deque(sorted(requests, key=lambda r: r["arrival"]))
        queue = collections.deque()
        live = {}          # slot -> [request, steps left, admit time]
        done = []
        rejected = []      # requests larger than the whole budget
        cancelled = []
        t0 = self.clock()
        steps_done = 0     # particle-steps completed
        max_live = 0
        timed = collections.deque(sorted((r["cancel_at"], request_key(r)) for r in requests if "cancel_at" in r))
        t_report = 0.0
        while pending or queue or live:
            now = self.clock() - t0
            if max_wall_s is not None and now > max_wall_s:
                break
            if progress is not None and now - t_report >= progress_every_s:
                t_report = now
                progress(dict(t=now, completed=len(done), cancelled=len(cancelled), live=len(live),
                              queued=len(queue), pending=len(pending)))
            while timed and timed[0][0] <= now:
                self.cancel(timed.popleft()[1])
            with self._lock:
                kill = set(self._cancel)
            if kill:
                for slot in [s for s, v in live.items() if request_key(v[0]) in kill]:
                    req, left, t_admit = live.pop(slot)
                    self.engine.release(slot)     # steps still queued for it finish in stream order
                    cancelled.append(dict(req=req, latency=math.nan, queued=t_admit - req["arrival"],
                                          status="cancelled", step=int(req["steps"]) - max(left, 0)))
                for q in (queue, pending):
                    for req in [r for r in q if request_key(r) in kill]:
                        q.remove(req)
                        cancelled.append(dict(req=req, latency=math.nan, queued=math.nan,
                                              status="cancelled", step=0))
                with self._lock:           # keys that matched nothing unfinished are dropped too
                    self._cancel -= kill
            while pending and pending[0]["arrival"] <= now:
                queue.append(pending.popleft())
            # queue the next chunk for the live boxes; the engine returns at
            # once and a box that reaches its step count idles on the device
            stepped = bool(live)
            if stepped:
                self.engine.step(self.chunk_steps)
                for v in live.values():
                    steps_done += v[0]["n"] * min(self.chunk_steps, v[1])
                    v[1] -= self.chunk_steps
            # admit while the chunk runs (a new box joins at the next chunk)
            while queue and (self.max_live is None or len(live) < self.max_live):
                slot = self.engine.admit(queue[0])
                if slot is None:
                    if live:
                        break      # over budget / no slot: wait for releases
                    # nothing left to release: this request can never fit
                    req = queue.popleft()
                    rejected.append(dict(req=req, latency=math.nan, queued=now - req["arrival"],
                                         status="rejected"))
                    continue
                req = queue.popleft()
                live[slot] = [req, int(req["steps"]), now]
            max_live = max(max_live, len(live))
            # boxes done after this chunk: observe (waits for the chunk), release
            for slot in [s for s, v in live.items() if v[1] <= 0]:
                req, _, t_admit = live.pop(slot)
                obs = self.engine.observe(slot)
                self.engine.release(slot)
                t_done = self.clock() - t0
                done.append(dict(req=req, latency=t_done - req["arrival"], queued=t_admit - req["arrival"],
                                 T=obs["T"], vacf=obs["vacf"], status=obs["status"], step=obs["step"]))
            if not stepped and not live and pending and not queue:
                self.sleep(max(0.0, min(0.01, pending[0]["arrival"] - (self.clock() - t0))))
        wall = self.clock() - t0
        lat = np.array([d["latency"] for d in done]) if done else np.zeros(0)
        summary = dict(
            completed=len(done), offered=len(requests), rejected=len(rejected), cancelled=len(cancelled),
            wall_s=wall,
            particle_steps_per_s=steps_done / wall if wall > 0 else 0.0,
            p50_latency_s=float(np.percentile(lat, 50)) if len(lat) else math.nan,
            p99_latency_s=float(np.percentile(lat, 99)) if len(lat) else math.nan,
            max_live=max_live, unfinished=len(live) + len(queue) + len(pending))
        return summary, done + cancelled
