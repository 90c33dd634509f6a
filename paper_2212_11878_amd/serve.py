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

The scheduler talks to an engine with four calls (admit / step / observe /
release).  `LibraryEngine` drives libmpcd through its C ABI; tests can plug
in another engine to exercise queueing and admission without a GPU.
"""
import collections
import math
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


class Server:
    """Admission by memory budget, batched stepping, per-request latency."""

    def __init__(self, engine, chunk_steps=50, clock=time.perf_counter, sleep=time.sleep):
        self.engine = engine
        self.chunk_steps = int(chunk_steps)
        self.clock = clock
        self.sleep = sleep

    def run(self, requests, max_wall_s=None):
        """Serve `requests` (dicts with arrival, L, n, dt, alpha_deg, steps,
        seed; arrival in seconds from the start).  Returns a summary dict
        and the per-request results."""
        pending = collections.deque(sorted(requests, key=lambda r: r["arrival"]))
        queue = collections.deque()
        live = {}          # slot -> [request, steps left, admit time]
        done = []
        rejected = []      # requests larger than the whole budget
        t0 = self.clock()
        steps_done = 0     # particle-steps completed
        max_live = 0
        while pending or queue or live:
            now = self.clock() - t0
            if max_wall_s is not None and now > max_wall_s:
                break
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
            while queue:
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
            if not stepped and not live and pending:
                self.sleep(max(0.0, min(0.01, pending[0]["arrival"] - (self.clock() - t0))))
        wall = self.clock() - t0
        lat = np.array([d["latency"] for d in done]) if done else np.zeros(0)
        summary = dict(
            completed=len(done), offered=len(requests), rejected=len(rejected), wall_s=wall,
            particle_steps_per_s=steps_done / wall if wall > 0 else 0.0,
            p50_latency_s=float(np.percentile(lat, 50)) if len(lat) else math.nan,
            p99_latency_s=float(np.percentile(lat, 99)) if len(lat) else math.nan,
            max_live=max_live, unfinished=len(live) + len(queue) + len(pending))
        return summary, done
