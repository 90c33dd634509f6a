"""Hybrid CPU+GPU execution of an ensemble of independent boxes.

The paper runs part of a simulation on CPU ranks next to the GPU ranks of
the same node and finds no gain over the GPU alone (Sec. 4, Fig. 2f; Sec. 5).
Here the unit of work is a whole box: the GPU context advances its share of
the boxes in one batched launch sequence per step while host worker threads
advance the rest with the CPU leg (mpcd_host_step, one box per worker at a
time, the interpreter lock released during the call).  The share follows
the two measured rates, so both sides finish together: a host share of
R_cpu / (R_cpu + R_gpu) of the particle-steps, taken from the smallest
boxes (cheapest to hand back and forth; a box never moves once placed).
"""
import concurrent.futures
import os
import time

import numpy as np

from . import inputs, mpcd


def host_workers():
    """Host threads for the CPU leg: every core the process may use, less one
    that drives the GPU."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, n - 1)


def split(boxes, cpu_fraction):
    """Indices of the boxes for the host: the smallest, until their particles
    reach cpu_fraction of the total."""
    order = sorted(range(len(boxes)), key=lambda i: boxes[i]["n"])
    total = sum(b["n"] for b in boxes)
    host, acc = [], 0
    for i in order:
        if acc + boxes[i]["n"] > cpu_fraction * total:
            break
        host.append(i)
        acc += boxes[i]["n"]
    return sorted(host)


class HostBox:
    """A box in host memory advanced by the CPU leg."""

    def __init__(self, b):
        self.desc = mpcd.make_desc(b["L"], b["n"], dt=b["dt"], alpha_deg=b["alpha_deg"], seed=b["seed"],
                                   init="external")
        pos, vel = inputs.thermal_state(b["L"], b["n"], seed=b["seed"] & 0x7FFFFFFF)
        self.xyzv = np.ascontiguousarray(np.concatenate([pos, vel]).astype(np.float32))
        self.step = 0

    def advance(self, n_steps, threads=1):
        rc = mpcd.mpcd_host_step(self.desc, self.xyzv, None, None, self.step, n_steps, threads)
        if rc != mpcd.MPCD_OK:
            raise mpcd.MPCDError(rc, "mpcd_host_step")
        self.step += n_steps

    def temperature(self):
        v = self.xyzv[3:].astype(np.float64)
        w = v - v.mean(axis=1, keepdims=True)
        return float(np.sum(w * w) / (3 * max(1, v.shape[1] - 1)))


class HybridEnsemble:
    """Boxes split between one GPU context and the host's cores."""

    def __init__(self, boxes, host_indices, workers=None, **ctx_options):
        self.boxes = boxes
        self.host_idx = list(host_indices)
        hs = set(self.host_idx)
        self.gpu_idx = [i for i in range(len(boxes)) if i not in hs]
        self.ctx = mpcd.Context(**ctx_options)
        self.slots = [self.ctx.admit(mpcd.make_desc(boxes[i]["L"], boxes[i]["n"], dt=boxes[i]["dt"],
                                                    alpha_deg=boxes[i]["alpha_deg"], seed=boxes[i]["seed"]))
                      for i in self.gpu_idx]
        self.host = [HostBox(boxes[i]) for i in self.host_idx]
        self.workers = workers or host_workers()
        self.pool = concurrent.futures.ThreadPoolExecutor(max_workers=self.workers)

    def step(self, n_steps):
        """Advance every box by n_steps; returns (wall seconds until both
        sides are done, seconds until the host side is done)."""
        t0 = time.perf_counter()
        if self.slots:
            self.ctx.step(n_steps)          # queued; returns at once
        # biggest host boxes first, so the workers end together
        order = sorted(self.host, key=lambda h: -h.desc.n_particles)
        futs = [self.pool.submit(h.advance, n_steps) for h in order]
        for f in futs:
            f.result()
        t_host = time.perf_counter() - t0
        self.ctx.synchronize()
        return time.perf_counter() - t0, t_host

    def observe(self):
        """Temperature and status of every box, in ensemble order."""
        out = [None] * len(self.boxes)
        for i, s in zip(self.gpu_idx, self.slots):
            o = self.ctx.observe(s)
            out[i] = dict(T=o["T"], step=o["step"], status=o["status"], where="gpu")
        for i, h in zip(self.host_idx, self.host):
            out[i] = dict(T=h.temperature(), step=h.step, status=0, where="cpu")
        return out

    def close(self):
        self.pool.shutdown()
        self.ctx.close()


def host_rate(boxes, workers, steps=20):
    """Particle-steps/s of the CPU leg over the host workers, one box per
    worker (a sample of the smallest boxes, which the split sends there)."""
    sample = sorted(boxes, key=lambda b: b["n"])[:workers]
    hb = [HostBox(b) for b in sample]
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as pool:
        t0 = time.perf_counter()
        list(pool.map(lambda h: h.advance(steps), hb))
        t = time.perf_counter() - t0
    return sum(b["n"] for b in sample) * steps / t
