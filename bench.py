"""Benchmark of the SRD step on one MI355X.

Default workload: one periodic box of 256^3 unit cells with 10 particles per
cell (167,772,160 particles), dt = 0.1, alpha = 130 deg, seed 3, positions
uniform and velocities Maxwellian at kT = 1 drawn on the device (the paper's
benchmark system, Sec. 4, at its L = 256 size).  A "step" is one SRD update of
the whole box: stream, random shift, binning, exact cell sums, rotation, and
the range check that guards the sums (momentum, energy and temperature are
summed on demand by mpcd_observe, outside the timed region).  By default the
box keeps no particle ids (MPCD_UNORDERED: the steps move x and v only);
--ids times the id-carrying configuration, and the line also reports a
shorter run of it.

Prints ONE JSON line: particle-steps/s of K steps replayed from the captured
graph; the roofline of the dominant kernel (algorithmic bytes per launch / its
average HIP-event duration, from a separate profiled pass of eagerly launched
steps on the library stream); the counter-based fraction when the committed
counter summary matches the kernel sources; the streaming-copy ceiling of the
same GPU; and the FP64 oracle on the host (one core, and one process per core).
"""
import argparse
import gc
import hashlib
import json
import math
import multiprocessing
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (L, particles per cell, dt, alpha_deg, seed)
    "srd_256cube_10ppc": ((256, 256, 256), 10, 0.1, 130.0, 3),
    "srd_100cube_10ppc": ((100, 100, 100), 10, 0.1, 130.0, 2),
    "srd_512cube_10ppc": ((512, 512, 512), 10, 0.1, 130.0, 5),   # the paper's largest system
}
DEFAULT_WORKLOAD = "srd_256cube_10ppc"
ENSEMBLE = "ensemble_512_boxes"      # 512 boxes, edges U{8..48}, densities U[5,20]
SERVED = "served_poisson"            # Poisson arrivals of single-box requests

# Algorithmic bytes each kernel's function has to move, per particle (P) and
# per cell (C), independent of how the kernel is written:
#   brick_step : the whole step of the brick boxes; read x, v (24 B) and
#                write x, v (24 B); the cell sums live and die in LDS   -> 48 P
#   cell_rotate: SORT binning, plain rule: move every particle to its
#                slot in cell order and collide it; read x, v (24 B),
#                write x, v (24 B)                                    -> 48 P
#   scatter    : SORT binning, plain rule: the permutation; read the
#                key and rank (8 B), write the source slot (4 B)      -> 12 P
#   count      : read x, v (24 B: the key is the streamed position's
#                cell), write the key (4 B)                           -> 28 P
ALGO_BYTES = {
    "brick_step": (48, 0),
    "cell_rotate": (48, 0),
    "scatter": (12, 0),
    "count": (28, 0),
}
# the whole step: every particle's x and v read once and written once
STEP_ALGO_BYTES_PER_PARTICLE = 48
PROFILED_STEPS = 20      # eagerly launched steps with per-kernel events
REPEATS = 5              # further timed runs of K graph-replayed steps (median reported)
COPY_BYTES = 4 << 30     # streaming-copy ceiling: 4 GiB copied


def context_options():
    """Launch configuration the benchmark times (also used by the full-size
    parity test)."""
    from paper_2212_11878_amd import mpcd
    return dict(binning=mpcd.MPCD_BIN_AUTO, use_graph=True)


def kernel_sources_sha():
    """Hash of the sources that decide a step's memory traffic (kernels, and
    the engine's bucket layout and launch order)."""
    h = hashlib.sha256()
    for f in ("mpcd_dev.h", "mpcd_kernels.hip", "mpcd_engine.hip"):
        with open(os.path.join(ROOT, "paper_2212_11878_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per dispatch from the committed rocprofv3 counter summary,
    or None when missing or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_sources_sha") != kernel_sources_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def _oracle_rate(L, ppc, dt, alpha, seed, steps):
    """Particle-steps/s of the FP64 oracle on one core (one box, `steps` steps)."""
    from oracle import oracle as orc
    from paper_2212_11878_amd import inputs
    n = ppc * L[0] * L[1] * L[2]
    pos, vel = inputs.thermal_state(L, n, seed)
    st = orc.State(pos, vel)
    del pos, vel
    box = orc.make_box(L, dt=dt, alpha_deg=alpha, seed=seed)
    t0 = time.perf_counter()
    orc.run(box, 0, steps, st)
    return n * steps, time.perf_counter() - t0


def _oracle_worker(args):
    L, ppc, dt, alpha, seed, steps = args
    return _oracle_rate(L, ppc, dt, alpha, seed, steps)


def host_cores():
    """Processing units available to this process, as `nproc` reports them
    (it honours the affinity mask and OMP_NUM_THREADS), at most 16."""
    try:
        n = int(subprocess.run(["nproc"], capture_output=True, text=True, check=True).stdout.strip())
    except (OSError, ValueError, subprocess.CalledProcessError):
        n = len(os.sched_getaffinity(0))
    return max(1, min(16, n)), n


def cpu_baseline(workload):
    """The FP64 oracle as it stands, on bounded samples of the workload: one
    core on a 128^3-cell box (3 steps), then one oracle process per core,
    each on its own 96^3-cell box of the same density (2 steps).  Runs before
    the GPU is touched, entirely in spawned worker processes (their memory is
    returned before the GPU is timed)."""
    L, ppc, dt, alpha, seed = WORKLOADS[workload]
    Ls = tuple(min(128, l) for l in L)
    cores, nproc = host_cores()
    Lw = tuple(min(96, l) for l in L)
    jobs = [(Lw, ppc, dt, alpha, seed + 1000 * (i + 1), 2) for i in range(cores)]
    ctx = multiprocessing.get_context("spawn")
    with ctx.Pool(1) as pool:
        work1, t1 = pool.apply(_oracle_worker, ((Ls, ppc, dt, alpha, seed, 3),))
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    work = sum(r[0] for r in res)
    # the rate of the slowest worker's span, not the pool start-up
    span = max(r[1] for r in res)
    return {"value": work / span, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "nproc": nproc,
            "sample": "%d processes (one per core), each a %dx%dx%d-cell box x %d particles/cell, 2 steps, "
                      "FP64; rate = all particle-steps / the slowest process's stepping time (%.1f s; "
                      "%.1f s with start-up)" % (cores, Lw[0], Lw[1], Lw[2], ppc, span, wall),
            "per_core": {"value": work1 / t1, "sample": "%dx%dx%d cells x %d particles/cell (%d particles), "
                                                        "3 steps, FP64, %.1f s"
                                                        % (Ls[0], Ls[1], Ls[2], ppc, ppc * Ls[0] * Ls[1] * Ls[2],
                                                           t1)}}


def copy_ceiling():
    """The GPU's practical HBM rate: the library's streaming copy of 4 GiB
    (read and write: 8 GiB moved), best of 5 after a warm-up, HIP events on
    the stream it runs on; a PyTorch device copy for comparison."""
    import torch
    from paper_2212_11878_amd import mpcd
    n = COPY_BYTES // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    s = torch.cuda.current_stream()
    out = {}
    def lib_copy():
        rc = mpcd.mpcd_hbm_copy(a.data_ptr(), b.data_ptr(), COPY_BYTES, 0, s.cuda_stream)
        if rc != mpcd.MPCD_OK:
            raise RuntimeError("mpcd_hbm_copy failed: %d" % rc)

    for name, fn in (("hbm_copy", lib_copy), ("torch_copy", lambda: b.copy_(a))):
        best = None
        for r in range(6):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fn()
            e1.record(s)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            if r > 0:
                best = ms if best is None else min(best, ms)
        out[name] = round(2 * COPY_BYTES / (best * 1e-3) / 1e9, 1)
    assert torch.equal(a[:1024], b[:1024])
    del a, b
    torch.cuda.empty_cache()
    return {"GBs": out["hbm_copy"], "frac": round(out["hbm_copy"] / HBM_PEAK_GBS, 4),
            "torch_copy_GBs": out["torch_copy"], "bytes_moved": 2 * COPY_BYTES}


def run_box(args, L, n, dt, alpha, seed, ids, steps, warmup, repeats, profiled):
    """Admit one box, warm up, time `steps` graph-replayed steps (then
    `repeats` more runs of the same length), then a profiled pass."""
    import torch
    from paper_2212_11878_amd import mpcd
    opts = context_options()
    if args.binning != "auto":
        opts["binning"] = mpcd.MPCD_BIN_ATOMIC if args.binning == "atomic" else mpcd.MPCD_BIN_SORT
    opts["brick"] = tuple(args.brick)
    ctx = mpcd.Context(**opts)
    slot = ctx.admit(mpcd.make_desc(L, n, dt=dt, alpha_deg=alpha, seed=seed, init="maxwell",
                                    particle_mass=args.masses, conserve_l=args.conserve_l,
                                    unordered=not ids))
    ctx.step(warmup)
    ctx.synchronize()
    print("[bench] warmup done, timing %d steps (graph replay, ids=%s)" % (steps, ids), file=sys.stderr,
          flush=True)

    def timed(k):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(ctx.stream)
        ctx.step(k)
        e1.record(ctx.stream)
        ctx.synchronize()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, e0.elapsed_time(e1) * 1e-3

    t, t_ev = timed(steps)
    runs = [t_ev] + [timed(steps)[1] for _ in range(repeats)]
    stats = {}
    if profiled:
        ctx.profile(True)
        ctx.step(profiled)
        stats = ctx.kernel_stats()
        ctx.profile(False)
    obs = ctx.observe(slot)
    ctx.close()
    total = warmup + steps * (1 + repeats) + profiled
    if obs["status"] != 0 or obs["step"] != total:
        print("[bench] box state invalid: %r" % obs, file=sys.stderr)
        sys.exit(1)
    return t, runs, stats, obs


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS) + [ENSEMBLE, SERVED])
    ap.add_argument("--rate", type=float, nargs="+", default=[200.0],
                    help="served: arrival rates (req/s) to sweep")
    ap.add_argument("--window", type=float, default=60.0, help="served: seconds of arrivals")
    ap.add_argument("--hybrid", action="store_true",
                    help="ensemble: also split the boxes between the GPU and the host's cores")
    ap.add_argument("--compare-serial", action="store_true",
                    help="served: also serve the same requests one box at a time")
    ap.add_argument("--binning", default="auto", choices=["auto", "atomic", "sort"])
    ap.add_argument("--brick", type=int, nargs=3, default=[0, 0, 0])
    ap.add_argument("--masses", action="store_true",
                    help="every particle carries its own mass (all 1: the mass-weighted path; implies --ids)")
    ap.add_argument("--conserve-l", action="store_true", help="angular-momentum-conserving collision")
    ap.add_argument("--ids", action="store_true", help="the box keeps particle ids (56 B per particle-step)")
    ap.add_argument("--no-ids-run", action="store_true", help="skip the short reference run with particle ids")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-ceiling", action="store_true")
    ap.add_argument("--profiled-steps", type=int, default=PROFILED_STEPS)
    ap.add_argument("--repeats", type=int, default=REPEATS)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs each box on one device "
              "(a multi-GPU halo decomposition is not implemented); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        import torch
        from paper_2212_11878_amd import mpcd
        # copies of known size: their FETCH_SIZE / WRITE_SIZE counters per
        # dispatch calibrate the kernels' counters to bytes
        nbytes = args.copy_calibration << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):   # the library's streaming copy: reads and writes nbytes
            mpcd.mpcd_hbm_copy(a.data_ptr(), b.data_ptr(), nbytes, 0, torch.cuda.current_stream().cuda_stream)
        for _ in range(5):   # full-grid elementwise kernel: reads and writes nbytes
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "dispatches": 5}), flush=True)
        return

    if args.workload == ENSEMBLE:
        return bench_ensemble(args)
    if args.workload == SERVED:
        return bench_served(args)

    L, ppc, dt, alpha, seed = WORKLOADS[args.workload]
    n = ppc * L[0] * L[1] * L[2]
    ncell = L[0] * L[1] * L[2]
    ids = args.ids or args.masses
    cpu = None
    if not args.no_cpu_baseline:   # before any GPU call: its workers are separate processes
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.workload)
        gc.collect()

    print("[bench] workload %s: %d particles, admitting" % (args.workload, n), file=sys.stderr, flush=True)
    t, runs, stats, obs = run_box(args, L, n, dt, alpha, seed, ids, args.steps, args.warmup, args.repeats,
                                  args.profiled_steps)
    value = n * args.steps / t
    ms_per_step = 1000.0 * t / args.steps

    # dominant kernel by total time in the profiled pass
    roofline = None
    kern = {}
    if stats:
        dom = max(stats.items(), key=lambda kv: kv[1][1])
        kname, (launches, total_ms) = dom
        avg_ms = total_ms / max(1, launches)
        per_p, per_c = ALGO_BYTES.get(kname, (0, 0))
        algo = per_p * n + per_c * ncell
        achieved = algo / (avg_ms * 1e-3) / 1e9
        workload_tag = args.workload + ("" if not ids else "_ids")
        traffic = load_traffic(kname, workload_tag)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": kname, "kernel_avg_ms": round(avg_ms, 4),
                    "algorithmic_bytes_per_launch": algo,
                    "counter_frac": (round(traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                     if traffic else None)}
        kern = {k: {"launches": v[0], "avg_ms": round(v[1] / max(1, v[0]), 4)} for k, v in stats.items()}

    out = {
        "metric": "particle-steps/s",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": list(L), "particles": n, "dt": dt,
                   "alpha_deg": alpha, "seed": seed, "binning": obs["binning"],
                   "brick": list(obs["brick"]), "particle_ids": bool(ids),
                   "particle_masses": bool(args.masses),
                   "conserve_angular_momentum": bool(args.conserve_l), "graph": True},
        "useful_hbm_frac": round(value * STEP_ALGO_BYTES_PER_PARTICLE / 1e9 / HBM_PEAK_GBS, 4),
        "ms_per_step_runs": [round(1000.0 * r / args.steps, 4) for r in runs],
        "ms_per_step_median": round(1000.0 * statistics.median(runs) / args.steps, 4),
        "roofline": roofline,
        "kernels": kern,
        "profiled_steps": args.profiled_steps,
    }
    if not ids and not args.no_ids_run:
        # the same box with particle ids (56 B per particle-step), shorter run
        k2 = max(10, args.steps // 5)
        t2, _, st2, _ = run_box(args, L, n, dt, alpha, seed, True, k2, args.warmup, 0, 10)
        ref = {"value": n * k2 / t2, "steps": k2, "ms_per_step": 1000.0 * t2 / k2}
        if st2:
            kn, (la, tm) = max(st2.items(), key=lambda kv: kv[1][1])
            ref["kernel"] = kn
            ref["kernel_avg_ms"] = round(tm / max(1, la), 4)
        out["with_particle_ids"] = ref
    if not args.no_copy_ceiling:
        out["copy_ceiling"] = copy_ceiling()
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def bench_ensemble(args):
    """512 independent boxes advanced together (one batched launch sequence
    per step, graph replay) against the same boxes advanced one at a time."""
    import torch
    from paper_2212_11878_amd import inputs, mpcd
    boxes = inputs.ensemble_boxes(512, seed=4)
    total = sum(b["n"] for b in boxes)

    def desc(b):
        return mpcd.make_desc(b["L"], b["n"], dt=b["dt"], alpha_deg=b["alpha_deg"], seed=b["seed"])

    print("[bench] ensemble: %d boxes, %d particles" % (len(boxes), total), file=sys.stderr, flush=True)
    ctx = mpcd.Context(**context_options())
    t_adm = time.perf_counter()
    slots = [ctx.admit(desc(b)) for b in boxes]
    t_adm = time.perf_counter() - t_adm
    ctx.step(args.warmup)
    ctx.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(args.steps)
    ctx.synchronize()
    t_batch = time.perf_counter() - t0
    ctx.profile(True)
    ctx.step(2)
    stats = ctx.kernel_stats()
    ctx.profile(False)
    bad = [s for s in slots if ctx.observe(s)["status"] != 0]
    ctx.close()
    # baseline: the same boxes one at a time on the same GPU, same step count
    print("[bench] ensemble: one box at a time", file=sys.stderr, flush=True)
    solo = mpcd.Context(**context_options())
    t_one = 0.0
    for b in boxes:
        s = solo.admit(desc(b))
        solo.step(args.warmup)
        solo.synchronize()
        t1 = time.perf_counter()
        solo.step(args.steps)
        solo.synchronize()
        t_one += time.perf_counter() - t1
        solo.release(s)
    solo.close()
    value = total * args.steps / t_batch
    one = total * args.steps / t_one
    hybrid = bench_hybrid(args, boxes, value) if args.hybrid else None
    out = {"metric": "particle-steps/s", "value": value, "unit": "particle-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1000 * t_batch / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": ENSEMBLE, "boxes": len(boxes), "particles": total,
                      "edges": "U{8..48}", "density": "U[5,20]", "alpha_deg": [90, 120, 130], "dt": 0.1},
           "one_box_at_a_time": {"value": one, "ms_per_step": 1000 * t_one / args.steps},
           "batched_over_one_at_a_time": value / one, "admission_s": t_adm,
           "nonfinite_boxes": len(bad),
           "kernels": {k: {"launches": v[0], "avg_ms": round(v[1] / max(1, v[0]), 4)}
                       for k, v in stats.items()}}
    if hybrid is not None:
        out["hybrid_cpu_gpu"] = hybrid
    print(json.dumps(out), flush=True)


def bench_hybrid(args, boxes, gpu_rate):
    """The same boxes split between the GPU and the host's cores (the CPU leg,
    one box per worker thread), in the proportion of the two measured rates,
    both advancing at once."""
    from paper_2212_11878_amd import hybrid
    workers = hybrid.host_workers()
    print("[bench] hybrid: host rate on %d workers" % workers, file=sys.stderr, flush=True)
    cpu_rate = hybrid.host_rate(boxes, workers)
    frac = cpu_rate / (cpu_rate + gpu_rate)
    host_idx = hybrid.split(boxes, frac)
    ens = hybrid.HybridEnsemble(boxes, host_idx, workers=workers, **context_options())
    total = sum(b["n"] for b in boxes)
    ens.step(args.warmup)
    print("[bench] hybrid: %d boxes on the host (%.3f of the particles), %d on the GPU"
          % (len(host_idx), sum(boxes[i]["n"] for i in host_idx) / total, len(ens.gpu_idx)),
          file=sys.stderr, flush=True)
    wall, t_host = ens.step(args.steps)
    obs = ens.observe()
    ens.close()
    rate = total * args.steps / wall
    return {"value": rate, "ms_per_step": 1000 * wall / args.steps, "over_gpu_only": rate / gpu_rate,
            "host_workers": workers, "host_rate_measured": cpu_rate, "host_boxes": len(host_idx),
            "host_particle_fraction": sum(boxes[i]["n"] for i in host_idx) / total,
            "host_side_ms_per_step": 1000 * t_host / args.steps,
            "bad_status_boxes": sum(1 for o in obs if o["status"] != 0)}


def bench_served(args):
    """Continuous batching of Poisson-arriving single-box requests: p50/p99
    latency and sustained throughput per arrival rate over a fixed window of
    arrivals; with --compare-serial the same requests also go through the
    same server one box at a time."""
    from paper_2212_11878_amd import inputs, serve

    def served(reqs, max_live, label):
        eng = serve.LibraryEngine(hbm_budget=64 << 30)

        def report(p):
            print("[bench] %s: t %.0f s, %d done, %d live, %d queued, %d not yet arrived"
                  % (label, p["t"], p["completed"], p["live"], p["queued"], p["pending"]),
                  file=sys.stderr, flush=True)
        summary, _ = serve.Server(eng, chunk_steps=50, max_live=max_live).run(
            reqs, max_wall_s=args.window * 2, progress=report)
        eng.close()
        summary["offered_particle_steps_per_s"] = sum(r["n"] * r["steps"] for r in reqs) / args.window
        print("[bench] %s: %r" % (label, summary), file=sys.stderr, flush=True)
        return summary

    sweep = []
    for rate in args.rate:
        reqs = inputs.served_requests(rate_hz=rate, window_s=args.window, seed=5)
        print("[bench] served: %g req/s, %d requests" % (rate, len(reqs)), file=sys.stderr, flush=True)
        summary = served(reqs, None, "served %g req/s" % rate)
        summary["rate_hz"] = rate
        if args.compare_serial:
            summary["one_at_a_time"] = served([dict(r) for r in reqs], 1, "one at a time %g req/s" % rate)
        sweep.append(summary)
    head = sweep[-1]
    out = {"metric": "p50/p99 request latency and particle-steps/s", "value": head["particle_steps_per_s"],
           "unit": "particle-steps/s", "n_gpus": 1, "steps": None, "warmup": None, "ms_per_step": None,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": SERVED, "edges": "U{8..64}", "density": "U[5,20]", "dt": "U[0.05,0.2]",
                      "alpha_deg": "U[90,150]", "steps": "U{200..2000}", "window_s": args.window,
                      "max_wall_s": args.window * 2, "rate_hz": head["rate_hz"], "vacf_stride": 10,
                      "chunk_steps": 50},
           "p50_latency_s": head["p50_latency_s"], "p99_latency_s": head["p99_latency_s"],
           "sweep": sweep}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
