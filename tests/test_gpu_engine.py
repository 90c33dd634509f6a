"""GPU tests of the engine behaviour around the step: binning modes, graph
replay, batching, device-side initial state, diagnostics, VACF, errors."""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2212_11878_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_11878_amd import mpcd
    return mpcd


def _say(*a):
    print("[case]", *a, flush=True)


def _run(mp, boxes, steps, binning, use_graph=True, chunks=1, brick=(0, 0, 0)):
    """Admit (L, n, seed, alpha) boxes with a shared-input state, run, return states."""
    out = []
    with mp.Context(binning=binning, use_graph=use_graph, brick=brick) as ctx:
        slots = []
        for (L, n, seed, alpha) in boxes:
            pos, vel = inputs.thermal_state(L, n, seed)
            s = ctx.admit(mp.make_desc(L, n, alpha_deg=alpha, seed=seed, init="external"))
            ctx.set_state(s, (pos, vel))
            slots.append(s)
        for _ in range(chunks):
            ctx.step(steps)
        for s in slots:
            out.append(ctx.get_state(s))
    return out


def test_binning_modes_bit_identical(mp):
    """Cell sums are exact integers, so brick binning (any brick shape) and
    sort binning give the same bits for every particle."""
    _say("modes")
    boxes = [((12, 20, 9), 21600, 4, 130.0)]
    a = _run(mp, boxes, 25, mp.MPCD_BIN_ATOMIC)[0]
    b = _run(mp, boxes, 25, mp.MPCD_BIN_SORT)[0]
    c = _run(mp, boxes, 25, mp.MPCD_BIN_ATOMIC, brick=(4, 4, 4))[0]
    d = _run(mp, boxes, 25, mp.MPCD_BIN_ATOMIC, brick=(16, 2, 4))[0]
    for x, y in ((a, b), (a, c), (a, d)):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])


def test_fast_particles_go_past_the_neighbour_bricks(mp):
    """dt = 1.5 moves particles several cells per step: many are bound for
    buckets beyond the 27 neighbours of their brick (one-at-a-time slots,
    overflow when those fill); the result must still equal sort binning bit
    for bit."""
    _say("escapes")
    L, n = (10, 12, 8), 9600
    pos, vel = inputs.thermal_state(L, n, 19)
    out = []
    for binning in (mp.MPCD_BIN_ATOMIC, mp.MPCD_BIN_SORT):
        with mp.Context(binning=binning, brick=(4, 4, 4)) as ctx:
            s = ctx.admit(mp.make_desc(L, n, dt=1.5, seed=19, init="external"))
            ctx.set_state(s, (pos, vel))
            ctx.step(6)
            out.append(ctx.get_state(s))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def _slab(n, seed, drift):
    """Particles in the slab x < 3 of a 16^3 box, drifting along +x."""
    g = np.random.default_rng(seed)
    pos = np.empty((3, n), np.float32)
    pos[0] = g.uniform(0.0, 3.0, n)
    pos[1] = g.uniform(0.0, 16.0, n)
    pos[2] = g.uniform(0.0, 16.0, n)
    vel = g.standard_normal((3, n)).astype(np.float32)
    vel[0] += np.float32(drift)
    return pos, vel


def test_bucket_overflow_matches_sort(mp):
    """A dense slab drifting into bricks that were empty when the buckets
    were sized overflows them: those particles go to the overflow bucket
    (escape sums for their next cells, the overflow pass of the next step)
    until the host re-buckets at its next step call.  The trajectory must
    equal sort binning bit for bit, and the counters must show both."""
    _say("overflow")
    L, n = (16, 16, 16), 20000
    pos, vel = _slab(n, 31, 4.0)
    out, obs = [], []
    for binning in (mp.MPCD_BIN_ATOMIC, mp.MPCD_BIN_SORT):
        with mp.Context(binning=binning, brick=(4, 4, 4)) as ctx:
            s = ctx.admit(mp.make_desc(L, n, dt=0.1, seed=31, init="external"))
            ctx.set_state(s, (pos, vel))
            for _ in range(8):
                ctx.step(3)   # overflow in one step is drained by the next ones
            out.append(ctx.get_state(s))
            obs.append(ctx.observe(s))
    print("[overflow] steps with overflow %d, re-bucketings %d" % (obs[0]["overflow_steps"], obs[0]["rebuckets"]),
          flush=True)
    assert obs[0]["overflow_steps"] > 0 and obs[0]["rebuckets"] >= 2
    assert out[0][2] == out[1][2] == 24
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert obs[0]["E"] == obs[1]["E"] and np.array_equal(obs[0]["P"], obs[1]["P"])


def test_bucket_overflow_one_step_parity(mp):
    """The overflow slab stepped one call at a time, each step checked
    against the oracle from the GPU's own previous state."""
    from gpu_util import compare_step
    _say("overflow-parity")
    L, n = (16, 16, 16), 20000
    pos, vel = _slab(n, 37, 4.0)
    box = orc.make_box(L, dt=0.1, alpha_deg=130.0, seed=37)
    with mp.Context(binning=mp.MPCD_BIN_ATOMIC, brick=(4, 4, 4)) as ctx:
        s = ctx.admit(mp.make_desc(L, n, dt=0.1, seed=37, init="external"))
        ctx.set_state(s, (pos, vel))
        ctx.step(2)
        for k in range(2, 8):
            p0, v0, step = ctx.get_state(s)
            assert step == k
            ctx.step(1)
            p1, v1, _ = ctx.get_state(s)
            compare_step(p0, v0, p1, v1, box, k)
        o = ctx.observe(s)
    assert o["rebuckets"] >= 2


def test_buckets_larger_than_one_chunk(mp):
    """Buckets of ~10^4 particles (8^3 bricks at 20 per cell) exceed what a
    workgroup holds in registers: the step runs in chunks, re-reading all
    but the first; bits equal sort binning."""
    _say("chunks")
    boxes = [((16, 16, 16), 81920, 41, 130.0)]
    a = _run(mp, boxes, 6, mp.MPCD_BIN_ATOMIC, brick=(8, 8, 8))[0]
    b = _run(mp, boxes, 6, mp.MPCD_BIN_SORT)[0]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_graph_replay_matches_eager(mp):
    """Every replay of the captured step equals the eager sequence, with
    host synchronisations between replays."""
    _say("graph")
    boxes = [((10, 10, 10), 10000, 6, 120.0)]
    eager = _run(mp, boxes, 5, mp.MPCD_BIN_ATOMIC, use_graph=False, chunks=4)[0]
    graph = _run(mp, boxes, 5, mp.MPCD_BIN_ATOMIC, use_graph=True, chunks=4)[0]
    assert np.array_equal(eager[0], graph[0]) and np.array_equal(eager[1], graph[1])


def test_box_alone_equals_box_in_mix(mp):
    """Results depend only on (seed, step, state): a box advanced alone and
    advanced in a batch of uneven boxes ends in the same bits."""
    _say("mix")
    mix = [((8, 8, 8), 5120, 11, 90.0), ((20, 20, 20), 160000, 12, 130.0),
           ((9, 13, 5), 4000, 13, 120.0), ((3, 3, 3), 0, 14, 130.0), ((16, 16, 16), 61440, 15, 150.0)]
    for binning in (mp.MPCD_BIN_ATOMIC, mp.MPCD_BIN_SORT):
        together = _run(mp, mix, 30, binning)
        for i, box in enumerate(mix):
            alone = _run(mp, [box], 30, binning)[0]
            assert np.array_equal(alone[0], together[i][0])
            assert np.array_equal(alone[1], together[i][1])
            assert alone[2] == together[i][2] == 30


def test_device_maxwell_initial_state(mp):
    _say("init")
    L, n = (30, 30, 30), 270000
    with mp.Context() as ctx:
        s = ctx.admit(mp.make_desc(L, n, seed=77, kT=1.7, mass=1.0))
        o = ctx.observe(s)
        pos, vel, step = ctx.get_state(s)
    assert step == 0 and o["step"] == 0
    assert abs(o["T"] - 1.7) < 1e-5
    assert np.all(np.abs(o["P"]) < 1e-2)
    assert pos.min() >= 0 and pos.max() < 30
    # uniform positions: occupancy of 1000 coarse bins
    h, _ = np.histogramdd(pos.T, bins=(10, 10, 10), range=[(0, 30)] * 3)
    assert abs(h.mean() - 270) < 1e-9 and h.std() < 4 * math.sqrt(270)
    # Gaussian components
    x = vel.reshape(-1).astype(np.float64) / math.sqrt(1.7)
    assert abs(np.mean(x ** 2) - 1) < 0.01 and abs(np.mean(x ** 4) - 3) < 0.05


def test_conservation_over_many_steps(mp):
    """FP32 state, exact cell sums: over 500 steps of a 10^6-particle box the
    energy drifts by less than 1e-6 relative and the momentum by less than
    1e-8 N m sqrt(kT/m)."""
    _say("conservation")
    L, n = (50, 50, 40), 1000000
    with mp.Context() as ctx:
        s = ctx.admit(mp.make_desc(L, n, seed=3))
        o0 = ctx.observe(s)
        ctx.step(500)
        o1 = ctx.observe(s)
    assert o1["step"] == 500 and o1["status"] == 0
    print("[conservation] E0 %.12e E1 %.12e rel %.3e P0 %s P1 %s" % (
        o0["E"], o1["E"], (o1["E"] - o0["E"]) / o0["E"], o0["P"], o1["P"]), flush=True)
    assert abs(o1["E"] - o0["E"]) / o0["E"] < 1e-6, (o0["E"], o1["E"])
    assert np.all(np.abs(o1["P"] - o0["P"]) < 1e-8 * n), (o0["P"], o1["P"])


def test_diagnostics_match_oracle(mp):
    _say("diag")
    L, n = (10, 10, 10), 10000
    pos, vel = inputs.thermal_state(L, n, 21)
    with mp.Context() as ctx:
        s = ctx.admit(mp.make_desc(L, n, seed=21, init="external"))
        ctx.set_state(s, (pos, vel))
        ctx.step(10)
        o = ctx.observe(s)
        gp, gv, _ = ctx.get_state(s)
    P, E, T, M = orc.diagnostics(orc.State(gp, gv))
    assert np.allclose(o["P"], P, rtol=0, atol=1e-9)
    assert abs(o["E"] - E) < 1e-9 * E and abs(o["T"] - T) < 1e-9 * T and o["M"] == M


@pytest.mark.parametrize("binning", ["auto", "sort"])
def test_vacf_samples(mp, binning):
    """VACF sample j = (1/N) sum v(j stride) . v(0), recorded on the device
    (with counting-sort binning the collision reads each particle's id from
    the buffer it has just gathered into)."""
    _say("vacf", binning)
    L, n = (12, 12, 12), 17280
    pos, vel = inputs.thermal_state(L, n, 8)
    with mp.Context(**({} if binning == "auto" else dict(binning=mp.MPCD_BIN_SORT))) as ctx:
        s = ctx.admit(mp.make_desc(L, n, seed=8, init="external", vacf_stride=3, n_steps=12))
        ctx.set_state(s, (pos, vel))
        ctx.step(20)                       # stops at n_steps
        o = ctx.observe(s)
        gp, gv, step = ctx.get_state(s)
    assert step == 12 and o["step"] == 12
    assert len(o["vacf"]) == 5
    v0 = vel.astype(np.float64)
    assert abs(o["vacf"][0] - np.sum(v0 * v0) / n) < 1e-9
    assert abs(o["vacf"][-1] - np.sum(gv.astype(np.float64) * v0) / n) < 1e-9


@pytest.mark.parametrize("binning", ["auto", "sort"])
def test_one_step_vacf_closed_form_gpu(mp, binning):
    """Same statistical pin as the oracle's, on the GPU path at 1.6e6 particles."""
    _say("vacf-closed-form", binning)
    L, n = 54, 10 * 54 ** 3
    alpha = math.radians(130.0)
    inv_n = L ** 3 / n * (1 - (1 - 1 / L ** 3) ** n)
    want = 1 - (2 / 3) * (1 - math.cos(alpha)) * (1 - inv_n)
    with mp.Context(**({} if binning == "auto" else dict(binning=mp.MPCD_BIN_SORT))) as ctx:
        s = ctx.admit(mp.make_desc(L, n, seed=31, vacf_stride=1, n_steps=1))
        ctx.step(1)
        v = ctx.observe(s)["vacf"]
    got = v[1] / v[0]
    assert abs(got - want) < 5 * math.sqrt(3.0 / n), (got, want)


def test_stop_after_n_steps_and_release(mp):
    _say("lifecycle")
    with mp.Context() as ctx:
        a = ctx.admit(mp.make_desc(8, 5120, seed=1, n_steps=5))
        b = ctx.admit(mp.make_desc(8, 5120, seed=2, n_steps=0))
        ctx.step(8)
        assert ctx.observe(a)["step"] == 5
        assert ctx.observe(b)["step"] == 8
        ctx.release(a)
        with pytest.raises(mp.MPCDError) as e:
            ctx.observe(a)
        assert e.value.status == mp.MPCD_ENOTFOUND
        c = ctx.admit(mp.make_desc(6, 2160, seed=3))
        assert c == a                        # slot reused
        ctx.step(2)
        assert ctx.observe(b)["step"] == 10 and ctx.observe(c)["step"] == 2


def test_admission_errors_leave_context_unchanged(mp):
    _say("errors")
    with mp.Context(hbm_budget=64 << 20, max_slots=2) as ctx:
        bad = mp.make_desc(8, 100)
        bad.L[1] = 0
        assert mp.mpcd_admit(ctx.handle, bad)[0] == mp.MPCD_EINVAL
        bad = mp.make_desc(8, 100, dt=-1.0)
        assert mp.mpcd_admit(ctx.handle, bad)[0] == mp.MPCD_EINVAL
        bad = mp.make_desc(8, 100)
        bad.flags = mp.MPCD_INIT_MAXWELL | mp.MPCD_INIT_EXTERNAL
        assert mp.mpcd_admit(ctx.handle, bad)[0] == mp.MPCD_EINVAL
        # over the 64 MiB budget
        assert ctx.try_admit(mp.make_desc(100, 10 ** 6)) is None
        s0 = ctx.admit(mp.make_desc(8, 5120, seed=1))
        s1 = ctx.admit(mp.make_desc(8, 5120, seed=2))
        assert mp.mpcd_admit(ctx.handle, mp.make_desc(8, 10))[0] == mp.MPCD_EBUSY
        ctx.step(3)
        assert ctx.observe(s0)["step"] == 3 and ctx.observe(s1)["step"] == 3
        # set_state rejects positions outside the box and non-finite values
        pos, vel = inputs.thermal_state(8, 5120, 1)
        p2 = pos.copy()
        p2[0, 5] = 8.0
        assert mp.mpcd_set_state(ctx.handle, s0, np.concatenate([p2, vel]), 0) == mp.MPCD_EINVAL
        v2 = vel.copy()
        v2[1, 7] = np.nan
        assert mp.mpcd_set_state(ctx.handle, s0, np.concatenate([pos, v2]), 0) == mp.MPCD_EINVAL
        assert ctx.observe(s0)["step"] == 3


def test_nonfinite_velocity_flags_only_its_box(mp):
    """A huge velocity overflows that box's energy to Inf; the other box in the
    batch stays healthy."""
    _say("nan-guard")
    with mp.Context() as ctx:
        a = ctx.admit(mp.make_desc(8, 5120, seed=1, init="external"))
        b = ctx.admit(mp.make_desc(8, 5120, seed=2))
        pos, vel = inputs.thermal_state(8, 5120, 1)
        vel[0, 10] = np.float32(3e38)
        ctx.set_state(a, (pos, vel))
        ctx.step(2)
        oa = ctx.observe(a)
        ob = ctx.observe(b)
    assert oa["status"] == mp.MPCD_ESTATE
    assert ob["status"] == mp.MPCD_OK and ob["step"] == 2


def test_admission_and_release_while_steps_are_queued(mp):
    """mpcd_admit queues a new box's initial state behind the steps already
    queued (nothing waits) and mpcd_release frees a box whose steps may still
    be queued: the other boxes' trajectories are unchanged, and the new box
    starts from the same initial state as in an idle context."""
    _say("queued-admission")
    descs = [dict(L=(20, 20, 20), n=80000, seed=51), dict(L=(16, 12, 10), n=19200, seed=52),
             dict(L=(10, 10, 10), n=10000, seed=53)]
    d = [mp.make_desc(x["L"], x["n"], seed=x["seed"]) for x in descs]
    with mp.Context() as ctx:
        a = ctx.admit(d[0])
        c = ctx.admit(d[2])
        ctx.step(10)           # queued, not waited for
        b = ctx.admit(d[1])    # joins at the next step
        ctx.release(c)
        ctx.step(10)
        sa, sb = ctx.get_state(a), ctx.get_state(b)
    with mp.Context() as ctx:
        a = ctx.admit(d[0])
        ctx.step(20)
        ra = ctx.get_state(a)
    with mp.Context() as ctx:
        b = ctx.admit(d[1])
        ctx.step(10)
        rb = ctx.get_state(b)
    assert sa[2] == ra[2] == 20 and sb[2] == rb[2] == 10
    assert np.array_equal(sa[0], ra[0]) and np.array_equal(sa[1], ra[1])
    assert np.array_equal(sb[0], rb[0]) and np.array_equal(sb[1], rb[1])


def test_random_box_mixes_match_sort(mp):
    """Seeded random batches of boxes (edges 1..40 per dimension, 0..20
    particles per cell, dt, alpha, per-particle masses, the angular-momentum
    rule, VACF) stepped together on bricks, with a box released and another
    admitted mid-run, end bit for bit where counting-sort binning ends."""
    _say("random-mixes")
    g = np.random.default_rng(2024)
    for trial in range(3):
        boxes = []
        for _ in range(6):
            L = tuple(int(x) for x in g.integers(1, 41, 3))
            n = int(g.integers(0, 21) * L[0] * L[1] * L[2] // 1 + g.integers(0, 5))
            boxes.append(dict(L=L, n=n, dt=float(g.uniform(0.05, 0.6)), alpha=float(g.uniform(30, 170)),
                              seed=int(g.integers(1, 1 << 40)), mass=bool(g.integers(0, 2)),
                              am=bool(g.integers(0, 4) == 0), vacf=bool(g.integers(0, 2))))
        res = {}
        for binning in (mp.MPCD_BIN_ATOMIC, mp.MPCD_BIN_SORT):
            with mp.Context(binning=binning) as ctx:
                slots = []
                for bx in boxes[:5]:
                    d = mp.make_desc(bx["L"], bx["n"], dt=bx["dt"], alpha_deg=bx["alpha"], seed=bx["seed"],
                                     particle_mass=bx["mass"], conserve_l=bx["am"],
                                     vacf_stride=3 if bx["vacf"] else 0)
                    slots.append(ctx.admit(d))
                ctx.step(4)
                ctx.release(slots[1])
                bx = boxes[5]
                slots[1] = ctx.admit(mp.make_desc(bx["L"], bx["n"], dt=bx["dt"], alpha_deg=bx["alpha"],
                                                  seed=bx["seed"], particle_mass=bx["mass"], conserve_l=bx["am"]))
                ctx.step(5)
                res[binning] = [(ctx.get_state(s), ctx.observe(s)) for s in slots]
        for i, ((sa, oa), (sb, ob)) in enumerate(zip(res[mp.MPCD_BIN_ATOMIC], res[mp.MPCD_BIN_SORT])):
            assert oa["status"] == ob["status"] == 0, (trial, i)
            assert sa[2] == sb[2], (trial, i)
            assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1]), (trial, i, boxes[i])
            assert np.array_equal(oa["vacf"], ob["vacf"]), (trial, i)
