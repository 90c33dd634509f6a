"""Parity at the benchmark's full size: 256^3 cells, 10 particles per cell
(167,772,160 particles), in the launch configuration bench.py times (no
particle ids, graph replay), and the same with counting-sort binning every
step.  The box first routes (or sorts) itself through three steps; then the oracle takes step 3 from the GPU's own state and recomputes
three whole slabs of collision cells (about 2 million particles), matched
with the GPU's particles by position."""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2212_11878_amd import inputs

from gpu_util import check_against, face_band_mask, match_unordered

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
@pytest.mark.parametrize("binning", ["bench", "sort"])
def test_full_size_step_after_self_routing_sampled_cells(binning):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_11878_amd import mpcd
    import bench

    L, n, seed, k = (256, 256, 256), 167772160, 3, 3
    print("[case] full-size inputs (%s)" % binning, flush=True)
    pos, vel = inputs.thermal_state(L, n, seed)
    print("[case] full-size gpu steps", flush=True)
    opts = bench.context_options() if binning == "bench" else dict(binning=mpcd.MPCD_BIN_SORT, use_graph=True)
    with mpcd.Context(**opts) as ctx:
        slot = ctx.admit(mpcd.make_desc(L, n, dt=0.1, alpha_deg=130.0, seed=seed, init="external",
                                        unordered=True))
        ctx.set_state(slot, (pos, vel))
        del pos, vel
        ctx.step(k)
        p3, v3, step = ctx.get_state(slot)
        assert step == k
        ctx.step(1)
        gp, gv, step = ctx.get_state(slot)
        obs = ctx.observe(slot)
    assert step == k + 1 and obs["status"] == 0
    assert obs["binning"] == (mpcd.MPCD_BIN_SORT if binning == "sort" else mpcd.MPCD_BIN_ATOMIC)
    print("[case] full-size oracle sample", flush=True)
    box = orc.make_box(L, dt=0.1, alpha_deg=130.0, seed=seed)
    st = orc.State(p3, v3)
    v3_64 = v3.astype(np.float64)
    del p3, v3
    orc.stream(box, st)
    s = orc.shift(seed, k, 1.0)
    cells = orc.cells(box, s, st)
    iz = cells // (256 * 256)
    iy = (cells // 256) % 256
    pick = np.nonzero((iz == 0) | (iz == 255) | (iy == 131))[0]
    sub = orc.State(st.pos[:, pick], st.vel[:, pick])
    # face-band particles anywhere may move into a sampled cell on the FP32 path
    near = face_band_mask(st.pos, s, box)
    band_pos, band_cells = st.pos[:, near].copy(), cells[near].copy()
    del st
    orc.collide(box, k, sub)
    # the GPU's particles of the same slabs (with a margin of one cell layer)
    gq = gp.astype(np.float64)
    gi = [np.floor((gq[d] - s[d])).astype(np.int64) % 256 for d in range(3)]
    cand = np.nonzero((gi[2] <= 1) | (gi[2] >= 254) | (np.abs(gi[1] - 131) <= 1))[0]
    del gq, gi
    mpos, mvel = match_unordered(sub.pos, gp[:, cand], gv[:, cand], L)
    band, err = check_against(sub, s, cells[pick], box, mpos, mvel, band_from=(band_pos, band_cells))
    print("[case] full-size sample after %d routed steps: %d particles, %d in face band, max rel err %.2e"
          % (k, len(pick), band, err), flush=True)
    assert len(pick) > 1_900_000
    # whole-box invariants of the GPU result
    assert gp.min() >= 0 and gp.max() < 256
    v1 = gv.astype(np.float64)
    P0, P1 = v3_64.sum(axis=1), v1.sum(axis=1)
    E0, E1 = 0.5 * np.sum(v3_64 * v3_64), 0.5 * np.sum(v1 * v1)
    assert np.all(np.abs(P1 - P0) < 1e-3 * math.sqrt(n))
    assert abs(E1 - E0) < 1e-6 * E0


@pytest.mark.timeout(600)
def test_brick_buffers_beyond_32bit_offsets():
    """A box whose brick buffers hold more than 2^30 slots (byte offsets past
    32 bits: 4.95e8 particles, 1.1e9 slots per buffer) runs on bricks with
    64-bit store offsets, and after a few steps its exact momentum and energy
    sums equal those of counting-sort binning bit for bit."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_11878_amd import mpcd
    L, seed = (384, 384, 336), 17
    n = 10 * L[0] * L[1] * L[2]
    obs = []
    for binning in (mpcd.MPCD_BIN_ATOMIC, mpcd.MPCD_BIN_SORT):
        print("[case] wide offsets, binning %d" % binning, flush=True)
        with mpcd.Context(binning=binning, brick=(8, 4, 4)) as ctx:
            slot = ctx.admit(mpcd.make_desc(L, n, dt=0.1, alpha_deg=130.0, seed=seed))
            ctx.step(5)
            obs.append(ctx.observe(slot))
        torch.cuda.empty_cache()
    a, b = obs
    print("[case] wide offsets: E %.17g / %.17g, overflow steps %d" % (a["E"], b["E"], a["overflow_steps"]),
          flush=True)
    assert a["binning"] == mpcd.MPCD_BIN_ATOMIC and b["binning"] == mpcd.MPCD_BIN_SORT
    assert a["step"] == b["step"] == 5 and a["status"] == b["status"] == 0
    assert a["E"] == b["E"] and np.array_equal(a["P"], b["P"])


@pytest.mark.timeout(600)
def test_full_size_drift_over_500_steps():
    """256^3 cells, 1.68e8 particles, 500 steps in the benchmark's launch
    configuration: SRD conserves momentum and kinetic energy exactly (the
    FP64 oracle holds them to its rounding), so the GPU's drift measures its
    own rounding: relative energy drift below 1e-6 and momentum drift below
    1e-8 N sqrt(kT/m)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_11878_amd import mpcd
    import bench
    L, n, seed = (256, 256, 256), 167772160, 3
    print("[case] full-size drift", flush=True)
    with mpcd.Context(**bench.context_options()) as ctx:
        slot = ctx.admit(mpcd.make_desc(L, n, dt=0.1, alpha_deg=130.0, seed=seed, unordered=True))
        o0 = ctx.observe(slot)
        ctx.step(500)
        o1 = ctx.observe(slot)
    print("[case] full-size drift: E0 %.15e E500 %.15e rel %.3e, |P0| %.3e |P500 - P0| %.3e" % (
        o0["E"], o1["E"], (o1["E"] - o0["E"]) / o0["E"], np.abs(o0["P"]).max(),
        np.abs(o1["P"] - o0["P"]).max()), flush=True)
    assert o1["step"] == 500 and o1["status"] == 0
    assert abs(o1["E"] - o0["E"]) / o0["E"] < 1e-6
    assert np.all(np.abs(o1["P"] - o0["P"]) < 1e-8 * n)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("ids", [True, False])
def test_100cube_one_step_every_particle(ids):
    """100^3 cells, 10^7 particles (the 100^3 workload) in the benchmark's
    launch configuration, with and without particle ids: one step from a
    seeded state against the oracle, for every particle (face-band
    exemptions as in the small cases; without ids the particles are matched
    by position)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_11878_amd import mpcd
    from gpu_util import oracle_one_step
    import bench
    L, n, seed, k = (100, 100, 100), 10_000_000, 2, 3
    print("[case] 100^3 inputs, ids=%s" % ids, flush=True)
    pos, vel = inputs.thermal_state(L, n, seed)
    with mpcd.Context(**bench.context_options()) as ctx:
        slot = ctx.admit(mpcd.make_desc(L, n, dt=0.1, alpha_deg=130.0, seed=seed, init="external",
                                        unordered=not ids))
        ctx.set_state(slot, (pos, vel), step=k)
        ctx.step(1)
        gp, gv, step = ctx.get_state(slot)
    assert step == k + 1
    print("[case] 100^3 oracle step", flush=True)
    box = orc.make_box(L, dt=0.1, alpha_deg=130.0, seed=seed)
    st, s, cells = oracle_one_step(pos, vel, box, k)
    if not ids:
        gp, gv = match_unordered(st.pos, gp, gv, L)
    band, err = check_against(st, s, cells, box, gp, gv)
    print("[case] 100^3: %d particles, %d in face band, max rel err %.2e" % (n, band, err), flush=True)
    assert band < n // 1000
