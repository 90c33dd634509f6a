"""GPU parity of the angular-momentum-conserving collision (MPCD_CONSERVE_L)
against the oracle's rule, and its conservation laws on the GPU state."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2212_11878_amd import inputs

from gpu_util import check_against, ulp_top

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_11878_amd import mpcd
    return mpcd


def _ill_conditioned_cells(box, s, st, cells, limit=1e4):
    """Cells whose inertia tensor I (about the centre of mass) has a condition
    number above `limit` (three or more almost collinear particles).  The GPU
    sums the position moments as fixed-point terms rounded to 2^-32 (relative
    error about 1e-9 of I and of the angular-momentum change dL), and
    omega = -I^+ dL amplifies a relative error of I or dL by up to cond(I), so
    the rigid-rotation velocity omega x r' is held to 1e-5 only where
    cond(I) 1e-9 stays below 1e-5: cond(I) <= 1e4.  Rank-deficient cells
    (one or two particles, exactly collinear) are not exempt: their
    pseudo-inverse drops the null direction on both sides."""
    bad = set()
    order = np.argsort(cells, kind="stable")
    cs = cells[order]
    starts = np.flatnonzero(np.r_[True, cs[1:] != cs[:-1]])
    ends = np.r_[starts[1:], len(cs)]
    for a, b in zip(starts, ends):
        idx = order[a:b]
        if len(idx) < 3:
            continue
        r = np.array([orc.cell_local(box, s, *st.pos[:, i]) for i in idx])
        rp = r - r.mean(axis=0)
        Q = rp.T @ rp
        I = np.trace(Q) * np.eye(3) - Q
        e = np.linalg.eigvalsh(I)
        if e[0] < e[-1] / limit:
            bad.add(int(cs[a]))
    return bad


@pytest.mark.parametrize("binning", ["atomic", "sort"])
@pytest.mark.parametrize("case", [
    dict(L=(8, 8, 8), n=5120, alpha=130.0, k=0, mass=False),
    dict(L=(6, 9, 5), n=2700, alpha=90.0, k=7, mass=True),
])
def test_one_step_parity_am(mp, case, binning):
    """One step of the angular-momentum rule.  Streaming is checked on its own
    (GPU positions within 1 ulp of the oracle's streamed FP64 positions); the
    collision is then checked with the oracle colliding at the GPU's streamed
    positions, so that an ill-conditioned inertia tensor does not amplify the
    FP32 rounding of the positions (only of the exact sums; see
    _ill_conditioned_cells)."""
    print("[case] am", binning, case, flush=True)
    L, n = case["L"], case["n"]
    pos, vel = inputs.thermal_state(L, n, seed=41)
    mass = np.random.default_rng(41).uniform(0.5, 2.0, n).astype(np.float32) if case["mass"] else None
    bin_id = mp.MPCD_BIN_ATOMIC if binning == "atomic" else mp.MPCD_BIN_SORT
    with mp.Context(binning=bin_id, brick=(4, 4, 4)) as ctx:
        s = ctx.admit(mp.make_desc(L, n, alpha_deg=case["alpha"], seed=41, init="external",
                                   conserve_l=True, particle_mass=case["mass"]))
        ctx.set_state(s, (pos, vel), step=case["k"])
        if mass is not None:
            ctx.set_mass(s, mass)
        ctx.step(1)
        gp, gv, _ = ctx.get_state(s)
    box = orc.make_box(L, alpha_deg=case["alpha"], seed=41)
    m64 = None if mass is None else mass.astype(np.float64)
    # streaming: the GPU's positions against the oracle's
    ref = orc.State(pos, vel, m64)
    orc.stream(box, ref)
    edge = np.array(L, dtype=np.float64)[:, None]
    dpos = gp.astype(np.float64) - ref.pos
    dpos -= np.round(dpos / edge) * edge
    assert np.max(np.abs(dpos)) <= ulp_top(max(L))
    # collision at the GPU's streamed positions
    st = orc.State(gp.astype(np.float64), vel.astype(np.float64), m64)
    sh = orc.shift(41, case["k"], 1.0)
    cells = orc.cells(box, sh, st)
    orc.collide_am(box, case["k"], st)
    bad = _ill_conditioned_cells(box, sh, st, cells)
    keep = ~np.isin(cells, np.fromiter(bad, dtype=np.int64, count=len(bad)))
    print("[case] am: %d of %d particles in cells with cond(I) > 1e4" % (n - keep.sum(), n), flush=True)
    assert keep.sum() > 0.995 * n
    sub = orc.State(st.pos[:, keep], st.vel[:, keep])
    check_against(sub, sh, cells[keep], box, gp[:, keep], gv[:, keep])


@pytest.mark.parametrize("binning", ["atomic", "sort"])
def test_am_is_deterministic_alone_and_in_mix(mp, binning):
    print("[case] am-mix", binning, flush=True)
    boxes = [((8, 8, 8), 5120, 3), ((5, 7, 6), 2100, 4)]
    states = {}
    bin_id = mp.MPCD_BIN_ATOMIC if binning == "atomic" else mp.MPCD_BIN_SORT
    for mix in (False, True):
        with mp.Context(binning=bin_id) as ctx:
            slots = []
            for (L, n, seed) in (boxes if mix else boxes[:1]):
                pos, vel = inputs.thermal_state(L, n, seed)
                sl = ctx.admit(mp.make_desc(L, n, seed=seed, init="external", conserve_l=True))
                ctx.set_state(sl, (pos, vel))
                slots.append(sl)
            ctx.step(20)
            states[mix] = ctx.get_state(slots[0])
    assert np.array_equal(states[False][0], states[True][0])
    assert np.array_equal(states[False][1], states[True][1])


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


@pytest.mark.parametrize("mass", [False, True])
def test_am_bricks_match_sort_through_overflow(mp, mass):
    """The brick form of the angular-momentum rule (moments and angular
    momentum summed in LDS, overflow particles read directly by their flagged
    bricks) gives the counting-sort form's trajectory bit for bit, also while
    a dense drifting slab overflows buckets."""
    print("[case] am-overflow mass=%s" % mass, flush=True)
    L, n = (16, 16, 16), 20000
    pos, vel = _slab(n, 33, 4.0)
    m = np.random.default_rng(33).uniform(0.5, 2.0, n).astype(np.float32) if mass else None
    out, obs = [], []
    for binning in (mp.MPCD_BIN_ATOMIC, mp.MPCD_BIN_SORT):
        with mp.Context(binning=binning, brick=(4, 4, 4)) as ctx:
            s = ctx.admit(mp.make_desc(L, n, dt=0.1, seed=33, init="external", conserve_l=True,
                                       particle_mass=mass))
            ctx.set_state(s, (pos, vel))
            if m is not None:
                ctx.set_mass(s, m)
            for _ in range(8):
                ctx.step(3)
            out.append(ctx.get_state(s))
            obs.append(ctx.observe(s))
    print("[am-overflow] binning %d/%d, steps with overflow %d, re-bucketings %d" % (
        obs[0]["binning"], obs[1]["binning"], obs[0]["overflow_steps"], obs[0]["rebuckets"]), flush=True)
    assert obs[0]["binning"] == mp.MPCD_BIN_ATOMIC and obs[1]["binning"] == mp.MPCD_BIN_SORT
    assert obs[0]["overflow_steps"] > 0 and obs[0]["rebuckets"] >= 2
    assert out[0][2] == out[1][2] == 24
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert obs[0]["E"] == obs[1]["E"] and np.array_equal(obs[0]["P"], obs[1]["P"])


def test_am_and_plain_boxes_share_a_launch(mp):
    """Brick boxes with the angular-momentum rule, with per-particle masses
    and plain ones advance in one launch; each ends where it ends alone."""
    print("[case] am-plain-mix", flush=True)
    boxes = [dict(L=(8, 8, 8), n=5120, seed=5, am=True, mass=False),
             dict(L=(12, 10, 8), n=9600, seed=6, am=False, mass=True),
             dict(L=(9, 9, 9), n=7290, seed=7, am=False, mass=False),
             dict(L=(10, 8, 6), n=4800, seed=8, am=True, mass=True)]

    def run(sel):
        res = []
        with mp.Context(binning=mp.MPCD_BIN_ATOMIC, brick=(4, 4, 4)) as ctx:
            slots = []
            for bx in sel:
                pos, vel = inputs.thermal_state(bx["L"], bx["n"], bx["seed"])
                sl = ctx.admit(mp.make_desc(bx["L"], bx["n"], seed=bx["seed"], init="external",
                                            conserve_l=bx["am"], particle_mass=bx["mass"]))
                ctx.set_state(sl, (pos, vel))
                if bx["mass"]:
                    ctx.set_mass(sl, np.random.default_rng(bx["seed"]).uniform(0.5, 2.0, bx["n"]).astype(np.float32))
                slots.append(sl)
            ctx.step(15)
            for sl in slots:
                res.append(ctx.get_state(sl))
        return res

    together = run(boxes)
    for i, bx in enumerate(boxes):
        alone = run([bx])[0]
        assert alone[2] == together[i][2] == 15
        assert np.array_equal(alone[0], together[i][0]) and np.array_equal(alone[1], together[i][1]), i
