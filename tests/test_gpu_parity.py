"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded FP32 inputs, element by element."""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2212_11878_amd import inputs

from gpu_util import compare_step, f32_state

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


def _gpu_one_step(mp, binning, L, pos32, vel32, k, alpha_deg=130.0, dt=0.1, seed=1, a=1.0,
                  use_graph=True):
    with mp.Context(binning=binning, use_graph=use_graph) as ctx:
        d = mp.make_desc(L, pos32.shape[1], dt=dt, alpha_deg=alpha_deg, seed=seed, a=a,
                         init="external")
        slot = ctx.admit(d)
        ctx.set_state(slot, (pos32, vel32), step=k)
        ctx.step(1)
        pos, vel, step = ctx.get_state(slot)
        assert step == k + 1
    return pos, vel


@pytest.mark.parametrize("binning", ["atomic", "sort"])
@pytest.mark.parametrize("k", [0, 1, 37, 99, (1 << 32) + 5])
def test_one_step_parity_small_box(mp, binning, k):
    """10^3 cells, 10 particles per cell, alpha 130 deg, dt 0.1, seed 1; the
    state at step k comes from the oracle's own FP64 trajectory."""
    mode = mp.MPCD_BIN_ATOMIC if binning == "atomic" else mp.MPCD_BIN_SORT
    L = (10, 10, 10)
    _say("one_step", binning, k)
    pos, vel = inputs.thermal_state(L, 10000, seed=1)
    box = orc.make_box(L, dt=0.1, alpha_deg=130.0, seed=1)
    if 0 < k < 200:
        st = orc.State(pos, vel)
        orc.run(box, 0, k, st)
        pos, vel = f32_state(st.pos, st.vel, L)
    gp, gv = _gpu_one_step(mp, mode, L, pos, vel, k)
    compare_step(pos, vel, gp, gv, box, k)


@pytest.mark.parametrize("case", [
    dict(L=(7, 3, 11), n=2311, a=1.0, alpha=90.0, dt=0.1),      # non-cubic, ragged tile
    dict(L=(16, 16, 16), n=4096 * 9 + 37, a=1.0, alpha=120.0, dt=0.2),
    dict(L=(5, 6, 4), n=1800, a=0.5, alpha=150.0, dt=0.05),     # cell edge != 1
    dict(L=(4, 4, 4), n=640, a=1.5, alpha=130.0, dt=1.0),       # long free path
    dict(L=(1, 1, 1), n=50, a=1.0, alpha=130.0, dt=0.1),        # one cell
    dict(L=(200, 1, 1), n=3000, a=1.0, alpha=130.0, dt=0.1),    # thin box
])
@pytest.mark.parametrize("binning", ["atomic", "sort"])
def test_one_step_parity_shapes(mp, case, binning):
    mode = mp.MPCD_BIN_ATOMIC if binning == "atomic" else mp.MPCD_BIN_SORT
    _say("shapes", binning, case)
    L = case["L"]
    pos, vel = inputs.thermal_state(L, case["n"], seed=17, a=case["a"])
    box = orc.make_box(L, a=case["a"], dt=case["dt"], alpha_deg=case["alpha"], seed=99)
    gp, gv = _gpu_one_step(mp, mode, L, pos, vel, 3, alpha_deg=case["alpha"], dt=case["dt"],
                           seed=99, a=case["a"])
    compare_step(pos, vel, gp, gv, box, 3)


def test_particles_on_faces_and_edges(mp):
    """Positions exactly on cell faces of the unshifted grid and at the box
    edge, and velocities that carry particles across the periodic boundary."""
    _say("faces")
    L = (6, 6, 6)
    g = np.random.default_rng(3)
    n = 2000
    pos = g.integers(0, 6, size=(3, n)).astype(np.float32)        # on faces
    pos[:, :100] = np.float32(np.nextafter(np.float32(6.0), np.float32(0)))  # top edge
    vel = g.standard_normal((3, n)).astype(np.float32)
    vel[:, :50] = 3.0
    box = orc.make_box(L, seed=5)
    gp, gv = _gpu_one_step(mp, mp.MPCD_BIN_ATOMIC, L, pos, vel, 0, seed=5)
    compare_step(pos, vel, gp, gv, box, 0)


def test_empty_and_single_particle_boxes(mp):
    _say("empty")
    with mp.Context() as ctx:
        s0 = ctx.admit(mp.make_desc((4, 4, 4), 0, init="external"))
        s1 = ctx.admit(mp.make_desc((4, 4, 4), 1, init="external", seed=2))
        ctx.set_state(s1, (np.array([[1.5], [2.5], [3.5]], np.float32),
                           np.array([[0.3], [-0.2], [0.1]], np.float32)))
        ctx.step(3)
        o0 = ctx.observe(s0)
        assert o0["step"] == 3 and o0["n"] == 0
        pos, vel, step = ctx.get_state(s1)
        assert step == 3
        # a lone particle keeps its velocity (relative velocity zero)
        assert np.allclose(vel[:, 0], [0.3, -0.2, 0.1], atol=1e-7)
        assert np.allclose(pos[:, 0], [1.5 + 0.09, 2.5 - 0.06, 3.5 + 0.03], atol=1e-5)


@pytest.mark.parametrize("binning", ["atomic", "sort"])
def test_one_step_parity_particle_masses(mp, binning):
    """Per-particle masses: the cell velocity is sum(m v)/sum(m) (Listing 4)."""
    mode = mp.MPCD_BIN_ATOMIC if binning == "atomic" else mp.MPCD_BIN_SORT
    _say("masses", binning)
    L, n, k = (9, 8, 7), 5040, 2
    pos, vel = inputs.thermal_state(L, n, seed=23)
    mass = np.random.default_rng(23).uniform(0.25, 4.0, n).astype(np.float32)
    box = orc.make_box(L, dt=0.1, alpha_deg=130.0, seed=23)
    with mp.Context(binning=mode) as ctx:
        s = ctx.admit(mp.make_desc(L, n, seed=23, init="external", particle_mass=True))
        ctx.set_state(s, (pos, vel), step=k)
        ctx.set_mass(s, mass)
        o0 = ctx.observe(s)
        ctx.step(1)
        gp, gv, _ = ctx.get_state(s)
    assert abs(o0["M"] - float(np.sum(mass.astype(np.float64)))) < 1e-6
    compare_step(pos, vel, gp, gv, box, k, mass32=mass, kT=1.0)


def test_masses_follow_their_particles(mp):
    """Masses travel with particles through re-bucketing and survive
    set_state: after 10 steps, reloading the state and stepping once more
    matches the oracle with the same per-id masses."""
    _say("masses-travel")
    L, n = (10, 10, 10), 10000
    pos, vel = inputs.thermal_state(L, n, seed=29)
    mass = np.random.default_rng(29).uniform(0.5, 2.0, n).astype(np.float32)
    box = orc.make_box(L, dt=0.1, alpha_deg=130.0, seed=29)
    st = orc.State(pos, vel, mass)
    orc.run(box, 0, 10, st)
    p10, v10 = f32_state(st.pos, st.vel, L)
    with mp.Context(binning=mp.MPCD_BIN_ATOMIC) as ctx:
        s = ctx.admit(mp.make_desc(L, n, seed=29, init="external", particle_mass=True))
        ctx.set_state(s, (pos, vel))
        ctx.set_mass(s, mass)
        ctx.step(10)
        ctx.set_state(s, (p10, v10), step=10)     # masses must stay with the ids
        ctx.step(1)
        gp, gv, _ = ctx.get_state(s)
        o = ctx.observe(s)
    compare_step(p10, v10, gp, gv, box, 10, mass32=mass)
    P, E, T, M = orc.diagnostics(orc.State(gp, gv, mass))
    assert np.allclose(o["P"], P, rtol=0, atol=1e-6) and abs(o["E"] - E) < 1e-8 * E
    assert abs(o["T"] - T) < 1e-8 * T
