"""Pins for the oracle's collision step (paper Sec. 2; mass-weighted cell
velocity as in Listing 4) against hand-worked values, textbook properties of
rotations and the conservation laws the method guarantees."""
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _worked_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "worked_cell.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([float(t) for t in line.split()])
    return np.array(rows)


def _one_cell_state(orc, vel, pos=None, mass=None):
    vel = np.asarray(vel, dtype=np.float64).T.copy()
    n = vel.shape[1]
    if pos is None:
        pos = np.full((3, n), 0.5)
    return orc.State(pos, vel, mass)


def test_worked_example_three_particles(orc):
    rows = _worked_rows()
    box = orc.make_box(1, alpha_deg=90.0)
    st = _one_cell_state(orc, rows[:, 0:3])
    orc.collide_given(box, np.zeros(3), [0.0, 0.0, 1.0], st)
    assert np.allclose(st.vel.T, rows[:, 3:6], rtol=0, atol=1e-14)
    assert np.allclose(st.vel.sum(axis=1), [3, 3, 3], atol=1e-14)
    assert abs(np.sum(st.vel ** 2) - 19.0) < 1e-13


def test_half_turn_and_identity(orc):
    g = np.random.default_rng(1)
    v = g.standard_normal((7, 3))
    u = v.mean(axis=0)
    w = v - u
    # 180 degrees about e_x: (w_x, -w_y, -w_z)
    box = orc.make_box(1, alpha_deg=180.0)
    st = _one_cell_state(orc, v)
    orc.collide_given(box, np.zeros(3), [1.0, 0.0, 0.0], st)
    assert np.allclose(st.vel.T, u + w * np.array([1, -1, -1]), atol=1e-14)
    # 0 and 360 degrees: identity
    for deg in (0.0, 360.0):
        box = orc.make_box(1, alpha_deg=deg)
        st = _one_cell_state(orc, v)
        orc.collide_given(box, np.zeros(3), [0.6, 0.0, 0.8], st)
        assert np.allclose(st.vel.T, v, atol=1e-13)


def test_rotation_is_proper_and_keeps_axis(orc):
    g = np.random.default_rng(2)
    for _ in range(50):
        n = g.standard_normal(3)
        n /= np.linalg.norm(n)
        alpha = g.uniform(0, 2 * math.pi)
        R = np.column_stack([orc.rotate(n, alpha, e) for e in np.eye(3)])
        assert np.allclose(R.T @ R, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1.0) < 1e-14
        assert np.allclose(R @ n, n, atol=1e-14)
        # the perpendicular part turns by alpha, right handed about n
        w = g.standard_normal(3)
        wp = w - n * (n @ w)
        rp = R @ wp
        cosang = (wp @ rp) / (wp @ wp)
        sinang = (np.cross(wp, rp) @ n) / (wp @ wp)
        assert abs(cosang - math.cos(alpha)) < 1e-13
        assert abs(sinang - math.sin(alpha)) < 1e-13


def test_single_particle_cell_unchanged(orc):
    box = orc.make_box(1, alpha_deg=130.0)
    st = _one_cell_state(orc, [[0.3, -1.2, 2.0]])
    orc.collide_given(box, np.zeros(3), [0.0, 1.0, 0.0], st)
    assert np.allclose(st.vel[:, 0], [0.3, -1.2, 2.0], atol=1e-15)


def _random_state(orc, L, n, seed, mass=False):
    g = np.random.default_rng(seed)
    pos = g.random((3, n)) * L
    vel = g.standard_normal((3, n))
    m = g.uniform(0.5, 2.0, n) if mass else None
    return orc.State(pos, vel, m)


def test_per_cell_momentum_and_energy_conserved(orc):
    for use_mass in (False, True):
        box = orc.make_box(6, alpha_deg=130.0, seed=9)
        st = _random_state(orc, 6, 3000, 4, mass=use_mass)
        s = orc.shift(box.seed, 3, box.a)
        m = st.mass if use_mass else np.ones(st.n)
        cnt0, P0, M0 = orc.cell_sums(box, s, st)
        cells = np.array([orc.cell_of(box, s, *st.pos[:, i]) for i in range(st.n)])
        E0 = np.bincount(cells, weights=m * np.sum(st.vel ** 2, axis=0), minlength=216)
        orc.collide(box, 3, st)
        cnt1, P1, M1 = orc.cell_sums(box, s, st)
        E1 = np.bincount(cells, weights=m * np.sum(st.vel ** 2, axis=0), minlength=216)
        assert np.array_equal(cnt0, cnt1)
        scale = np.sqrt(np.maximum(E0, 1e-300) * np.maximum(M0, 1e-300))
        assert np.all(np.abs(P1 - P0) <= 1e-13 * scale[:, None] + 1e-15)
        assert np.all(np.abs(E1 - E0) <= 1e-13 * E0 + 1e-15)


def test_galilean_invariance(orc):
    """Collision of v + V equals (collision of v) + V, same positions/bins."""
    box = orc.make_box(5, alpha_deg=120.0, seed=3)
    st = _random_state(orc, 5, 2000, 5)
    V = np.array([0.7, -1.3, 0.25])
    st2 = orc.State(st.pos, st.vel + V[:, None])
    orc.collide(box, 2, st)
    orc.collide(box, 2, st2)
    assert np.allclose(st2.vel, st.vel + V[:, None], rtol=0, atol=1e-12)


def test_order_invariance(orc):
    """Storage order changes nothing but the rounding order of the FP64 cell
    sums: random numbers are keyed by cell, never by storage index."""
    box = orc.make_box(4, alpha_deg=130.0, seed=12)
    st = _random_state(orc, 4, 900, 6)
    perm = np.random.default_rng(0).permutation(st.n)
    stp = orc.State(st.pos[:, perm], st.vel[:, perm])
    orc.step(box, 7, st)
    orc.step(box, 7, stp)
    assert np.array_equal(stp.pos, st.pos[:, perm])
    assert np.allclose(stp.vel, st.vel[:, perm], rtol=0, atol=1e-13)


def test_global_conservation_over_steps(orc):
    box = orc.make_box(8, alpha_deg=130.0, seed=1)
    st = _random_state(orc, 8, 5120, 8)
    P0, E0, _, _ = orc.diagnostics(st)
    orc.run(box, 0, 50, st)
    P1, E1, _, _ = orc.diagnostics(st)
    assert np.all(np.abs(P1 - P0) < 1e-11 * math.sqrt(st.n))
    assert abs(E1 - E0) < 1e-12 * E0


def test_temperature_definition(orc):
    """T uses 3(N-1) degrees of freedom and the centre-of-mass frame."""
    vel = np.array([[1.0, -1.0, 0.0], [0.0, 0.0, 2.0], [0.0, 0.0, 0.0]]).T
    st = orc.State(np.zeros((3, 3)), vel.T.copy() + 5.0)
    P, E, T, M = orc.diagnostics(st)
    w = vel.T - vel.T.mean(axis=1, keepdims=True)
    assert abs(T - np.sum(w ** 2) / 6.0) < 1e-14
    assert M == 3.0
