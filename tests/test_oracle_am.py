"""Pins for the oracle's angular-momentum-conserving collision (SRD+a)."""
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _rows():
    rows = []
    with open(os.path.join(HERE, "golden", "worked_cell_am.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([float(t) for t in line.split()])
    return np.array(rows)


def test_worked_pair(orc):
    r = _rows()
    box = orc.make_box(1, alpha_deg=90.0)
    st = orc.State(r[:, 0:3].T, r[:, 3:6].T)
    orc.collide_am_given(box, np.zeros(3), [0.0, 0.0, 1.0], st)
    assert np.allclose(st.vel.T, r[:, 6:9], atol=1e-12)


def test_pseudo_inverse_matches_numpy(orc):
    g = np.random.default_rng(4)
    for rank in (3, 2, 1, 0):
        B = g.standard_normal((3, rank))
        A = B @ B.T
        assert np.allclose(orc.sym3_pinv(A), np.linalg.pinv(A, rcond=1e-10, hermitian=True), atol=1e-9)


def _cell_moments(orc, box, s, st, cells):
    """Per-cell momentum and angular momentum about the cell's centre of mass."""
    C = orc.n_cells(box)
    m = st.mass if st.mass is not None else np.ones(st.n)
    r = np.array([orc.cell_local(box, s, *st.pos[:, i]) for i in range(st.n)]).T
    M = np.bincount(cells, weights=m, minlength=C)
    rcm = np.stack([np.bincount(cells, weights=m * r[d], minlength=C) for d in range(3)]) / np.maximum(M, 1e-300)
    rp = r - rcm[:, cells]
    P = np.stack([np.bincount(cells, weights=m * st.vel[d], minlength=C) for d in range(3)])
    Lp = np.cross(rp.T, st.vel.T).T * m
    Lc = np.stack([np.bincount(cells, weights=Lp[d], minlength=C) for d in range(3)])
    return P, Lc


def test_conserves_momentum_and_angular_momentum(orc):
    g = np.random.default_rng(6)
    for use_mass in (False, True):
        L = (4, 5, 3)
        n = 600
        box = orc.make_box(L, alpha_deg=130.0, seed=77)
        pos = g.random((3, n)) * np.array(L)[:, None]
        vel = g.standard_normal((3, n))
        mass = g.uniform(0.5, 2.0, n) if use_mass else None
        st = orc.State(pos, vel, mass)
        s = orc.shift(box.seed, 5, box.a)
        cells = orc.cells(box, s, st)
        P0, L0 = _cell_moments(orc, box, s, st, cells)
        E0 = np.sum((mass if use_mass else 1.0) * st.vel ** 2)
        orc.collide_am(box, 5, st)
        P1, L1 = _cell_moments(orc, box, s, st, cells)
        E1 = np.sum((mass if use_mass else 1.0) * st.vel ** 2)
        assert np.allclose(P1, P0, atol=1e-12)
        assert np.allclose(L1, L0, atol=1e-12)
        assert abs(E1 - E0) > 1e-6 * E0          # the rule does not conserve energy


def test_identity_at_zero_angle_and_galilean(orc):
    g = np.random.default_rng(8)
    L = (3, 3, 3)
    pos = g.random((3, 300)) * 3
    vel = g.standard_normal((3, 300))
    box0 = orc.make_box(L, alpha_deg=0.0, seed=2)
    st = orc.State(pos, vel)
    orc.collide_am(box0, 1, st)
    assert np.allclose(st.vel, vel, atol=1e-12)
    box = orc.make_box(L, alpha_deg=120.0, seed=2)
    a = orc.State(pos, vel)
    V = np.array([0.3, -2.0, 1.1])
    bshift = orc.State(pos, vel + V[:, None])
    orc.collide_am(box, 4, a)
    orc.collide_am(box, 4, bshift)
    assert np.allclose(bshift.vel, a.vel + V[:, None], atol=1e-11)
