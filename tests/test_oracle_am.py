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
    """The closed-form pseudo-inverse against numpy's SVD-based pinv (same
    cut: singular values at most 1e-10 of the largest count as zero) on
    random symmetric matrices of every rank, positive semi-definite and
    indefinite, over several scales."""
    g = np.random.default_rng(4)
    for trial in range(200):
        rank = trial % 4
        B = g.standard_normal((3, rank))
        D = np.diag(g.choice([-1.0, 1.0], rank)) if trial % 8 >= 4 else np.eye(rank)
        A = (B @ D @ B.T) * 10.0 ** g.uniform(-3, 3)
        ref = np.linalg.pinv(A, rcond=1e-10, hermitian=True)
        got = orc.sym3_pinv(A)
        scale = max(1.0, np.abs(ref).max())
        assert np.allclose(got, ref, rtol=1e-7, atol=1e-8 * scale), (trial, rank, A, got, ref)


def test_pseudo_inverse_closed_forms(orc):
    """Cases with a known answer: the inertia tensor of a collinear cell,
    I = q (1 - d d^T), has I^+ = (1 - d d^T)/q (rank 2 with a degenerate kept
    pair); an isotropic tensor c 1 inverts to 1/c (triple eigenvalue); a
    diagonal matrix inverts entry by entry; the Moore-Penrose identities
    A A^+ A = A and A^+ A A^+ = A^+ hold with A A^+ symmetric."""
    g = np.random.default_rng(5)
    for _ in range(50):
        d = g.standard_normal(3)
        d /= np.linalg.norm(d)
        q = 10.0 ** g.uniform(-2, 2)
        P = np.eye(3) - np.outer(d, d)
        assert np.allclose(orc.sym3_pinv(q * P), P / q, rtol=1e-9, atol=1e-9 / q)
        c = 10.0 ** g.uniform(-2, 2)
        assert np.allclose(orc.sym3_pinv(c * np.eye(3)), np.eye(3) / c, rtol=1e-12)
        e = g.uniform(0.1, 5.0, 3)
        assert np.allclose(orc.sym3_pinv(np.diag(e)), np.diag(1.0 / e), rtol=1e-12)
        B = g.standard_normal((3, 3))
        A = B @ B.T
        Ap = orc.sym3_pinv(A)
        assert np.allclose(A @ Ap @ A, A, atol=1e-9 * np.abs(A).max())
        assert np.allclose(Ap @ A @ Ap, Ap, atol=1e-9 * np.abs(Ap).max())
        assert np.allclose(A @ Ap, (A @ Ap).T, atol=1e-9)
    assert np.all(orc.sym3_pinv(np.zeros((3, 3))) == 0.0)


def test_cell_local_against_brute_force(orc):
    """Position inside the shifted collision cell at nonzero shifts and
    a != 1: the test finds the cell by a point-in-shifted-cube search over
    every periodic image, independently of the oracle, and expects
    r_d = x_d - s_d - a i_d for the image that contains the particle."""
    g = np.random.default_rng(12)
    for trial in range(300):
        L = tuple(int(v) for v in g.integers(1, 5, 3))
        a = float(g.choice([1.0, 0.5, 1.75]))
        box = orc.make_box(L, a=a)
        s = g.uniform(-a / 2, a / 2, 3)
        x = g.uniform(0, 1, 3) * np.array(L) * a
        want = np.zeros(3)
        for d in range(3):
            hits = [x[d] + m * L[d] * a - s[d] - a * i
                    for m in (-1, 0, 1) for i in range(L[d])
                    if a * i + s[d] <= x[d] + m * L[d] * a < a * (i + 1) + s[d]]
            assert len(hits) == 1, (trial, d, hits)
            want[d] = hits[0]
        got = orc.cell_local(box, s, *x)
        assert np.all(got >= 0) and np.all(got < a)
        assert np.allclose(got, want, atol=1e-12), (trial, L, a, s, x, got, want)


def _cell_moments(orc, box, s, st, cells):
    """Per-cell momentum and angular momentum about the cell's centre of mass.
    Positions inside the shifted cells are computed here with numpy (the
    shifted coordinate folded into the box, minus the cell's lower corner),
    not with the oracle's own cell_local."""
    C = orc.n_cells(box)
    m = st.mass if st.mass is not None else np.ones(st.n)
    Lvec = np.array([box.L[d] for d in range(3)], dtype=np.float64) * box.a
    q = np.mod(st.pos - np.asarray(s)[:, None], Lvec[:, None])
    r = q - box.a * np.floor(q / box.a)
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
