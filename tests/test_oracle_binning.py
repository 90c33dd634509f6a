"""Pins for streaming, the shifted grid and per-cell sums of the oracle,
checked by brute force on tiny boxes (Sec. 3.1, Listing 1: cell of x is
floor((x - s)/a) on the grid displaced by the random offset s; Listing 4:
per-cell sums of m v and of m)."""
import itertools
import math

import numpy as np


def _brute_cell(L, a, s, p):
    """Try every cell and every periodic image; the particle must lie in the
    half-open cube [i a + s, (i+1) a + s) of exactly one cell."""
    hits = []
    for idx in itertools.product(range(L[0]), range(L[1]), range(L[2])):
        for img in itertools.product((-1, 0, 1), repeat=3):
            q = [p[d] + img[d] * L[d] * a for d in range(3)]
            if all(idx[d] * a + s[d] <= q[d] < (idx[d] + 1) * a + s[d] for d in range(3)):
                hits.append(idx[0] + L[0] * (idx[1] + L[1] * idx[2]))
    return hits


def test_binning_matches_brute_force(orc):
    g = np.random.default_rng(5)
    for L, a in [((2, 2, 2), 1.0), ((3, 4, 2), 1.0), ((4, 4, 4), 0.75), ((2, 3, 4), 1.5)]:
        box = orc.make_box(L, a=a, seed=int(g.integers(1, 1 << 40)))
        for k in range(3):
            s = orc.shift(box.seed, k, a)
            pts = g.random((40, 3)) * np.array(L) * a
            for p in pts:
                hits = _brute_cell(L, a, s, p)
                assert len(set(hits)) == 1
                assert orc.cell_of(box, s, *p) == hits[0]


def test_face_goes_to_upper_cell(orc):
    box = orc.make_box(4, seed=3)
    s = np.array([0.25, -0.375, 0.0])
    # exactly on the plane between cells 1 and 2 along x (x - s_x = 2)
    c = orc.cell_of(box, s, 2.25, 1.0, 1.0)
    ix = c % 4
    assert ix == 2
    # x - s = -0.375 + 0 ... wraps to the last cell
    c = orc.cell_of(box, s, 0.0, 0.2, 0.0)
    assert (c // 4) % 4 == 0       # y: 0.2 + 0.375 = 0.575 -> cell 0
    assert c % 4 == 3              # x: -0.25 -> cell -1 -> 3


def test_cell_sums_brute_force(orc):
    g = np.random.default_rng(7)
    L = (3, 2, 4)
    box = orc.make_box(L, seed=99)
    n = 50
    pos = g.random((3, n)) * np.array(L)[:, None]
    vel = g.standard_normal((3, n))
    mass = g.uniform(0.5, 3.0, n)
    st = orc.State(pos, vel, mass)
    s = orc.shift(box.seed, 4, 1.0)
    count, P, M = orc.cell_sums(box, s, st)
    C = 24
    bc = np.zeros(C, dtype=np.int64)
    bP = np.zeros((C, 3))
    bM = np.zeros(C)
    for c in range(C):                 # O(N C) double loop
        for i in range(n):
            if _brute_cell(L, 1.0, s, pos[:, i])[0] == c:
                bc[c] += 1
                bP[c] += mass[i] * vel[:, i]
                bM[c] += mass[i]
    assert np.array_equal(count, bc)
    assert np.allclose(P, bP, rtol=0, atol=1e-13)
    assert np.allclose(M, bM, rtol=0, atol=1e-13)
    assert count.sum() == n


def test_streaming_closed_form(orc):
    """With alpha = 0 the collision is the identity, so after k steps
    x = x0 + k v0 dt folded into the box."""
    L = (5, 6, 7)
    box = orc.make_box(L, dt=0.13, alpha_deg=0.0, seed=2)
    g = np.random.default_rng(8)
    n = 400
    pos0 = g.random((3, n)) * np.array(L)[:, None]
    vel0 = 3 * g.standard_normal((3, n))
    st = orc.State(pos0, vel0)
    k = 40
    orc.run(box, 0, k, st)
    want = np.mod(pos0 + k * 0.13 * vel0, np.array(L, dtype=float)[:, None])
    d = st.pos - want
    d -= np.round(d / np.array(L)[:, None]) * np.array(L)[:, None]   # torus distance
    assert np.max(np.abs(d)) < 1e-11
    assert np.allclose(st.vel, vel0, atol=1e-12)
    assert st.pos.min() >= 0 and np.all(st.pos < np.array(L)[:, None])


def test_wrap_edge_cases(orc):
    box = orc.make_box((2, 2, 2), dt=1.0, alpha_deg=0.0)
    # tiny negative step lands just below 0 and must fold to [0, L)
    st = orc.State(np.array([[0.0], [1.0], [1.999999999999]]),
                   np.array([[-1e-300], [2.0], [1e-12]]))
    orc.stream(box, st)
    assert 0.0 <= st.pos[0, 0] < 2.0
    assert st.pos[1, 0] == 1.0
    assert 0.0 <= st.pos[2, 0] < 2.0
