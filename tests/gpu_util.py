"""Helpers for the GPU parity tests: run the FP64 oracle on the same FP32
input the HIP path gets and compare element by element.

Tolerances (what the FP32 path can and must reach against FP64):
  * positions: torus distance <= 1 ulp_FP32 of the box edge (one FP32
    rounding of x + v dt, one of the periodic fold);
  * collision cells: bit-exact, except particles whose FP64 (x - s)/a lies
    within a face band of 4 ulp_FP32(edge) of a cell face, where the FP32
    position may round onto the other side;
  * velocities: |v_gpu - v_oracle|_inf <= 1e-5 max(|v_oracle|_inf, sqrt(kT/m))
    per particle, outside the (at most two) cells each face-band particle
    may belong to.
"""
import math

import numpy as np

from oracle import oracle as orc


def ulp_top(length):
    """Spacing of float32 numbers just below `length`."""
    return float(np.spacing(np.float32(np.nextafter(np.float32(length), np.float32(0)))))


def f32_state(pos, vel, L, a=1.0):
    """Round an FP64 state to FP32 keeping positions inside [0, L a)."""
    pos32 = np.asarray(pos, dtype=np.float32).copy()
    for d in range(3):
        edge = np.float32(L[d] * a)
        pos32[d][pos32[d] >= edge] = np.float32(0.0)
        pos32[d][pos32[d] < 0] = np.float32(0.0)
    return pos32, np.asarray(vel, dtype=np.float32).copy()


def oracle_one_step(pos32, vel32, box, k, mass32=None):
    """One oracle step (stream + collide at step k) from the FP32 state."""
    st = orc.State(pos32.astype(np.float64), vel32.astype(np.float64),
                   None if mass32 is None else mass32.astype(np.float64))
    orc.stream(box, st)
    s = orc.shift(box.seed, k, box.a)
    cells = orc.cells(box, s, st)
    orc.collide(box, k, st)
    return st, s, cells


def face_band_mask(pos64, s, box):
    """Particles whose (x - s)/a is within the face band of a cell face."""
    L = [int(box.L[d]) for d in range(3)]
    delta = 4.0 * max(ulp_top(L[d] * box.a) for d in range(3)) / box.a
    near = np.zeros(pos64.shape[1], dtype=bool)
    for d in range(3):
        q = (pos64[d] - s[d]) / box.a
        near |= np.abs(q - np.round(q)) < delta
    return near


def neighbour_cells(cells, pos64, s, box):
    """For face-band particles: the cells on both sides of each nearby face
    (in every dimension where the particle is within the band)."""
    L = [int(box.L[d]) for d in range(3)]
    delta = 4.0 * max(ulp_top(L[d] * box.a) for d in range(3)) / box.a
    out = set()
    for i in range(len(cells)):
        idx = []
        for d in range(3):
            q = (pos64[d, i] - s[d]) / box.a
            r = int(round(q))
            if abs(q - r) < delta:
                idx.append(sorted({(r - 1) % L[d], r % L[d]}))
            else:
                idx.append([int(math.floor(q)) % L[d]])
        for ix in idx[0]:
            for iy in idx[1]:
                for iz in idx[2]:
                    out.add(ix + L[0] * (iy + L[1] * iz))
    return out


def check_against(ref, s, cells, box, gpu_pos, gpu_vel, kT=1.0, mass=1.0, band_from=None):
    """Compare a GPU result with the oracle's FP64 result `ref` (an
    oracle.State after stream + collide); `cells` are the oracle's collision
    cells of the streamed positions under shift s.  When `ref` is a sample of
    whole cells, `band_from` = (positions, cells) of ALL streamed particles,
    so a face-band particle outside the sample that the FP32 path puts into a
    sampled cell also exempts that cell."""
    L = np.array([int(box.L[d]) for d in range(3)], dtype=np.float64) * box.a
    dpos = gpu_pos.astype(np.float64) - ref.pos
    dpos -= np.round(dpos / L[:, None]) * L[:, None]
    ptol = max(ulp_top(x) for x in L)
    assert np.max(np.abs(dpos)) <= ptol, ("position", np.max(np.abs(dpos)), ptol)
    band = face_band_mask(ref.pos, s, box)
    if band_from is not None:
        all_pos, all_cells = band_from
        ball = face_band_mask(all_pos, s, box)
        exempt_cells = neighbour_cells(all_cells[ball], all_pos[:, ball], s, box) if ball.any() else set()
    else:
        exempt_cells = neighbour_cells(cells[band], ref.pos[:, band], s, box) if band.any() else set()
    keep = ~np.isin(cells, np.fromiter(exempt_cells, dtype=np.int64, count=len(exempt_cells)))
    scale = np.maximum(np.max(np.abs(ref.vel), axis=0), math.sqrt(kT / mass))
    err = np.max(np.abs(gpu_vel.astype(np.float64) - ref.vel), axis=0) / scale
    bad = keep & (err > 1e-5)
    if bad.any():
        i = int(np.flatnonzero(bad)[np.argmax(err[bad])])
        raise AssertionError(("velocity", int(bad.sum()), float(err[keep].max()), "worst particle", i,
                              "cell", int(cells[i]), "pos", ref.pos[:, i].tolist(),
                              "gpu v", gpu_vel[:, i].tolist(), "oracle v", ref.vel[:, i].tolist(),
                              "bad cells", sorted(set(int(c) for c in cells[bad]))[:20]))
    if band_from is None:   # each face-band particle exempts at most 8 cells (2 per near face)
        assert len(exempt_cells) <= 8 * int(band.sum()), "too many exemptions"
    return int(band.sum()), float(err[keep].max()) if keep.any() else 0.0


def compare_step(pos32, vel32, gpu_pos, gpu_vel, box, k, kT=1.0, mass=1.0, mass32=None):
    """Assert the GPU's one-step result matches the oracle's; returns the
    number of face-band particles and the largest kept velocity error."""
    st, s, cells = oracle_one_step(pos32, vel32, box, k, mass32)
    return check_against(st, s, cells, box, gpu_pos, gpu_vel, kT, mass)


def match_unordered(ref_pos, gpu_pos, gpu_vel, L, a=1.0):
    """Boxes without particle ids return their particles in storage order.
    Match every reference particle (oracle FP64 positions after the step's
    streaming, which the collision leaves unchanged) with the GPU particle at
    the same place on the torus (within the FP32 position tolerance, each GPU
    particle used once) and return the GPU positions and velocities in the
    reference order."""
    from scipy.spatial import cKDTree
    edge = np.array([L[d] * a for d in range(3)], dtype=np.float64)
    tol = 2.0 * max(ulp_top(x) for x in edge)
    g = np.mod(gpu_pos.astype(np.float64).T, edge)
    r = np.mod(np.asarray(ref_pos, dtype=np.float64).T, edge)
    tree = cKDTree(g, boxsize=edge)
    dist, idx = tree.query(r, k=1)
    assert np.all(dist <= tol), ("unmatched particle", float(dist.max()), tol)
    assert len(np.unique(idx)) == len(idx), "two reference particles matched one GPU particle"
    return gpu_pos[:, idx], gpu_vel[:, idx]


def same_particle_set(pa, va, pb, vb):
    """The two states hold the same particles bit for bit (any order)."""
    A = np.concatenate([pa, va]).view(np.uint32)
    B = np.concatenate([pb, vb]).view(np.uint32)
    if A.shape != B.shape:
        return False
    oa = np.lexsort(A[::-1])
    ob = np.lexsort(B[::-1])
    return bool(np.array_equal(A[:, oa], B[:, ob]))
