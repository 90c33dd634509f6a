"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws initial particle states and workload parameters; it holds
none of the SRD step's arithmetic (no streaming, binning, cell sums, axes or
rotations).  Both the HIP path and the oracle start from the FP32 arrays it
returns, so neither sees the other's numbers.

Workload shapes follow the paper's benchmark systems (Sec. 4): a pure SRD
fluid in a cubic periodic box of L^3 unit cells (a = 1) with 10 particles per
cell on average, positions uniform, velocities Maxwellian at kT = 1, m = 1,
zero net momentum.
"""
import math

import numpy as np


def _rng(seed, stream):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


def thermal_state(L, n_particles, seed, a=1.0, kT=1.0, mass=1.0):
    """Uniform positions in [0, L_d a), Gaussian velocities with zero mean,
    rescaled so that sum m|v|^2 / (3(N-1)) == kT before the FP32 rounding.

    Returns (pos, vel) as float32 arrays of shape (3, N).
    """
    if isinstance(L, int):
        L = (L, L, L)
    n = int(n_particles)
    g = _rng(seed, 2)
    pos = np.empty((3, n), dtype=np.float64)
    for d in range(3):
        pos[d] = g.random(n) * (L[d] * a)
    g = _rng(seed, 3)
    vel = g.standard_normal((3, n)) * math.sqrt(kT / mass)
    if n > 1:
        vel -= vel.mean(axis=1, keepdims=True)
        t = mass * float(np.sum(vel * vel)) / (3.0 * (n - 1))
        vel *= math.sqrt(kT / t)
    pos32 = pos.astype(np.float32)
    for d in range(3):
        # float32 rounding may land exactly on the upper edge; keep [0, L a)
        edge = np.float32(L[d] * a)
        pos32[d][pos32[d] >= edge] = np.float32(0.0)
    return pos32, vel.astype(np.float32)


def monoenergetic_state(L, n_particles, seed, a=1.0, speed=math.sqrt(3.0)):
    """Uniform positions; every velocity has the same magnitude, isotropic
    directions, then the mean is removed (|v| stays close to `speed`)."""
    if isinstance(L, int):
        L = (L, L, L)
    n = int(n_particles)
    pos, _ = thermal_state(L, n, seed, a)
    g = _rng(seed, 4)
    u = g.standard_normal((3, n))
    u /= np.linalg.norm(u, axis=0, keepdims=True)
    vel = u * speed
    vel -= vel.mean(axis=1, keepdims=True)
    return pos, vel.astype(np.float32)


def shear_wave_state(L, n_particles, seed, amplitude=0.1, a=1.0, kT=1.0):
    """Thermal state plus a transverse wave v_x += A sin(2 pi z / (L_z a))."""
    if isinstance(L, int):
        L = (L, L, L)
    pos, vel = thermal_state(L, n_particles, seed, a, kT)
    kz = 2.0 * math.pi / (L[2] * a)
    v = vel.astype(np.float64)
    v[0] += amplitude * np.sin(kz * pos[2].astype(np.float64))
    return pos, v.astype(np.float32)


def ensemble_boxes(n_boxes=512, seed=4, edge=(8, 48), density=(5.0, 20.0),
                   alphas_deg=(90.0, 120.0, 130.0), dt=0.1):
    """Batched-ensemble workload: independent cubic periodic boxes with edges
    uniform in [edge0, edge1], densities uniform in [density0, density1],
    angles drawn from alphas_deg, box b seeded (seed << 32) | b."""
    g = _rng(seed, 0)
    boxes = []
    for b in range(n_boxes):
        L = int(g.integers(edge[0], edge[1] + 1))
        rho = float(g.uniform(density[0], density[1]))
        alpha = float(alphas_deg[int(g.integers(0, len(alphas_deg)))])
        boxes.append(dict(L=L, n=int(round(rho * L ** 3)), alpha_deg=alpha, dt=dt,
                          seed=(int(seed) << 32) | b))
    return boxes


def served_requests(rate_hz=200.0, window_s=60.0, seed=5, edge=(8, 64), density=(5.0, 20.0),
                    dt=(0.05, 0.2), alpha_deg=(90.0, 150.0), steps=(200, 2000), max_requests=None):
    """Poisson arrivals at rate_hz over window_s seconds; each request is one
    periodic box with its own parameters and seed."""
    g = _rng(seed, 0)
    t = 0.0
    reqs = []
    while True:
        t += float(g.exponential(1.0 / rate_hz))
        if t >= window_s or (max_requests is not None and len(reqs) >= max_requests):
            break
        L = int(g.integers(edge[0], edge[1] + 1))
        rho = float(g.uniform(density[0], density[1]))
        reqs.append(dict(arrival=t, L=L, n=int(round(rho * L ** 3)),
                         dt=float(g.uniform(dt[0], dt[1])),
                         alpha_deg=float(g.uniform(alpha_deg[0], alpha_deg[1])),
                         steps=int(g.integers(steps[0], steps[1] + 1)),
                         seed=int(g.integers(1, 2 ** 63 - 1))))
    return reqs
