"""mpcd_moments: the exact momentum and kinetic-energy sums of mpcd_observe,
applied to caller device arrays, against the FP64 oracle's diagnostics
(within the fixed-point quantum of each term plus the oracle's own FP64
rounding) and bit for bit against mpcd_observe on a box."""
import ctypes

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


def _device(arr):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float32)).cuda()


def moments(mp, vel, mass=None):
    import torch
    v = [_device(vel[d]) for d in range(3)]
    m = _device(mass) if mass is not None else None
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    rc = mp.mpcd_moments(v[0].data_ptr(), v[1].data_ptr(), v[2].data_ptr(), m.data_ptr() if m is not None else 0,
                         vel.shape[1], out.data_ptr())
    assert rc == mp.MPCD_OK
    return out.cpu().numpy()


@pytest.mark.parametrize("n,masses", [(1, False), (4095, False), (4096, True), (1_000_003, True),
                                      (5_000_000, False)])
def test_moments_match_the_oracle(mp, n, masses):
    rng = np.random.default_rng(n)
    vel = rng.normal(size=(3, n)).astype(np.float32)
    mass = rng.uniform(0.25, 4.0, n).astype(np.float32) if masses else None
    out = moments(mp, vel, mass)
    st = orc.State(np.zeros((3, n)), vel.astype(np.float64), None if mass is None else mass.astype(np.float64))
    P, E, T, M = orc.diagnostics(st)
    # each fixed-point term is rounded to the quantum 2^-32 (error <= 2^-33
    # per particle), the oracle sums in FP64 (relative error well below 1e-14
    # of the sum of magnitudes at these sizes)
    m64 = np.ones(n) if mass is None else mass.astype(np.float64)
    v64 = vel.astype(np.float64)
    tol_p = n * 2.0 ** -33 + 1e-14 * np.sum(m64 * np.abs(v64), axis=1)
    tol_e = n * 2.0 ** -33 + 1e-14 * np.sum(m64 * v64 * v64)
    assert np.all(np.abs(out[:3] - P) <= tol_p), (out[:3], P)
    assert abs(out[3] - 2.0 * E) <= tol_e, (out[3], 2.0 * E)
    assert out[4] == 0


def test_moments_flag_out_of_range(mp):
    vel = np.zeros((3, 10), dtype=np.float32)
    vel[1, 3] = 300.0
    mass = np.ones(10, dtype=np.float32)
    mass[7] = 1000.0
    out = moments(mp, vel, mass)
    assert out[4] == 2


def test_moments_equal_observe(mp):
    """The same bits as mpcd_observe on a box in state (pos, vel)."""
    L, n = (12, 10, 8), 9600
    pos, vel = inputs.thermal_state(L, n, seed=77)
    with mp.Context() as ctx:
        slot = ctx.admit(mp.make_desc(L, n, init="external"))
        ctx.set_state(slot, (pos, vel))
        obs = ctx.observe(slot)
    out = moments(mp, vel)
    assert np.array_equal(out[:3], obs["P"]) and out[3] == 2.0 * obs["E"]
    assert mp.mpcd_moments(None, None, None, None, 5, 0) == mp.MPCD_EINVAL
