"""Pins for the oracle's Philox4x32-10 and the uniform mappings built on it."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = [int(t, 16) for t in line.split()]
                rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_known_answer_vectors(orc):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert orc.philox4x32_10(ctr, key) == want


@pytest.fixture(scope="module")
def rocrand_helper(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("philox") / "philox_rocrand_check")
    src = os.path.join(HERE, "philox_rocrand_check.cpp")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", src, "-o", out],
                   check=True, capture_output=True)
    return out


def test_matches_rocrand_engine(orc, rocrand_helper):
    """rocRAND's engine is an independent implementation of the same
    published generator; both must agree on arbitrary counters and keys."""
    g = np.random.default_rng(123)
    rows = g.integers(0, 2 ** 32, size=(2000, 6), dtype=np.uint64)
    rows[:50, 1] = 0          # small counters as used for steps and cells
    rows[50:100, 2:4] = 0
    text = "\n".join(" ".join("%08x" % int(v) for v in r) for r in rows) + "\n"
    res = subprocess.run([rocrand_helper], input=text, capture_output=True, text=True, check=True)
    got = [[int(t, 16) for t in line.split()] for line in res.stdout.strip().splitlines()]
    assert len(got) == len(rows)
    for r, ref in zip(rows, got):
        assert orc.philox4x32_10(r[0:4], r[4:6]) == ref


def test_u24_exact_and_range(orc):
    assert orc.u24(0) == 0.0
    assert orc.u24(0xffffffff) == (2 ** 24 - 1) / 2 ** 24
    assert orc.u24(0x00000100) == 2.0 ** -24
    # low 8 bits are discarded
    assert orc.u24(0x123456ff) == orc.u24(0x12345600)
    # every value is a float32 number (exact in both precisions)
    for r in [1 << 8, 0x80000000, 0xdeadbeef, 0x7fffff00]:
        v = orc.u24(r)
        assert float(np.float32(v)) == v


def test_shift_range_and_uniformity(orc):
    s = np.array([orc.shift(7, k, 1.0) for k in range(20000)])
    assert s.min() >= -0.5 and s.max() < 0.5
    # uniform on [-1/2, 1/2): mean 0, variance 1/12 per component
    assert np.all(np.abs(s.mean(axis=0)) < 4 * np.sqrt(1 / 12 / len(s)))
    assert np.all(np.abs(s.var(axis=0) - 1 / 12) < 0.004)
    # scales with the cell edge
    assert np.allclose(orc.shift(7, 3, 2.5), 2.5 * orc.shift(7, 3, 1.0), rtol=0, atol=1e-15)
    # different seeds and steps give different shifts
    assert not np.allclose(orc.shift(7, 3), orc.shift(8, 3))
    assert not np.allclose(orc.shift(7, 3), orc.shift(7, 4))


def test_axis_uniform_on_sphere(orc):
    n = np.array([orc.axis(11, 5, c) for c in range(40000)])
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-14)
    m = len(n)
    # <n> = 0, <n n^T> = I/3, <n_d^4> = 1/5 for the uniform sphere
    assert np.all(np.abs(n.mean(axis=0)) < 4 * np.sqrt(1 / 3 / m))
    nn = n.T @ n / m
    assert np.allclose(nn, np.eye(3) / 3, atol=0.01)
    assert np.allclose((n ** 4).mean(axis=0), 0.2, atol=0.01)
    # axes of neighbouring cells are uncorrelated
    assert abs(np.mean(np.sum(n[1:] * n[:-1], axis=1))) < 4 * np.sqrt(1 / 3 / m)
    # keyed by (seed, step, cell): same inputs, same axis
    assert np.array_equal(orc.axis(11, 5, 17), n[17])
    assert not np.allclose(orc.axis(11, 6, 17), n[17])
