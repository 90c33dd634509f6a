"""ctypes wrapper around the FP64 C oracle (mpcd_oracle.c).

Test infrastructure only: tests, the smoke check and the benchmark's CPU
baseline call it; the product path never does.  Every function takes and
returns float64 numpy arrays; the C side does all the arithmetic.
"""
import ctypes
import math

import numpy as np

from . import build as _build

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


class Box(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32 * 3),
        ("a", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


def make_box(L, a=1.0, dt=0.1, alpha_deg=130.0, seed=1, alpha_rad=None):
    if isinstance(L, int):
        L = (L, L, L)
    b = Box()
    for d in range(3):
        b.L[d] = int(L[d])
    b.a = float(a)
    b.dt = float(dt)
    b.alpha = float(alpha_rad) if alpha_rad is not None else math.radians(alpha_deg)
    b.seed = int(seed)
    return b


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = ctypes.CDLL(path)
        L.oracle_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.oracle_philox4x32_10.restype = None
        L.oracle_u24.argtypes = [ctypes.c_uint32]
        L.oracle_u24.restype = ctypes.c_double
        L.oracle_shift.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, _dp]
        L.oracle_shift.restype = None
        L.oracle_axis.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, _dp]
        L.oracle_axis.restype = None
        L.oracle_rotate.argtypes = [_dp, ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.oracle_rotate.restype = None
        bp = ctypes.POINTER(Box)
        L.oracle_stream.argtypes = [bp, ctypes.c_int64] + [_dp] * 6
        L.oracle_stream.restype = None
        L.oracle_cell_of.argtypes = [bp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.oracle_cell_of.restype = ctypes.c_int64
        L.oracle_cells.argtypes = [bp, _dp, ctypes.c_int64] + [_dp] * 3 + [_i64p]
        L.oracle_cells.restype = None
        L.oracle_cell_sums.argtypes = [bp, _dp, ctypes.c_int64] + [_dp] * 7 + [_i64p, _dp, _dp]
        L.oracle_cell_sums.restype = None
        L.oracle_collide.argtypes = [bp, ctypes.c_uint64, ctypes.c_int64] + [_dp] * 7 + [_i64p]
        L.oracle_collide.restype = ctypes.c_int
        L.oracle_collide_given.argtypes = [bp, _dp, _dp, ctypes.c_int64] + [_dp] * 7
        L.oracle_collide_given.restype = ctypes.c_int
        L.oracle_collide_am.argtypes = [bp, ctypes.c_uint64, ctypes.c_int64] + [_dp] * 7
        L.oracle_collide_am.restype = ctypes.c_int
        L.oracle_collide_am_given.argtypes = [bp, _dp, _dp, ctypes.c_int64] + [_dp] * 7
        L.oracle_collide_am_given.restype = ctypes.c_int
        L.oracle_cell_local.argtypes = [bp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        L.oracle_cell_local.restype = None
        L.oracle_sym3_pinv.argtypes = [_dp, ctypes.c_double, _dp]
        L.oracle_sym3_pinv.restype = None
        L.oracle_step.argtypes = [bp, ctypes.c_uint64, ctypes.c_int64] + [_dp] * 7 + [_i64p]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_run.argtypes = [bp, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64] + [_dp] * 7
        L.oracle_run.restype = ctypes.c_int
        L.oracle_diagnostics.argtypes = [ctypes.c_int64] + [_dp] * 4 + [_dp]
        L.oracle_diagnostics.restype = None
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "need contiguous float64"
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class State:
    """FP64 particle state: positions (3, N), velocities (3, N), masses or None."""

    def __init__(self, pos, vel, mass=None):
        self.pos = np.array(pos, dtype=np.float64, order="C", copy=True).reshape(3, -1)
        self.vel = np.array(vel, dtype=np.float64, order="C", copy=True).reshape(3, -1)
        self.mass = None if mass is None else _f64(np.array(mass, dtype=np.float64, copy=True))

    @property
    def n(self):
        return self.pos.shape[1]

    def copy(self):
        return State(self.pos, self.vel, self.mass)

    def _args(self):
        p, v = self.pos, self.vel
        return [p[0].ctypes.data_as(_dp), p[1].ctypes.data_as(_dp), p[2].ctypes.data_as(_dp),
                v[0].ctypes.data_as(_dp), v[1].ctypes.data_as(_dp), v[2].ctypes.data_as(_dp),
                _ptr(self.mass)]


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xffffffff for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return [int(o[i]) for i in range(4)]


def u24(r):
    return lib().oracle_u24(int(r) & 0xffffffff)


def shift(seed, k, a=1.0):
    s = np.zeros(3)
    lib().oracle_shift(int(seed), int(k), float(a), _ptr(s))
    return s


def axis(seed, k, c):
    n = np.zeros(3)
    lib().oracle_axis(int(seed), int(k), int(c), _ptr(n))
    return n


def rotate(n, alpha, w):
    n = _f64(n)
    w = _f64(w)
    out = np.zeros(3)
    lib().oracle_rotate(_ptr(n), math.cos(alpha), math.sin(alpha), _ptr(w), _ptr(out))
    return out


def stream(box, st: State):
    a = st._args()
    lib().oracle_stream(ctypes.byref(box), st.n, *a[:6])


def cell_of(box, s, x, y, z):
    s = _f64(s)
    return int(lib().oracle_cell_of(ctypes.byref(box), _ptr(s), float(x), float(y), float(z)))


def cells(box, s, st: State):
    out = np.zeros(st.n, dtype=np.int64)
    s = _f64(s)
    p = st.pos
    lib().oracle_cells(ctypes.byref(box), _ptr(s), st.n, p[0].ctypes.data_as(_dp),
                       p[1].ctypes.data_as(_dp), p[2].ctypes.data_as(_dp), out.ctypes.data_as(_i64p))
    return out


def n_cells(box):
    return int(box.L[0]) * int(box.L[1]) * int(box.L[2])


def cell_sums(box, s, st: State):
    C = n_cells(box)
    count = np.zeros(C, dtype=np.int64)
    P = np.zeros(3 * C)
    M = np.zeros(C)
    s = _f64(s)
    lib().oracle_cell_sums(ctypes.byref(box), _ptr(s), st.n, *st._args(),
                           count.ctypes.data_as(_i64p), _ptr(P), _ptr(M))
    return count, P.reshape(C, 3), M


def collide(box, k, st: State, want_cells=False):
    cells = np.zeros(st.n, dtype=np.int64) if want_cells else None
    rc = lib().oracle_collide(ctypes.byref(box), int(k), st.n, *st._args(),
                              cells.ctypes.data_as(_i64p) if want_cells else None)
    if rc:
        raise MemoryError("oracle_collide")
    return cells


def collide_given(box, s, axes, st: State):
    s = _f64(s)
    axes = _f64(np.asarray(axes, dtype=np.float64).reshape(-1))
    rc = lib().oracle_collide_given(ctypes.byref(box), _ptr(s), _ptr(axes), st.n, *st._args())
    if rc:
        raise MemoryError("oracle_collide_given")


def collide_am(box, k, st: State):
    rc = lib().oracle_collide_am(ctypes.byref(box), int(k), st.n, *st._args())
    if rc:
        raise MemoryError("oracle_collide_am")


def collide_am_given(box, s, axes, st: State):
    s = _f64(s)
    axes = _f64(np.asarray(axes, dtype=np.float64).reshape(-1))
    rc = lib().oracle_collide_am_given(ctypes.byref(box), _ptr(s), _ptr(axes), st.n, *st._args())
    if rc:
        raise MemoryError("oracle_collide_am_given")


def cell_local(box, s, x, y, z):
    s = _f64(s)
    r = np.zeros(3)
    lib().oracle_cell_local(ctypes.byref(box), _ptr(s), float(x), float(y), float(z), _ptr(r))
    return r


def sym3_pinv(A, tol=1e-10):
    A = _f64(np.asarray(A, dtype=np.float64).reshape(9))
    out = np.zeros(9)
    lib().oracle_sym3_pinv(_ptr(A), float(tol), _ptr(out))
    return out.reshape(3, 3)


def step(box, k, st: State, want_cells=False):
    cells = np.zeros(st.n, dtype=np.int64) if want_cells else None
    rc = lib().oracle_step(ctypes.byref(box), int(k), st.n, *st._args(),
                           cells.ctypes.data_as(_i64p) if want_cells else None)
    if rc:
        raise MemoryError("oracle_step")
    return cells


def run(box, k0, nsteps, st: State):
    rc = lib().oracle_run(ctypes.byref(box), int(k0), int(nsteps), st.n, *st._args())
    if rc:
        raise MemoryError("oracle_run")


def diagnostics(st: State):
    """(P[3], E_kin, T with 3(N-1) dof, total mass)."""
    out = np.zeros(6)
    v = st.vel
    lib().oracle_diagnostics(st.n, v[0].ctypes.data_as(_dp), v[1].ctypes.data_as(_dp),
                             v[2].ctypes.data_as(_dp), _ptr(st.mass), _ptr(out))
    return out[:3].copy(), float(out[3]), float(out[4]), float(out[5])


def vacf(vel, vel0):
    """(1/N) sum_i v_i . v0_i -- the velocity autocorrelation sample."""
    vel = np.asarray(vel, dtype=np.float64)
    vel0 = np.asarray(vel0, dtype=np.float64)
    return float(np.einsum("dn,dn->", vel, vel0) / vel.shape[1])
