"""ctypes binding of libmpcd.so (C ABI in include/mpcd.h).

The functions below carry the C names and only marshal arguments; every step
of the SRD update runs in the library's HIP kernels.  PyTorch supplies device
memory (through the allocator callback) and the HIP stream.  Importing this
module fails loudly if the library has not been built.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpcd.so")

MPCD_OK = 0
MPCD_EINVAL = -1
MPCD_ENOMEM = -2
MPCD_EDEVICE = -3
MPCD_EBUSY = -4
MPCD_ESTATE = -5
MPCD_ENOTFOUND = -6

MPCD_INIT_MAXWELL = 0x1
MPCD_INIT_EXTERNAL = 0x2
MPCD_TRACK_VACF = 0x4
MPCD_PARTICLE_MASS = 0x8
MPCD_CONSERVE_L = 0x10
MPCD_UNORDERED = 0x20

MPCD_BIN_AUTO = 0
MPCD_BIN_ATOMIC = 1
MPCD_BIN_SORT = 2


class mpcd_box_desc(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32 * 3),
        ("a", ctypes.c_double),
        ("n_particles", ctypes.c_int64),
        ("dt", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("kT", ctypes.c_double),
        ("mass", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("n_steps", ctypes.c_int64),
        ("flags", ctypes.c_uint32),
        ("vacf_stride", ctypes.c_int32),
        ("vacf_capacity", ctypes.c_int32),
    ]


mpcd_alloc_fn = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
mpcd_free_fn = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class mpcd_options(ctypes.Structure):
    _fields_ = [
        ("binning", ctypes.c_int32),
        ("brick", ctypes.c_int32 * 3),
        ("block", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("hbm_budget", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("alloc", mpcd_alloc_fn),
        ("free", mpcd_free_fn),
        ("user", ctypes.c_void_p),
        ("device", ctypes.c_int32),
        ("max_slots", ctypes.c_int32),
    ]


class mpcd_observables(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("P", ctypes.c_double * 3),
        ("E_kin", ctypes.c_double),
        ("T", ctypes.c_double),
        ("mass_total", ctypes.c_double),
        ("status", ctypes.c_int32),
        ("vacf_len", ctypes.c_int32),
        ("vacf", ctypes.POINTER(ctypes.c_double)),
        ("n_particles", ctypes.c_int64),
        ("binning", ctypes.c_int32),
        ("brick", ctypes.c_int32 * 3),
        ("overflow_steps", ctypes.c_int64),
        ("rebuckets", ctypes.c_int64),
    ]


class mpcd_kernel_stat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char_p),
        ("launches", ctypes.c_int64),
        ("total_ms", ctypes.c_double),
    ]


# every function the header declares, with its C signature
_SIGNATURES = {
    "mpcd_create": (ctypes.c_int, [ctypes.POINTER(mpcd_options), ctypes.POINTER(ctypes.c_void_p)]),
    "mpcd_admit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(mpcd_box_desc),
                                  ctypes.POINTER(ctypes.c_int32)]),
    "mpcd_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "mpcd_observe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(mpcd_observables)]),
    "mpcd_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_float),
                                      ctypes.POINTER(ctypes.c_int64)]),
    "mpcd_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_float),
                                      ctypes.c_int64]),
    "mpcd_set_mass": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]),
    "mpcd_get_mass": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]),
    "mpcd_get_vacf": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_float),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                     ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "mpcd_set_vacf": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_float),
                                     ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_int32]),
    "mpcd_hbm_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                     ctypes.c_void_p]),
    "mpcd_moments": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "mpcd_moments_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "mpcd_host_step": (ctypes.c_int, [ctypes.POINTER(mpcd_box_desc), ctypes.POINTER(ctypes.c_float),
                                      ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]),
    "mpcd_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "mpcd_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "mpcd_kernel_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(mpcd_kernel_stat), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32)]),
    "mpcd_destroy": (None, [ctypes.c_void_p]),
    "mpcd_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "mpcd_abi_version": (ctypes.c_int, []),
}

if not os.path.exists(LIB_PATH):
    raise ImportError("libmpcd.so is not built (%s); run `python -m paper_2212_11878_amd.csrc.build`"
                      % LIB_PATH)
# PyTorch ships its own HIP runtime.  Loading it first makes the library's
# libamdhip64 dependency resolve to that same copy (same soname); loading the
# library first would map a second runtime, whose streams and device pointers
# are not the ones PyTorch hands over.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)
for _name, (_res, _args) in _SIGNATURES.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

# layout of the structs above (include/mpcd.h, MPCD_ABI_VERSION)
ABI_VERSION = 4
if _lib.mpcd_abi_version() != ABI_VERSION:
    raise ImportError("libmpcd.so has ABI version %d, this binding expects %d; rebuild it"
                      % (_lib.mpcd_abi_version(), ABI_VERSION))


class MPCDError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__("%s: %s (%d)" % (what, mpcd_strerror(status), status))


def _check(rc, what):
    if rc != MPCD_OK:
        raise MPCDError(rc, what)
    return rc


# ---------------------------------------------------------------------------
# the C functions, same names, argument marshalling only

def mpcd_abi_version():
    return _lib.mpcd_abi_version()


def mpcd_strerror(status):
    return _lib.mpcd_strerror(int(status)).decode()


def mpcd_create(options):
    h = ctypes.c_void_p()
    rc = _lib.mpcd_create(ctypes.byref(options) if options is not None else None, ctypes.byref(h))
    return rc, h


def mpcd_admit(ctx, desc):
    slot = ctypes.c_int32(-1)
    rc = _lib.mpcd_admit(ctx, ctypes.byref(desc), ctypes.byref(slot))
    return rc, slot.value


def mpcd_step(ctx, n_steps):
    return _lib.mpcd_step(ctx, int(n_steps))


def mpcd_observe(ctx, slot):
    obs = mpcd_observables()
    rc = _lib.mpcd_observe(ctx, int(slot), ctypes.byref(obs))
    return rc, obs


def mpcd_get_state(ctx, slot, n):
    buf = np.empty(6 * int(n), dtype=np.float32)
    step = ctypes.c_int64(0)
    rc = _lib.mpcd_get_state(ctx, int(slot), buf.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                             ctypes.byref(step))
    return rc, buf.reshape(6, -1), step.value


def mpcd_set_state(ctx, slot, xyzv, step):
    buf = np.ascontiguousarray(xyzv, dtype=np.float32).reshape(-1)
    return _lib.mpcd_set_state(ctx, int(slot), buf.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                               int(step))


def mpcd_set_mass(ctx, slot, mass):
    buf = np.ascontiguousarray(mass, dtype=np.float32).reshape(-1)
    return _lib.mpcd_set_mass(ctx, int(slot), buf.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))


def mpcd_get_mass(ctx, slot, n):
    buf = np.empty(int(n), dtype=np.float32)
    rc = _lib.mpcd_get_mass(ctx, int(slot), buf.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    return rc, buf


def mpcd_get_vacf(ctx, slot, n, max_samples):
    v0 = np.empty(3 * int(n), dtype=np.float32)
    samples = np.empty(max(1, int(max_samples)), dtype=np.float64)
    origin = ctypes.c_int64(0)
    length = ctypes.c_int32(0)
    rc = _lib.mpcd_get_vacf(ctx, int(slot), v0.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                            ctypes.byref(origin), samples.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            int(max_samples), ctypes.byref(length))
    return rc, v0.reshape(3, -1), origin.value, samples[:min(length.value, int(max_samples))].copy()


def mpcd_set_vacf(ctx, slot, v0, origin, samples):
    v = np.ascontiguousarray(v0, dtype=np.float32).reshape(-1)
    smp = np.ascontiguousarray(samples, dtype=np.float64).reshape(-1)
    return _lib.mpcd_set_vacf(ctx, int(slot), v.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(origin),
                              smp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(smp))


def mpcd_hbm_copy(src_ptr, dst_ptr, nbytes, blocks=0, stream=None):
    return _lib.mpcd_hbm_copy(ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr), int(nbytes), int(blocks),
                              ctypes.c_void_p(stream) if stream else None)


def mpcd_moments(vx_ptr, vy_ptr, vz_ptr, mass_ptr, n, out_ptr, stream=None):
    return _lib.mpcd_moments(ctypes.c_void_p(vx_ptr), ctypes.c_void_p(vy_ptr), ctypes.c_void_p(vz_ptr),
                             ctypes.c_void_p(mass_ptr) if mass_ptr else None, int(n), ctypes.c_void_p(out_ptr),
                             ctypes.c_void_p(stream) if stream else None)


def mpcd_moments_noalloc(vx_ptr, vy_ptr, vz_ptr, mass_ptr, n, out_ptr, stream=None):
    return _lib.mpcd_moments_noalloc(ctypes.c_void_p(vx_ptr), ctypes.c_void_p(vy_ptr), ctypes.c_void_p(vz_ptr),
                                     ctypes.c_void_p(mass_ptr) if mass_ptr else None, int(n),
                                     ctypes.c_void_p(out_ptr), ctypes.c_void_p(stream) if stream else None)


def mpcd_host_step(desc, xyzv, mass, pid, step, n_steps, threads=0):
    """xyzv: float32 array of shape (6, n), C-contiguous, updated in place;
    mass (float32, n) and pid (int32, n) likewise, or None.  The call runs
    without the interpreter lock."""
    def ptr(a, dtype, shape, ctype):
        if a is None:
            return None
        if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags.c_contiguous and a.shape == shape):
            raise ValueError("expected a C-contiguous %s array of shape %s" % (np.dtype(dtype).name, shape))
        return a.ctypes.data_as(ctypes.POINTER(ctype))
    n = int(desc.n_particles)
    return _lib.mpcd_host_step(ctypes.byref(desc), ptr(xyzv, np.float32, (6, n), ctypes.c_float),
                               ptr(mass, np.float32, (n,), ctypes.c_float), ptr(pid, np.int32, (n,), ctypes.c_int32),
                               int(step), int(n_steps), int(threads))


def mpcd_release(ctx, slot):
    return _lib.mpcd_release(ctx, int(slot))


def mpcd_profile(ctx, enable):
    return _lib.mpcd_profile(ctx, 1 if enable else 0)


def mpcd_kernel_stats(ctx, max_entries=32):
    arr = (mpcd_kernel_stat * max_entries)()
    count = ctypes.c_int32(0)
    rc = _lib.mpcd_kernel_stats(ctx, arr, max_entries, ctypes.byref(count))
    out = {}
    for i in range(min(count.value, max_entries)):
        out[arr[i].name.decode()] = (int(arr[i].launches), float(arr[i].total_ms))
    return rc, out


def mpcd_destroy(ctx):
    _lib.mpcd_destroy(ctx)


# ---------------------------------------------------------------------------
# convenience wrapper: torch memory and stream, exceptions on errors

class _TorchAllocator:
    """Device memory for the library from PyTorch's caching allocator, in
    the pool of the library's stream: a freed block is reused only by
    allocations made for that stream, i.e. by work queued after the free."""

    def __init__(self, device, stream):
        import torch
        self._torch = torch
        self.device = device
        self.stream = stream
        self.blocks = {}
        self.c_alloc = mpcd_alloc_fn(self._alloc)
        self.c_free = mpcd_free_fn(self._free)

    def _alloc(self, nbytes, user):
        try:
            with self._torch.cuda.stream(self.stream):
                t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device=self.device)
        except Exception:
            return None
        p = t.data_ptr()
        self.blocks[p] = t
        return p

    def _free(self, ptr, user):
        self.blocks.pop(ptr, None)

    def bytes_held(self):
        return sum(t.numel() for t in self.blocks.values())


def make_desc(L, n_particles, dt=0.1, alpha_deg=130.0, seed=1, a=1.0, kT=1.0, mass=1.0,
              n_steps=0, init="maxwell", vacf_stride=0, vacf_capacity=0, alpha_rad=None,
              particle_mass=False, conserve_l=False, unordered=False):
    d = mpcd_box_desc()
    if isinstance(L, int):
        L = (L, L, L)
    for i in range(3):
        d.L[i] = int(L[i])
    d.a = float(a)
    d.n_particles = int(n_particles)
    d.dt = float(dt)
    d.alpha = float(alpha_rad) if alpha_rad is not None else math.radians(alpha_deg)
    d.kT = float(kT)
    d.mass = float(mass)
    d.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    d.n_steps = int(n_steps)
    d.flags = MPCD_INIT_MAXWELL if init == "maxwell" else MPCD_INIT_EXTERNAL
    if particle_mass:
        d.flags |= MPCD_PARTICLE_MASS
    if conserve_l:
        d.flags |= MPCD_CONSERVE_L
    if unordered:
        d.flags |= MPCD_UNORDERED
    if vacf_stride:
        d.flags |= MPCD_TRACK_VACF
        d.vacf_stride = int(vacf_stride)
        d.vacf_capacity = int(vacf_capacity)
    return d


class Context:
    """One library context on a torch-owned HIP stream."""

    def __init__(self, device=0, binning=MPCD_BIN_AUTO, brick=(0, 0, 0), use_graph=True,
                 hbm_budget=0, max_slots=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible to PyTorch; libmpcd needs a HIP device")
        self.device = torch.device("cuda", device)
        self.stream = torch.cuda.Stream(device=self.device)
        self.allocator = _TorchAllocator(self.device, self.stream)
        opt = mpcd_options()
        opt.binning = binning
        if isinstance(brick, int):
            brick = (brick, brick, brick)
        for i in range(3):
            opt.brick[i] = int(brick[i])
        opt.block = 0
        opt.use_graph = 1 if use_graph else 0
        opt.hbm_budget = int(hbm_budget)
        opt.stream = ctypes.c_void_p(self.stream.cuda_stream)
        opt.alloc = self.allocator.c_alloc
        opt.free = self.allocator.c_free
        opt.user = None
        opt.device = device
        opt.max_slots = max_slots
        self._opt = opt
        rc, h = mpcd_create(opt)
        _check(rc, "mpcd_create")
        self.handle = h
        self.n = {}

    def admit(self, desc, state=None, step=0):
        rc, slot = mpcd_admit(self.handle, desc)
        _check(rc, "mpcd_admit")
        self.n[slot] = int(desc.n_particles)
        if state is not None:
            self.set_state(slot, state, step)
        return slot

    def try_admit(self, desc):
        rc, slot = mpcd_admit(self.handle, desc)
        if rc == MPCD_OK:
            self.n[slot] = int(desc.n_particles)
            return slot
        if rc in (MPCD_ENOMEM, MPCD_EBUSY):
            return None
        raise MPCDError(rc, "mpcd_admit")

    def set_state(self, slot, state, step=0):
        pos, vel = state
        xyzv = np.concatenate([np.asarray(pos, np.float32).reshape(3, -1),
                               np.asarray(vel, np.float32).reshape(3, -1)])
        _check(mpcd_set_state(self.handle, slot, xyzv, step), "mpcd_set_state")

    def set_mass(self, slot, mass):
        _check(mpcd_set_mass(self.handle, slot, mass), "mpcd_set_mass")

    def get_mass(self, slot):
        rc, m = mpcd_get_mass(self.handle, slot, self.n[slot])
        _check(rc, "mpcd_get_mass")
        return m

    def get_vacf(self, slot, max_samples=1 << 16):
        """(v0 [3, N], origin step, samples so far)"""
        rc, v0, origin, samples = mpcd_get_vacf(self.handle, slot, self.n[slot], max_samples)
        _check(rc, "mpcd_get_vacf")
        return v0, origin, samples

    def set_vacf(self, slot, v0, origin, samples):
        _check(mpcd_set_vacf(self.handle, slot, v0, origin, samples), "mpcd_set_vacf")

    def get_state(self, slot):
        rc, buf, step = mpcd_get_state(self.handle, slot, self.n[slot])
        _check(rc, "mpcd_get_state")
        return buf[:3].copy(), buf[3:].copy(), step

    def step(self, n=1):
        _check(mpcd_step(self.handle, n), "mpcd_step")

    def observe(self, slot):
        rc, obs = mpcd_observe(self.handle, slot)
        if rc not in (MPCD_OK, MPCD_ESTATE):
            raise MPCDError(rc, "mpcd_observe")
        vacf = [obs.vacf[i] for i in range(obs.vacf_len)] if obs.vacf_len > 0 else []
        return dict(step=obs.step, P=np.array(obs.P[:]), E=obs.E_kin, T=obs.T, M=obs.mass_total,
                    status=obs.status, vacf=np.array(vacf), binning=obs.binning,
                    brick=tuple(obs.brick[:]), n=obs.n_particles, overflow_steps=obs.overflow_steps,
                    rebuckets=obs.rebuckets)

    def release(self, slot):
        _check(mpcd_release(self.handle, slot), "mpcd_release")
        self.n.pop(slot, None)

    def profile(self, enable):
        _check(mpcd_profile(self.handle, enable), "mpcd_profile")

    def kernel_stats(self):
        rc, out = mpcd_kernel_stats(self.handle)
        _check(rc, "mpcd_kernel_stats")
        return out

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if getattr(self, "handle", None):
            mpcd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
