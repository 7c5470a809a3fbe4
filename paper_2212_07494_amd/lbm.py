"""ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every function keeps the C name.  All lattice work runs in the HIP library
``liblbm.so`` next to this file; if that library is missing, loading fails with an
error (there is no fallback).  Build it with ``python -m paper_2212_07494_amd.build``.

Arrays: NumPy float64, node index n = (z*ny + y)*nx + x (x fastest); vector fields
are (D, N) component planes; populations are (Q, N).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_WMACH = 1  # warning: the call did its work, but max |u| exceeded the Mach limit
LATTICES = {"D2Q9": 0, "D3Q19": 1, "D3Q27": 2, "D3Q39": 3}
COLLISIONS = {"bgk": 0, "smrt": 1, "rmrt": 2}
STORAGES = {"f64": 0, "f32": 1, "f32s": 2, "f16s": 3}
STORAGE_BYTES = {"f64": 8, "f32": 4, "f32s": 4, "f16s": 2}
QOF = {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27, "D3Q39": 39}
G_UNIFORM, G_PROFILE, G_FIELD = 0, 1, 2
PERIODIC, WALLS = 0, 1


class LBMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"lbm status {status}: {message}")
        self.status = status


class MachWarning(UserWarning):
    """A monitor record showed max |u| above the lattice's Mach limit (LBM_WMACH)."""


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class lbm_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class lbm_params(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("collision", C.c_int32), ("storage", C.c_int32),
                ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("bc", C.c_int32 * 3), ("tau", C.c_double * 5), ("rho0", C.c_double),
                ("g_kind", C.c_int32), ("g_axis", C.c_int32), ("g_uniform", C.c_double * 3),
                ("g_data", C.c_void_p), ("monitor_every", C.c_int32),
                ("allocator", C.POINTER(lbm_allocator)), ("force_order", C.c_int32),
                ("solid", C.c_void_p), ("tau_bulk", C.c_double), ("tau_31", C.c_double),
                ("max_order", C.c_int32), ("mach_limit", C.c_double),
                ("debug_poison", C.c_int32)]


class lbm_tuning(C.Structure):
    _fields_ = [("bx", C.c_int32), ("by", C.c_int32), ("variant", C.c_int32)]

    def as_tuple(self):
        return (self.bx, self.by, self.variant)


class lbm_monitors(C.Structure):
    _fields_ = [("step", C.c_int64), ("mass", C.c_double), ("mom", C.c_double * 3),
                ("j", C.c_double * 3), ("umax", C.c_double), ("resid", C.c_double),
                ("nonfinite", C.c_int64)]

    def as_dict(self):
        return dict(step=self.step, mass=self.mass, mom=list(self.mom), j=list(self.j),
                    umax=self.umax, resid=self.resid, nonfinite=self.nonfinite)


EXPORTS = {
    "lbm_init": ([C.POINTER(lbm_params), C.c_void_p, C.c_void_p, C.c_void_p,
                  C.POINTER(C.c_void_p)], C.c_int),
    "lbm_save": ([C.c_void_p, C.c_char_p], C.c_int),
    "lbm_load": ([C.c_void_p, C.c_char_p], C.c_int),
    "lbm_step": ([C.c_void_p, C.c_int64, C.c_void_p], C.c_int),
    "lbm_moments": ([C.c_void_p, C.c_double, C.c_void_p, C.c_void_p], C.c_int),
    "lbm_monitors_get": ([C.c_void_p, C.POINTER(lbm_monitors)], C.c_int),
    "lbm_get_populations": ([C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p], C.c_int),
    "lbm_set_populations": ([C.c_void_p, C.c_void_p], C.c_int),
    "lbm_get_populations_noalloc": ([C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p], C.c_int),
    "lbm_set_waves": ([C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "lbm_lattice_info": ([C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_void_p,
                          C.c_void_p], C.c_int),
    "lbm_time": ([C.c_void_p, C.POINTER(C.c_int64)], C.c_int),
    "lbm_device_bytes": ([C.c_void_p, C.POINTER(C.c_size_t)], C.c_int),
    "lbm_free": ([C.c_void_p], C.c_int),
    "lbm_copy_probe": ([C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, C.c_int32, C.c_int32,
                        C.c_void_p], C.c_int),
    "lbm_set_tuning": ([C.c_void_p, C.c_void_p], C.c_int),
    "lbm_get_tuning": ([C.c_void_p, C.c_void_p], C.c_int),
    "lbm_autotune": ([C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_double)], C.c_int),
    "lbm_strerror": ([C.c_int], C.c_char_p),
    "lbm_last_error": ([], C.c_char_p),
    "lbm_version": ([], C.c_int),
}

_lib = None


def load():
    """Load liblbm.so (raises OSError if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"{LIB_PATH} is not built; run python -m paper_2212_07494_amd.build")
        # torch first: liblbm binds libamdhip64 by soname, so whichever copy of the HIP
        # runtime is loaded first serves both; loaded before torch's own copy, the
        # system one leaves torch without a device.  torch supplies device memory and
        # streams here, so its runtime is the one to share.
        import torch  # noqa: F401
        lib = C.CDLL(LIB_PATH)
        for name, (args, res) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _check(rc: int):
    if rc == LBM_WMACH:
        import warnings
        warnings.warn(load().lbm_last_error().decode(errors="replace"), MachWarning,
                      stacklevel=3)
    elif rc != LBM_OK:
        msg = load().lbm_last_error().decode(errors="replace")
        raise LBMError(rc, msg)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)  # torch.cuda.Stream


class TorchAllocator:
    """Device memory for the library from torch's caching allocator (uint8 tensors kept
    alive until the library frees them)."""

    def __init__(self, device="cuda"):
        import torch
        self._torch = torch
        self.device = device
        self.live = {}

        def _alloc(nbytes, user):
            t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device=self.device)
            p = t.data_ptr()
            self.live[p] = t
            return p

        def _free(ptr, user):
            self.live.pop(ptr, None)

        self._a = ALLOC_FN(_alloc)
        self._f = FREE_FN(_free)
        self.struct = lbm_allocator(self._a, self._f, None)


# ---- C-ABI functions ------------------------------------------------------------------

def make_params(lattice="D2Q9", collision="bgk", storage="f64", shape=(1, 1, 1), bc=(0, 0, 0),
                tau=(0.8, 0.8, 1.0), rho0=1.0, g=None, g_profile=None, g_field=None,
                monitor_every=0, allocator=None, force_order=1, solid=None, tau_bulk=0.0,
                tau_31=0.0, max_order=4, mach_limit=0.0, debug_poison=False):
    """Fill an lbm_params.  g: uniform (3,) acceleration; g_profile: (axis, (3, n) table);
    g_field: (3, N) array; force_order 1, 3 or 4 (SMRT force content to that order); solid: N
    flags (nonzero = solid node) or None; mach_limit: warn (MachWarning) when a monitor
    record has max |u| above mach_limit c_s (0 = off); debug_poison: fill the buffer each
    step writes with NaN first.  Returned together with the arrays it points to (keep
    both)."""
    nx, ny, nz = (tuple(shape) + (1, 1))[:3]
    p = lbm_params()
    p.lattice = LATTICES[lattice]
    p.collision = COLLISIONS[collision]
    p.storage = STORAGES[storage]
    p.nx, p.ny, p.nz = nx, ny, nz
    p.bc = (C.c_int32 * 3)(*[int(b) for b in bc])
    tau2, tau3, tau4 = tau
    p.tau = (C.c_double * 5)(0.0, 0.0, tau2, tau3, tau4)
    p.rho0 = rho0
    keep = []
    if g_field is not None:
        arr = np.ascontiguousarray(g_field, dtype=np.float64)
        p.g_kind, p.g_data = G_FIELD, arr.ctypes.data
        keep.append(arr)
    elif g_profile is not None:
        axis, table = g_profile
        arr = np.ascontiguousarray(table, dtype=np.float64)
        p.g_kind, p.g_axis, p.g_data = G_PROFILE, int(axis), arr.ctypes.data
        keep.append(arr)
    else:
        gv = [0.0, 0.0, 0.0] if g is None else [float(v) for v in g]
        p.g_kind = G_UNIFORM
        p.g_uniform = (C.c_double * 3)(*gv)
    p.monitor_every = monitor_every
    p.force_order = int(force_order)
    p.tau_bulk = float(tau_bulk)
    p.tau_31 = float(tau_31)
    p.max_order = int(max_order)
    p.mach_limit = float(mach_limit)
    p.debug_poison = int(bool(debug_poison))
    if solid is not None:
        mask = np.ascontiguousarray(np.asarray(solid).ravel() != 0, dtype=np.uint8)
        if mask.size != nx * ny * nz:
            raise ValueError("solid needs one flag per node")
        p.solid = mask.ctypes.data
        keep.append(mask)
    if allocator is not None:
        p.allocator = C.pointer(allocator.struct)
        keep.append(allocator)
    return p, keep


def lbm_init(params: lbm_params, rho_init=None, u_init=None, stream=None) -> C.c_void_p:
    lib = load()
    out = C.c_void_p()
    r = None if rho_init is None else np.ascontiguousarray(rho_init, dtype=np.float64)
    u = None if u_init is None else np.ascontiguousarray(u_init, dtype=np.float64)
    _check(lib.lbm_init(C.byref(params), _ptr(r), _ptr(u), _stream_handle(stream), C.byref(out)))
    return out


def lbm_step(ctx, n: int, g_scale=None):
    gs = None if g_scale is None else np.ascontiguousarray(g_scale, dtype=np.float64)
    if gs is not None and gs.size < n:
        raise ValueError("g_scale needs n entries")
    _check(load().lbm_step(ctx, int(n), _ptr(gs)))


def lbm_moments(ctx, N: int, D: int, g_scale: float = 1.0):
    rho = np.empty(N)
    u = np.empty((D, N))
    _check(load().lbm_moments(ctx, float(g_scale), _ptr(rho), _ptr(u)))
    return rho, u


def lbm_monitors_get(ctx) -> lbm_monitors:
    """The monitor record; a non-finite state is reported in it (nonfinite > 0), not
    raised."""
    m = lbm_monitors()
    rc = load().lbm_monitors_get(ctx, C.byref(m))
    if rc != LBM_ENONFINITE:
        _check(rc)
    return m


def lbm_get_populations(ctx, Q: int, N: int, nodes=None):
    if nodes is None:
        out = np.empty((Q, N))
        _check(load().lbm_get_populations(ctx, N, None, _ptr(out)))
        return out
    idx = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.empty((Q, idx.size))
    _check(load().lbm_get_populations(ctx, idx.size, _ptr(idx), _ptr(out)))
    return out


def lbm_get_populations_noalloc(ctx, Q: int, N: int, nodes=None):
    """lbm_get_populations staged through the library's fixed device array (no device
    allocation; bounded size, see LBM_NOALLOC_SCRATCH_BYTES)."""
    if nodes is None:
        out = np.empty((Q, N))
        _check(load().lbm_get_populations_noalloc(ctx, N, None, _ptr(out)))
        return out
    idx = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.empty((Q, idx.size))
    _check(load().lbm_get_populations_noalloc(ctx, idx.size, _ptr(idx), _ptr(out)))
    return out


def lbm_set_populations(ctx, f):
    arr = np.ascontiguousarray(f, dtype=np.float64)
    _check(load().lbm_set_populations(ctx, _ptr(arr)))


def lbm_set_waves(ctx, Q, k, phase, amp):
    """State w_i rho0 + sum_w Re[amp[w, i] exp(i theta_w)] (lbm_set_waves) on a context
    of Q populations; k: (n, 3) integers, phase: (n,), amp: (n, Q) complex."""
    k = np.asarray(k)
    if k.ndim != 2 or k.shape[1] != 3 or not np.all(k == np.round(k)):
        raise ValueError(f"k must be an (n, 3) integer array, got shape {k.shape}")
    k = np.ascontiguousarray(k, dtype=np.int32)
    n = k.shape[0]
    ph = np.ascontiguousarray(np.asarray(phase, np.float64).reshape(n))
    a = np.asarray(amp, np.complex128)
    if n and a.shape != (n, Q):
        raise ValueError(f"amp must have shape ({n}, {Q}), got {a.shape}")
    if not n:
        a = np.zeros((0, Q), np.complex128)
    ri = np.ascontiguousarray(np.stack([a.real, a.imag], axis=-1))
    _check(load().lbm_set_waves(ctx, n, _ptr(k), _ptr(ph), _ptr(ri)))


def lbm_lattice_info(lattice):
    """(velocities (Q, 3) int32, weights (Q,) binary64) of a lattice, in population order."""
    Q = QOF[lattice]
    e = np.zeros((Q, 3), np.int32)
    w = np.zeros(Q, np.float64)
    D, q = C.c_int32(), C.c_int32()
    _check(load().lbm_lattice_info(LATTICES[lattice], C.byref(D), C.byref(q), _ptr(e), _ptr(w)))
    return e, w


def lbm_time(ctx) -> int:
    t = C.c_int64()
    _check(load().lbm_time(ctx, C.byref(t)))
    return t.value


def lbm_device_bytes(ctx) -> int:
    b = C.c_size_t()
    _check(load().lbm_device_bytes(ctx, C.byref(b)))
    return b.value


def lbm_free(ctx):
    _check(load().lbm_free(ctx))


def lbm_copy_probe(src_ptr: int, dst_ptr: int, nbytes: int, reps: int = 1, block: int = 256,
                   variant: int = 0, stream=None):
    _check(load().lbm_copy_probe(C.c_void_p(src_ptr), C.c_void_p(dst_ptr), int(nbytes), int(reps),
                                 int(block), int(variant), _stream_handle(stream)))


def lbm_set_tuning(ctx, bx: int, by: int, variant: int):
    t = lbm_tuning(bx, by, variant)
    _check(load().lbm_set_tuning(ctx, C.byref(t)))


def lbm_get_tuning(ctx):
    t = lbm_tuning()
    _check(load().lbm_get_tuning(ctx, C.byref(t)))
    return t.as_tuple()


def lbm_autotune(ctx, steps: int = 10):
    t = lbm_tuning()
    ms = C.c_double()
    _check(load().lbm_autotune(ctx, int(steps), C.byref(t), C.byref(ms)))
    return t.as_tuple(), ms.value


# ---- convenience object -----------------------------------------------------------------

class Lattice:
    """Owns one lbm context (created by lbm_init, released by close())."""

    def __init__(self, lattice="D2Q9", collision="bgk", storage="f64", shape=(1, 1, 1),
                 walls=(0, 0, 0), tau=(0.8, 0.8, 1.0), rho0=1.0, rho=None, u=None, g=None,
                 g_profile=None, g_field=None, monitor_every=0, stream=None, allocator=None,
                 force_order=1, solid=None, tau_bulk=0.0, tau_31=0.0, max_order=4,
                 mach_limit=0.0, debug_poison=False):
        self.lattice = lattice
        self.Q = QOF[lattice]
        self.D = 2 if lattice == "D2Q9" else 3
        nx, ny, nz = (tuple(shape) + (1, 1))[:3]
        self.shape = (nx, ny, nz)
        self.N = nx * ny * nz
        self.storage = storage
        self._params, self._keep = make_params(lattice, collision, storage, self.shape, walls, tau,
                                               rho0, g, g_profile, g_field, monitor_every,
                                               allocator, force_order, solid, tau_bulk,
                                               tau_31, max_order, mach_limit, debug_poison)
        if u is not None:
            u = np.asarray(u, dtype=np.float64)[: self.D]
        self.ctx = lbm_init(self._params, rho, u, stream)

    def step(self, n=1, g_scale=None):
        lbm_step(self.ctx, n, g_scale)

    def save(self, path):
        """Checkpoint: state as stored, time and parameter identity (lbm_save)."""
        _check(load().lbm_save(self.ctx, os.fsencode(path)))

    def load(self, path):
        """Resume from a checkpoint of a lattice with the same parameters (lbm_load)."""
        _check(load().lbm_load(self.ctx, os.fsencode(path)))

    def moments(self, g_scale=1.0):
        return lbm_moments(self.ctx, self.N, self.D, g_scale)

    def monitors(self):
        return lbm_monitors_get(self.ctx)

    def tune(self, bx=None, by=None, variant=None, autotune_steps=None):
        """Set the launch configuration, or time all of them (autotune_steps) and keep the
        fastest; returns (bx, by, variant)."""
        if autotune_steps:
            return lbm_autotune(self.ctx, autotune_steps)[0]
        cur = lbm_get_tuning(self.ctx)
        lbm_set_tuning(self.ctx, bx or cur[0], by or cur[1], cur[2] if variant is None else variant)
        return lbm_get_tuning(self.ctx)

    def populations(self, nodes=None):
        return lbm_get_populations(self.ctx, self.Q, self.N, nodes)

    def set_populations(self, f):
        lbm_set_populations(self.ctx, f)

    def set_waves(self, k, phase, amp):
        lbm_set_waves(self.ctx, self.Q, k, phase, amp)

    @property
    def time(self):
        return lbm_time(self.ctx)

    def close(self):
        if self.ctx:
            lbm_free(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- batched engine (include/lbm_batch.h) ------------------------------------------------

class lbm_domain(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("bc", C.c_int32 * 3),
                ("tau", C.c_double * 5), ("g_kind", C.c_int32), ("g_axis", C.c_int32),
                ("g_uniform", C.c_double * 3), ("g_data", C.c_void_p), ("rho_init", C.c_void_p),
                ("u_init", C.c_void_p)]


class lbm_batch_tuning(C.Structure):
    _fields_ = [("tile_bx", C.c_int32), ("blocks_per_cu", C.c_int32), ("variant", C.c_int32)]

    def as_tuple(self):
        return (self.tile_bx, self.blocks_per_cu, self.variant)


DOM_RUNNING, DOM_CONVERGED, DOM_FLOOR, DOM_NONFINITE = 0, 1, 2, 3

EXPORTS_BATCH = {
    "lbm_batch_init": ([C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                        C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "lbm_batch_advance": ([C.c_void_p, C.c_int64], C.c_int),
    "lbm_batch_run": ([C.c_void_p, C.c_int64, C.c_double, C.c_int32, C.c_int32, C.c_void_p,
                       C.c_void_p, C.c_void_p], C.c_int),
    "lbm_batch_step": ([C.c_void_p, C.c_int64, C.c_double, C.c_void_p, C.c_void_p], C.c_int),
    "lbm_batch_status": ([C.c_void_p, C.c_void_p], C.c_int),
    "lbm_batch_moments": ([C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p], C.c_int),
    "lbm_batch_get_populations": ([C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "lbm_batch_set_populations": ([C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "lbm_batch_set_tuning": ([C.c_void_p, C.c_void_p], C.c_int),
    "lbm_batch_get_tuning": ([C.c_void_p, C.c_void_p], C.c_int),
    "lbm_batch_autotune": ([C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_double)], C.c_int),
    "lbm_batch_info": ([C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                        C.POINTER(C.c_size_t)], C.c_int),
    "lbm_batch_free": ([C.c_void_p], C.c_int),
}
EXPORTS.update(EXPORTS_BATCH)


def make_domain(shape, walls=(0, 0, 0), tau=(0.8, 0.8, 1.0), g=None, g_profile=None,
                g_field=None, rho=None, u=None):
    """Fill an lbm_domain; returns (struct, arrays it points to)."""
    nx, ny, nz = (tuple(shape) + (1, 1))[:3]
    d = lbm_domain()
    d.nx, d.ny, d.nz = nx, ny, nz
    d.bc = (C.c_int32 * 3)(*[int(w) for w in walls])
    d.tau = (C.c_double * 5)(0.0, 0.0, *tau)
    keep = []
    if g_field is not None:
        arr = np.ascontiguousarray(g_field, dtype=np.float64)
        d.g_kind, d.g_data = G_FIELD, arr.ctypes.data
        keep.append(arr)
    elif g_profile is not None:
        axis, table = g_profile
        arr = np.ascontiguousarray(table, dtype=np.float64)
        d.g_kind, d.g_axis, d.g_data = G_PROFILE, int(axis), arr.ctypes.data
        keep.append(arr)
    else:
        d.g_kind = G_UNIFORM
        d.g_uniform = (C.c_double * 3)(*([0.0] * 3 if g is None else [float(v) for v in g]))
    for name, val in (("rho_init", rho), ("u_init", u)):
        if val is not None:
            arr = np.ascontiguousarray(val, dtype=np.float64)
            setattr(d, name, arr.ctypes.data)
            keep.append(arr)
    return d, keep


class Batch:
    """Owns one lbm_batch context: many domains stepped by one persistent launch."""

    def __init__(self, domains, lattice="D2Q9", collision="smrt", storage="f32s", rho0=1.0,
                 stream=None):
        """domains: list of dicts with keys shape, walls, tau, and g / g_profile / g_field,
        optionally rho, u."""
        lib = load()
        self.lattice = lattice
        self.Q = QOF[lattice]
        self.D = 2 if lattice == "D2Q9" else 3
        self.shapes = []
        structs, self._keep = [], []
        for dd in domains:
            s, keep = make_domain(**dd)
            structs.append(s)
            self._keep.extend(keep)
            self.shapes.append((s.nx, s.ny, s.nz))
        arr = (lbm_domain * len(structs))(*structs)
        out = C.c_void_p()
        _check(lib.lbm_batch_init(C.cast(arr, C.c_void_p), len(structs), LATTICES[lattice],
                                  COLLISIONS[collision], STORAGES[storage], rho0,
                                  _stream_handle(stream), C.byref(out)))
        self.ctx = out
        self.ndom = len(structs)

    def advance(self, n):
        _check(load().lbm_batch_advance(self.ctx, int(n)))

    def run(self, max_steps, tol, check_every=200, stall_checks=10):
        steps = np.zeros(self.ndom, np.int64)
        resid = np.zeros(self.ndom)
        status = np.zeros(self.ndom, np.int32)
        _check(load().lbm_batch_run(self.ctx, int(max_steps), float(tol), int(check_every),
                                    int(stall_checks), _ptr(steps), _ptr(resid), _ptr(status)))
        return steps, resid, status

    def step(self, max_steps, tol):
        """lbm_batch_step: every domain to resid < tol (or its floor, or max_steps);
        returns steps, resid and the per-domain status (lbm_batch_status)."""
        steps = np.zeros(self.ndom, np.int64)
        resid = np.zeros(self.ndom)
        _check(load().lbm_batch_step(self.ctx, int(max_steps), float(tol), _ptr(steps),
                                     _ptr(resid)))
        return steps, resid, self.status()

    def status(self):
        st = np.zeros(self.ndom, np.int32)
        _check(load().lbm_batch_status(self.ctx, _ptr(st)))
        return st

    def N(self, d):
        nx, ny, nz = self.shapes[d]
        return nx * ny * nz

    def moments(self, d):
        rho = np.empty(self.N(d))
        u = np.empty((self.D, self.N(d)))
        _check(load().lbm_batch_moments(self.ctx, int(d), _ptr(rho), _ptr(u)))
        return rho, u

    def populations(self, d):
        f = np.empty((self.Q, self.N(d)))
        _check(load().lbm_batch_get_populations(self.ctx, int(d), _ptr(f)))
        return f

    def set_populations(self, d, f):
        arr = np.ascontiguousarray(f, dtype=np.float64)
        _check(load().lbm_batch_set_populations(self.ctx, int(d), _ptr(arr)))

    def tune(self, tile_bx=None, blocks_per_cu=None, variant=None, autotune_steps=None):
        lib = load()
        if autotune_steps:
            t = lbm_batch_tuning()
            ms = C.c_double()
            _check(lib.lbm_batch_autotune(self.ctx, int(autotune_steps), C.byref(t), C.byref(ms)))
            return t.as_tuple(), ms.value
        t = lbm_batch_tuning()
        _check(lib.lbm_batch_get_tuning(self.ctx, C.byref(t)))
        if tile_bx is not None:
            t.tile_bx = tile_bx
        if blocks_per_cu is not None:
            t.blocks_per_cu = blocks_per_cu
        if variant is not None:
            t.variant = variant
        _check(lib.lbm_batch_set_tuning(self.ctx, C.byref(t)))
        return t.as_tuple(), None

    def info(self):
        n, t, b = C.c_int64(), C.c_int64(), C.c_size_t()
        _check(load().lbm_batch_info(self.ctx, C.byref(n), C.byref(t), C.byref(b)))
        return dict(nodes=n.value, tiles=t.value, bytes=b.value)

    def close(self):
        if self.ctx:
            _check(load().lbm_batch_free(self.ctx))
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- warm-start network (include/lbm_nn.h) -----------------------------------------------

class lbm_ws_problem(C.Structure):
    _fields_ = [("tau2", C.c_double), ("nmodes", C.c_int32), ("k", (C.c_double * 3) * 8),
                ("p", (C.c_double * 3) * 8), ("amp", C.c_double * 8), ("phase", C.c_double * 8)]


WS_FEATURES = 46
WS_RESUM_FEATURES = 19
WS_MODE_FEATURES = 13
RESET_MASS, RESET_MOMENTUM, RESET_FILTER, RESET_NONEQ = 1, 2, 4, 8

EXPORTS_NN = {
    "lbm_mlp_create": ([C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.POINTER(C.c_void_p)],
                       C.c_int),
    "lbm_mlp_num_params": ([C.c_void_p, C.POINTER(C.c_int64)], C.c_int),
    "lbm_mlp_set_params": ([C.c_void_p, C.c_void_p, C.c_int64], C.c_int),
    "lbm_mlp_get_params": ([C.c_void_p, C.c_void_p, C.c_int64], C.c_int),
    "lbm_mlp_get_grads": ([C.c_void_p, C.c_void_p, C.c_int64], C.c_int),
    "lbm_mlp_forward": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p], C.c_int),
    "lbm_mlp_loss_backward": ([C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)],
                              C.c_int),
    "lbm_mlp_backward": ([C.c_void_p, C.c_void_p], C.c_int),
    "lbm_mlp_zero_grads": ([C.c_void_p], C.c_int),
    "lbm_mlp_adam": ([C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int64],
                     C.c_int),
    "lbm_mlp_free": ([C.c_void_p], C.c_int),
    "lbm_ws_features": ([C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                         C.c_double, C.c_void_p, C.POINTER(C.c_double), C.c_void_p], C.c_int),
    "lbm_ws_mode_features": ([C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p], C.c_int),
    "lbm_ws_lattice_response": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "lbm_ws_lattice_waves": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)],
                             C.c_int),
    "lbm_ws_max_waves": ([C.c_int32, C.c_int32], C.c_int32),
    "lbm_ws_lattice_waves_ordered": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32),
                                      C.c_void_p], C.c_int),
    "lbm_ws_resum_features": ([C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.POINTER(C.c_double)], C.c_int),
    "lbm_ws_scale_orders": ([C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p], C.c_int),
    "lbm_mlp_set_output_scale": ([C.c_void_p, C.c_void_p], C.c_int),
    "lbm_mlp_loss_grad": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                           C.POINTER(C.c_double)], C.c_int),
    "lbm_reset_fields": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_int32],
                         C.c_int),
}
EXPORTS.update(EXPORTS_NN)


def _dptr(t):
    """Device pointer of a torch tensor (or an int)."""
    return C.c_void_p(t if isinstance(t, int) else t.data_ptr())


class MLP:
    """Owns one lbm_mlp: BF16 per-point network with FP32 master weights.  Device arrays
    are torch float32 CUDA tensors (row-major, one row per point)."""

    def __init__(self, widths, max_rows, stream=None):
        lib = load()
        self.widths = list(widths)
        arr = (C.c_int32 * len(widths))(*widths)
        out = C.c_void_p()
        _check(lib.lbm_mlp_create(C.cast(arr, C.c_void_p), len(widths) - 1, int(max_rows),
                                  _stream_handle(stream), C.byref(out)))
        self.ctx = out
        n = C.c_int64()
        _check(lib.lbm_mlp_num_params(self.ctx, C.byref(n)))
        self.nparams = n.value

    def set_params(self, p):
        arr = np.ascontiguousarray(p, dtype=np.float32)
        _check(load().lbm_mlp_set_params(self.ctx, _ptr(arr), arr.size))

    def params(self):
        out = np.empty(self.nparams, np.float32)
        _check(load().lbm_mlp_get_params(self.ctx, _ptr(out), out.size))
        return out

    def grads(self):
        out = np.empty(self.nparams, np.float32)
        _check(load().lbm_mlp_get_grads(self.ctx, _ptr(out), out.size))
        return out

    def forward(self, x, y, addend=None):
        """y = network(x) (+ addend, same shape as y)."""
        _check(load().lbm_mlp_forward(self.ctx, _dptr(x), int(x.shape[0]),
                                      _optr(addend), _dptr(y)))

    def zero_grads(self):
        _check(load().lbm_mlp_zero_grads(self.ctx))

    def set_output_scale(self, scale):
        s = np.ascontiguousarray(scale, np.float32)
        _check(load().lbm_mlp_set_output_scale(self.ctx, _ptr(s)))

    def loss_grad(self, y, target, dy, weight=None):
        """Weighted mean-square loss of any y against target; dL/dy into dy."""
        w = None if weight is None else np.ascontiguousarray(weight, np.float32)
        loss = C.c_double()
        _check(load().lbm_mlp_loss_grad(self.ctx, _dptr(y), _dptr(target), _ptr(w),
                                        int(y.shape[0]), _dptr(dy), C.byref(loss)))
        return loss.value

    def loss_backward(self, target, weight=None):
        w = None if weight is None else np.ascontiguousarray(weight, np.float32)
        loss = C.c_double()
        _check(load().lbm_mlp_loss_backward(self.ctx, _dptr(target), _ptr(w), C.byref(loss)))
        return loss.value

    def backward(self, dy):
        _check(load().lbm_mlp_backward(self.ctx, _dptr(dy)))

    def adam(self, lr, t, b1=0.9, b2=0.999, eps=1e-8):
        _check(load().lbm_mlp_adam(self.ctx, lr, b1, b2, eps, int(t)))

    def close(self):
        if self.ctx:
            _check(load().lbm_mlp_free(self.ctx))
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ws_problem_struct(problem):
    """lbm_ws_problem from dict(tau2, modes=[dict(k, p, amp, phase)])."""
    s = lbm_ws_problem()
    s.tau2 = problem["tau2"]
    s.nmodes = len(problem["modes"])
    for j, m in enumerate(problem["modes"]):
        for a in range(3):
            s.k[j][a] = float(m["k"][a])
            s.p[j][a] = float(m["p"][a])
        s.amp[j] = m["amp"]
        s.phase[j] = m["phase"]
    return s


def lbm_ws_features(problem, n, box, x_dev, base_dev=None, base_order=2, rho_scale=1.0,
                    mode_coef=None, stream=None):
    """Features into x_dev (n^3 x WS_FEATURES, may be None), the perturbative steady
    solution of order base_order (1: Stokes, 2: with the first advective correction) into
    base_dev (n^3 x 4: u / U, (rho - 1) / (U rho_scale)) if given, each mode's own
    response corrected by mode_coef (device, 4 x 8) if given; returns the scale U."""
    s = ws_problem_struct(problem)
    U = C.c_double()
    _check(load().lbm_ws_features(C.byref(s), int(n), int(box), _optr(x_dev),
                                  _optr(base_dev), int(base_order), float(rho_scale),
                                  _optr(mode_coef), C.byref(U), _stream_handle(stream)))
    return U.value


def lbm_ws_mode_features(problem, box, out_dev, stream=None):
    """Per-mode network inputs (nmodes x WS_MODE_FEATURES, device)."""
    s = ws_problem_struct(problem)
    _check(load().lbm_ws_mode_features(C.byref(s), int(box), _dptr(out_dev),
                                       _stream_handle(stream)))


def lbm_ws_lattice_response(problem, box, lattice="D3Q27", collision="smrt", tau3=1.0,
                            rho0=1.0, **rates):
    """Each mode's exact linear steady response on the periodic lattice as mode_coef
    coefficients (nmodes x 8, binary64, host); rates: tau_bulk, tau_31, max_order,
    force_order as for make_params."""
    s = ws_problem_struct(problem)
    params, keep = make_params(lattice, collision, "f64", (1, 1, 1),
                               tau=(problem["tau2"], tau3, 1.0), rho0=rho0, **rates)
    out = np.zeros((int(s.nmodes), 8), np.float64)
    _check(load().lbm_ws_lattice_response(C.byref(params), C.byref(s), int(box),
                                          out.ctypes.data))
    return out


def lbm_ws_lattice_waves(problem, box, order=2, lattice="D3Q27", collision="smrt", tau3=1.0,
                         rho0=1.0, **rates):
    """The steady state of the problem's forced periodic lattice to order 1 to 4 in the
    forcing, as waves for lbm_set_waves: k (n, 3) int32, phase (n,), amp (n, Q) complex;
    rates as for lbm_ws_lattice_response."""
    s = ws_problem_struct(problem)
    params, keep = make_params(lattice, collision, "f64", (1, 1, 1),
                               tau=(problem["tau2"], tau3, 1.0), rho0=rho0, **rates)
    Q = QOF[lattice.upper()]
    nm = int(s.nmodes)
    cap = int(load().lbm_ws_max_waves(nm, int(order)))
    if cap == 0:
        raise LBMError(LBM_EINVAL, f"nmodes = {nm} or order = {order} out of range")
    k = np.zeros((cap, 3), np.int32)
    ph = np.zeros(cap, np.float64)
    amp = np.zeros((cap, Q, 2), np.float64)
    count = C.c_int32()
    _check(load().lbm_ws_lattice_waves(C.byref(params), C.byref(s), int(box), int(order), cap,
                                       _ptr(k), _ptr(ph), _ptr(amp), C.byref(count)))
    n = count.value
    return k[:n].copy(), ph[:n].copy(), amp[:n, :, 0] + 1j * amp[:n, :, 1]


def lbm_ws_lattice_waves_ordered(problem, box, order=4, lattice="D3Q27", collision="smrt",
                                 tau3=1.0, rho0=1.0, **rates):
    """lbm_ws_lattice_waves with the order boundaries: (k, phase, amp (n, Q, 2) binary64,
    order_end (4,) int32); order n's waves are [order_end[n-2], order_end[n-1])."""
    s = ws_problem_struct(problem)
    params, keep = make_params(lattice, collision, "f64", (1, 1, 1),
                               tau=(problem["tau2"], tau3, 1.0), rho0=rho0, **rates)
    Q = QOF[lattice.upper()]
    cap = int(load().lbm_ws_max_waves(int(s.nmodes), int(order)))
    if cap == 0:
        raise LBMError(LBM_EINVAL, f"nmodes = {int(s.nmodes)} or order = {order} out of range")
    k = np.zeros((cap, 3), np.int32)
    ph = np.zeros(cap, np.float64)
    amp = np.zeros((cap, Q, 2), np.float64)
    ends = np.zeros(4, np.int32)
    count = C.c_int32()
    _check(load().lbm_ws_lattice_waves_ordered(C.byref(params), C.byref(s), int(box), int(order),
                                               cap, _ptr(k), _ptr(ph), _ptr(amp), C.byref(count),
                                               _ptr(ends)))
    n = count.value
    return k[:n].copy(), ph[:n].copy(), np.ascontiguousarray(amp[:n]), ends


def lbm_ws_resum_features(problem, box, amp, order_end):
    """Network inputs (WS_RESUM_FEATURES float32) and sigma of a problem and its order-4
    waves (amp: (n, Q, 2) binary64 as returned by lbm_ws_lattice_waves_ordered)."""
    s = ws_problem_struct(problem)
    a = np.ascontiguousarray(amp, np.float64)
    ends = np.ascontiguousarray(order_end, np.int32)
    feat = np.zeros(WS_RESUM_FEATURES, np.float32)
    sigma = C.c_double()
    _check(load().lbm_ws_resum_features(C.byref(s), int(box), int(a.shape[1]), _ptr(a),
                                        _ptr(ends), _ptr(feat), C.byref(sigma)))
    return feat, sigma.value


def lbm_ws_scale_orders(amp, order_end, c):
    """Scale each order's waves of amp ((n, Q, 2) binary64, in place) by c (4,)."""
    if amp.dtype != np.float64 or not amp.flags.c_contiguous:
        raise ValueError("amp must be a C-contiguous float64 array")
    ends = np.ascontiguousarray(order_end, np.int32)
    cc = np.ascontiguousarray(c, np.float64)
    _check(load().lbm_ws_scale_orders(_ptr(amp), int(amp.shape[1]), _ptr(ends), _ptr(cc)))
    return amp


def _optr(t):
    return None if t is None else _dptr(t)


def lbm_reset_fields(ctx, fields, layout, U=1.0, R=None, flags=0):
    """layout 0: planes rho, u; 1: network rows (u/U, (rho-rho0)/R); 2: those as planes
    (R defaults to U).  flags: RESET_FILTER (periodic low-pass removing wavenumber pi),
    RESET_MASS and RESET_MOMENTUM (project onto the plain start's totals)."""
    R = U if R is None else R
    _check(load().lbm_reset_fields(ctx, _dptr(fields), int(layout), float(U), float(R), int(flags)))
