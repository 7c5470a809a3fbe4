"""CPU oracle of the forced lattice-Boltzmann step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does, and this
package never imports the product package.

The arithmetic lives in ``lbm_oracle.c`` (built by ``oracle/build.py`` into a
double and a float library); this module only marshals NumPy arrays.  Array
layout: populations ``f[i, n]`` with ``n = (z*ny + y)*nx + x`` (x fastest), the
stored value being ``f-bar_i - w_i * shift``; velocity and acceleration fields
``u[a, n]`` / ``g[a, n]`` with three component planes (z plane zero in 2-D).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build
from . import lattice as lat

_LIBS: dict = {}


class _Lattice(C.Structure):
    _fields_ = [("D", C.c_int32), ("Q", C.c_int32), ("NM", C.c_int32),
                ("e", C.c_void_p), ("opp", C.c_void_p), ("mi", C.c_void_p),
                ("w", C.c_void_p), ("H", C.c_void_p), ("Minv", C.c_void_p),
                ("ics2", C.c_double)]


def _params_struct(real_t):
    class _Params(C.Structure):
        _fields_ = [("collision", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                    ("nz", C.c_int32), ("wall", C.c_int32 * 3), ("store16", C.c_int32),
                    ("shift", real_t), ("omega", real_t), ("hforce", real_t),
                    ("q2", real_t), ("q3", real_t), ("fq3", real_t), ("h2", real_t),
                    ("h3", real_t), ("dqb", real_t), ("dq31", real_t), ("max_order", C.c_int32),
                    ("fo4", C.c_int32), ("solid", C.c_void_p)]
    return _Params


_P64 = _params_struct(C.c_double)
_P32 = _params_struct(C.c_float)


def _lib(kind: str):
    if kind not in _LIBS:
        path = _build.lib_path(kind)
        if not os.path.exists(path):
            _build.build(force=False)
        L = C.CDLL(path)
        vp = C.c_void_p
        real = C.c_float if kind == "f32" else C.c_double
        L.oracle_step.argtypes = [vp, vp, vp, vp, vp, real]
        L.oracle_run.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int64]
        L.oracle_init.argtypes = [vp, vp, vp, vp, vp, vp]
        L.oracle_moments.argtypes = [vp, vp, vp, vp, real, vp, vp]
        L.oracle_collide_node.argtypes = [vp, vp, vp, vp, vp]
        L.oracle_init_node.argtypes = [vp, vp, real, vp, vp, vp]
        L.oracle_bgk_terms.argtypes = [vp, real, vp, vp, vp, vp]
        L.oracle_round_half.argtypes = [C.c_float]
        L.oracle_round_half.restype = C.c_float
        L.oracle_is_plain.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = C.c_int
        _LIBS[kind] = L
    return _LIBS[kind]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def set_threads(n: int, real: str = "f64") -> int:
    """Threads of the oracle's whole-lattice loops (n <= 0: leave); the count in effect."""
    return int(_lib(real).oracle_set_threads(int(n)))


def round_half(x: float) -> float:
    """The oracle's own binary16 rounding (IEEE round to nearest even)."""
    return float(_lib("f32").oracle_round_half(float(x)))


class Oracle:
    """Plain forced LB step on one periodic / walled box.

    lattice: 'D2Q9' | 'D3Q19' | 'D3Q27' | 'D3Q39' (the high-order lattice: periodic boxes,
    no solid nodes, no tau_31); collision: 'bgk' | 'smrt' | 'rmrt' (the raw-moment MRT of
    the paper's appendix);
    shape (nx, ny, nz) (nz = 1 in 2-D); walls: per-axis flags (halfway bounce-back
    on both faces); tau: dict or tuple of tau-hat per Hermite order (tau2, tau3,
    tau4) -- BGK uses tau2 only, SMRT and RMRT require tau4 == 1 (order 4 is trimmed);
    shift: constant s removed from stored populations (f-bar_i - w_i s);
    real: 'f64' (reference) or 'f32' (emulation); store16: round stores to binary16;
    plain: use the PLAIN build (FP64 only): the textbook operation order (plain sums over
    all populations, plain inverse-transform rows, no fused multiply-add) instead of the
    operation-order twin the library is compared with bit for bit;
    force_order: 1, or 3 for SMRT's third-order force content, or 4 for the third- and
    fourth-order content (not on D3Q39, not with max_order 6); solid: N flags of solid
    nodes (halfway bounce-back against them; not stepped; zero moments) or None;
    tau_bulk: SMRT rate of the trace of order 2 (0 = tau2); tau_31: SMRT rate of the trace
    of order 3 on D3Q19/D3Q27 (0 = tau3); max_order: 4 (raw moments above order 4
    dropped after the collision), or 6 on D3Q27 (orders 5-6 carried, their central
    parts trimmed).
    """

    def __init__(self, lattice: str, collision: str, shape, walls=(0, 0, 0), tau=(0.8, 0.8, 1.0),
                 shift: float = 0.0, real: str = "f64", store16: bool = False,
                 force_order: int = 1, solid=None, tau_bulk: float = 0.0,
                 tau_31: float = 0.0, max_order: int = 4, plain: bool = False):
        self.lattice = lattice
        self.collision = collision.lower()
        nx, ny, nz = (tuple(shape) + (1, 1))[:3]
        self.shape = (nx, ny, nz)
        self.N = nx * ny * nz
        self.real = real
        self.dtype = np.float64 if real == "f64" else np.float32
        self.L = lat.tables(lattice, self.dtype)
        self.Q = self.L["Q"]
        self.D = self.L["D"]
        tau2, tau3, tau4 = tau
        if min(tau2, tau3) <= 0.5:
            raise ValueError("tau-hat must exceed 1/2")
        if self.collision not in ("bgk", "smrt", "rmrt"):
            raise ValueError(f"unknown collision {collision}")
        if self.collision in ("smrt", "rmrt") and tau4 != 1.0:
            raise ValueError("SMRT and RMRT trim order 4: tau4 must be 1")
        self._lat = _Lattice(self.L["D"], self.L["Q"], self.L["NM"],
                             self.L["e"].ctypes.data, self.L["opp"].ctypes.data,
                             self.L["mi"].ctypes.data, self.L["w"].ctypes.data,
                             self.L["H"].ctypes.data, self.L["Minv"].ctypes.data,
                             float(self.L["ics2"]))
        if lattice in lat.HIGH_ORDER and (any(walls) or solid is not None or tau_31):
            raise ValueError(f"{lattice} takes periodic boxes without solid nodes or tau_31")
        omega = 1.0 / tau2
        if force_order not in (1, 3, 4) or (force_order > 1 and self.collision != "smrt"):
            raise ValueError("force_order is 1, or 3 or 4 with SMRT")
        if force_order == 4 and lattice in lat.HIGH_ORDER:
            raise ValueError(f"{lattice} does not resolve the fourth-order moments independently")
        fq3 = (1.0 - 0.5 / tau3) if force_order >= 3 else 0.0
        if tau_bulk and (self.collision != "smrt" or tau_bulk <= 0.5):
            raise ValueError("tau_bulk is for SMRT and must exceed 1/2")
        dim = 2 if self.lattice == "D2Q9" else 3
        dqb = (((1.0 - 1.0 / tau_bulk) - (1.0 - 1.0 / tau2)) / dim
               if tau_bulk and tau_bulk != tau2 else 0.0)
        if tau_31 and (self.collision != "smrt" or lattice == "D2Q9" or force_order >= 3
                       or tau_31 <= 0.5):
            raise ValueError("tau_31 is for SMRT on D3Q19/D3Q27, without force_order 3 or 4, "
                             "and must exceed 1/2")
        dq31 = ((1.0 - 1.0 / tau_31) - (1.0 - 1.0 / tau3)) / 2 if tau_31 and tau_31 != tau3 else 0.0
        if max_order not in (4, 6) or (max_order == 6 and (self.collision != "smrt"
                                                            or lattice != "D3Q27")):
            raise ValueError("max_order is 4, or 6 for SMRT on D3Q27")
        if max_order == 6 and force_order == 4:
            raise ValueError("force_order 4 is not combined with max_order 6")
        vals = dict(shift=shift, omega=omega, hforce=1.0 - 0.5 * omega,
                    q2=1.0 - 1.0 / tau2, q3=1.0 - 1.0 / tau3, fq3=fq3,
                    h2=1.0 - 0.5 / tau2, h3=1.0 - 0.5 / tau3, dqb=dqb, dq31=dq31)
        P = _P64 if real == "f64" else _P32
        cast = float if real == "f64" else (lambda v: float(np.float32(v)))
        self._p = P({"bgk": 0, "smrt": 1, "rmrt": 2}[self.collision], nx, ny, nz,
                    (C.c_int32 * 3)(*[int(bool(w)) for w in walls]), int(bool(store16)),
                    *[cast(vals[k]) for k in ("shift", "omega", "hforce", "q2", "q3", "fq3",
                                              "h2", "h3", "dqb", "dq31")], int(max_order),
                    int(force_order == 4))
        self.solid = None
        if solid is not None:
            self.solid = np.ascontiguousarray(np.asarray(solid).ravel() != 0, dtype=np.uint8)
            if self.solid.size != self.N:
                raise ValueError("solid needs one flag per node")
            self._p.solid = self.solid.ctypes.data
        if plain and real != "f64":
            raise ValueError("the plain build is binary64")
        self.plain = bool(plain)
        self._l = _lib("plain" if plain else real)
        self._lref = C.byref(self._lat)
        self._pref = C.byref(self._p)

    # ---- helpers ------------------------------------------------------------------
    def _arr(self, a, rows):
        a = np.ascontiguousarray(a, dtype=self.dtype)
        return a.reshape(rows, self.N)

    def field(self, g):
        """Broadcast an acceleration (3,), (3, N) or None to a (3, N) array."""
        if g is None:
            return np.zeros((3, self.N), self.dtype)
        g = np.asarray(g, dtype=np.float64)
        if g.ndim == 1:
            g = np.repeat(g[:, None], self.N, axis=1)
        return self._arr(g, 3)

    # ---- whole-lattice operations -------------------------------------------------
    def init(self, rho, u, g):
        rho = self._arr(np.broadcast_to(np.asarray(rho, np.float64), (self.N,)), 1)
        u = self.field(u)
        g = self.field(g)
        f = np.empty((self.Q, self.N), self.dtype)
        self._l.oracle_init(self._lref, self._pref, _ptr(rho), _ptr(u), _ptr(g), _ptr(f))
        return f

    def step(self, f, g, gscale: float = 1.0):
        f = self._arr(f, self.Q)
        g = self.field(g)
        out = np.empty_like(f)
        self._l.oracle_step(self._lref, self._pref, _ptr(f), _ptr(out), _ptr(g), gscale)
        return out

    def run(self, f, g, nsteps: int, gscale=None):
        f = self._arr(f, self.Q).copy()
        g = self.field(g)
        tmp = np.empty_like(f)
        gs = None
        if gscale is not None:
            gs = np.ascontiguousarray(gscale, dtype=self.dtype)
            assert gs.shape == (nsteps,)
        self._l.oracle_run(self._lref, self._pref, _ptr(f), _ptr(tmp), _ptr(g),
                           None if gs is None else _ptr(gs), int(nsteps))
        return f

    def moments(self, f, g, gscale: float = 1.0):
        f = self._arr(f, self.Q)
        g = self.field(g)
        rho = np.empty(self.N, self.dtype)
        u = np.empty((3, self.N), self.dtype)
        self._l.oracle_moments(self._lref, self._pref, _ptr(f), _ptr(g), gscale,
                               _ptr(rho), _ptr(u))
        return rho, u

    # ---- single-node pieces (pins) --------------------------------------------------
    def collide_node(self, f, g):
        f = np.ascontiguousarray(f, self.dtype)
        g = np.ascontiguousarray(np.resize(np.asarray(g, np.float64), 3), self.dtype)
        out = np.empty(self.Q, self.dtype)
        self._l.oracle_collide_node(self._lref, self._pref, _ptr(f), _ptr(g), _ptr(out))
        return out

    def init_node(self, rho, u, g):
        u = np.ascontiguousarray(np.resize(np.asarray(u, np.float64), 3), self.dtype)
        g = np.ascontiguousarray(np.resize(np.asarray(g, np.float64), 3), self.dtype)
        out = np.empty(self.Q, self.dtype)
        self._l.oracle_init_node(self._lref, self._pref, rho, _ptr(u), _ptr(g), _ptr(out))
        return out

    def bgk_terms(self, rho, u, g):
        u = np.ascontiguousarray(np.resize(np.asarray(u, np.float64), 3), self.dtype)
        g = np.ascontiguousarray(np.resize(np.asarray(g, np.float64), 3), self.dtype)
        feq = np.empty(self.Q, self.dtype)
        Fi = np.empty(self.Q, self.dtype)
        self._l.oracle_bgk_terms(self._lref, rho, _ptr(u), _ptr(g), _ptr(feq), _ptr(Fi))
        return feq, Fi
