"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds no lattice-Boltzmann arithmetic: it only builds initial fields
(density, velocity) and acceleration fields g(x) from fixed seeds and analytic
profiles, as plain NumPy float64 arrays.  Both the HIP library and the CPU oracle
consume its output; neither is imported here.

Array conventions: node index n = (z*ny + y)*nx + x (x fastest); vector fields
are (3, N) component planes; 2-D lattices use nz = 1 and a zero z plane.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    lattice: str
    collision: str
    shape: tuple           # (nx, ny, nz)
    walls: tuple           # per axis, 1 = halfway bounce-back on both faces
    tau: tuple             # (tau2, tau3, tau4) tau-hat per Hermite order
    rho: np.ndarray        # (N,)
    u: np.ndarray          # (3, N)
    g: np.ndarray          # (3, N) acceleration field
    steps: int
    rho0: float = 1.0
    g_profile: tuple | None = None  # (axis, (3, n_axis) table) when g depends on one axis only
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(np.prod(self.shape))


def coords(shape):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def profile_field(shape, axis: int, table: np.ndarray) -> np.ndarray:
    """Expand a (3, n_axis) table along one axis into a (3, N) field."""
    c = coords(shape)[axis]
    return np.ascontiguousarray(table[:, c])


def poiseuille_channel(nx=64, ny=32, tau=0.8, g=1e-6, steps=10_000, collision="bgk") -> Workload:
    """Force-driven channel: periodic x, halfway bounce-back walls in y, uniform g_x,
    rho0 = 1, u0 = 0."""
    shape = (nx, ny, 1)
    N = nx * ny
    gv = np.zeros((3, N))
    gv[0] = g
    return Workload("poiseuille", "D2Q9", collision, shape, (0, 1, 0), (tau, tau, 1.0),
                    np.ones(N), np.zeros((3, N)), gv, steps,
                    g_profile=(1, np.array([[g] * ny, [0.0] * ny, [0.0] * ny])))


def kolmogorov_box(L=1024, tau2=0.6, tau3=1.0, amp=None, mode=1, noise=1e-4, seed=2212,
                   steps=20_000, target_u=0.01, collision="smrt") -> Workload:
    """Periodic L x L box forced by g_x = A sin(2 pi mode y / L).

    amp None -> A chosen so that the continuum steady amplitude A/(nu k^2) is target_u.
    Initial u = continuum steady profile + seeded uniform noise in [-noise, noise] on
    both components at every node; rho = 1.
    """
    nu = (tau2 - 0.5) / 3
    k = 2 * math.pi * mode / L
    A = target_u * nu * k * k if amp is None else amp
    U = A / (nu * k * k)
    shape = (L, L, 1)
    x, y, _ = coords(shape)
    N = L * L
    rng = np.random.default_rng(seed)
    u = np.zeros((3, N))
    u[0] = U * np.sin(k * y) + rng.uniform(-noise, noise, N)
    u[1] = rng.uniform(-noise, noise, N)
    table = np.zeros((3, L))
    table[0] = A * np.sin(k * np.arange(L))
    g = profile_field(shape, 1, table)
    return Workload("kolmogorov", "D2Q9", collision, shape, (0, 0, 0), (tau2, tau3, 1.0),
                    np.ones(N), u, g, steps, g_profile=(1, table),
                    meta=dict(A=A, k=k, U=U, mode=mode))


def taylor_green_3d(n=256, u0=0.02, rho0=1.0, gamp=1e-6, tau2=0.56, tau3=1.0, steps=5000,
                    lattice="D3Q19", collision="smrt") -> Workload:
    """Periodic n^3 box, Taylor-Green initial field plus a steady body force
    g = gamp (sin 2 pi z / n, 0, 0).

    u = u0 [sin kx cos ky cos kz, -cos kx sin ky cos kz, 0], k = 2 pi / n (node indices);
    rho = rho0 + rho0 u0^2 / (16 c_s^2) (cos 2kx + cos 2ky)(cos 2kz + 2), c_s^2 = 1/3.
    """
    shape = (n, n, n)
    x, y, z = coords(shape)
    k = 2 * math.pi / n
    N = n ** 3
    u = np.zeros((3, N))
    u[0] = u0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
    u[1] = -u0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
    rho = rho0 + rho0 * u0 * u0 / (16 / 3) * (np.cos(2 * k * x) + np.cos(2 * k * y)) * (
        np.cos(2 * k * z) + 2)
    table = np.zeros((3, n))
    table[0] = gamp * np.sin(k * np.arange(n))
    g = profile_field(shape, 2, table)
    return Workload("taylor_green_3d", lattice, collision, shape, (0, 0, 0), (tau2, tau3, 1.0),
                    rho, u, g, steps, rho0=rho0, g_profile=(2, table))


def taylor_green_2d(L=64, u0=0.005, Re=50.0, collision="smrt", tau3=1.0) -> Workload:
    """Paper Sec. III.A: periodic L x L box, u = -u0 [cos kx sin ky, -sin kx cos ky],
    rho = 1, acceleration -(u0^2/2) [k sin 2kx, k sin 2ky]; nu = u0 L / Re; run to
    T = ln 2 / (2 nu k^2)."""
    nu = u0 * L / Re
    tau = 3 * nu + 0.5
    k = 2 * math.pi / L
    shape = (L, L, 1)
    x, y, _ = coords(shape)
    N = L * L
    u = np.zeros((3, N))
    u[0] = -u0 * np.cos(k * x) * np.sin(k * y)
    u[1] = u0 * np.sin(k * x) * np.cos(k * y)
    g = np.zeros((3, N))
    g[0] = -(u0 ** 2) / 2 * k * np.sin(2 * k * x)
    g[1] = -(u0 ** 2) / 2 * k * np.sin(2 * k * y)
    T = math.log(2) / (2 * nu * k * k)
    return Workload("taylor_green_2d", "D2Q9", collision, shape, (0, 0, 0),
                    (tau, tau if collision == "bgk" else tau3, 1.0), np.ones(N), u, g,
                    int(round(T)), meta=dict(nu=nu, u0=u0))


def fourier_modes(seed=2022, nmodes=4, kmax=4, amp_range=(1e-7, 1e-5)):
    """Random solenoidal Fourier forcing modes: integer wavevector k with
    max |k_a| in 1..kmax (not all zero), unit polarisation perpendicular to k, phase in
    [0, 2 pi), amplitude log-uniform in amp_range.  Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    modes = []
    while len(modes) < nmodes:
        kv = rng.integers(-kmax, kmax + 1, size=3)
        if not kv.any():
            continue
        kh = kv / np.linalg.norm(kv)
        r = rng.normal(size=3)
        p = r - np.dot(r, kh) * kh
        p /= np.linalg.norm(p)
        amp = math.exp(rng.uniform(math.log(amp_range[0]), math.log(amp_range[1])))
        modes.append(dict(k=kv.astype(np.int64), p=p, phase=rng.uniform(0, 2 * math.pi), amp=amp))
    return modes


def fourier_force(shape, modes) -> np.ndarray:
    """g(x) = sum_j amp_j p_j sin(2 pi k_j . x / n + phase_j) on an n^3 periodic box."""
    x, y, z = coords(shape)
    n = np.array(shape, dtype=np.float64)
    g = np.zeros((3, x.size))
    for m in modes:
        arg = 2 * math.pi * (m["k"][0] * x / n[0] + m["k"][1] * y / n[1] + m["k"][2] * z / n[2])
        s = np.sin(arg + m["phase"])
        for a in range(3):
            g[a] += m["amp"] * m["p"][a] * s
    return g


def random_state(Q: int, N: int, seed: int, scale: float = 0.05, weights=None) -> np.ndarray:
    """Seeded populations near rest: w_i (1 + scale * U(-1, 1)), as (Q, N) float64.
    weights: the lattice weights (length Q); uniform 1/Q when None."""
    rng = np.random.default_rng(seed)
    w = np.full(Q, 1.0 / Q) if weights is None else np.asarray(weights, np.float64)
    return w[:, None] * (1.0 + scale * rng.uniform(-1.0, 1.0, size=(Q, N)))


def random_fields(shape, seed: int, u_amp=0.05, rho_amp=0.02, g_amp=1e-4, dim=3):
    """Seeded smooth-ish random (rho, u, g) fields for parity tests."""
    N = int(np.prod(shape))
    rng = np.random.default_rng(seed)
    rho = 1.0 + rho_amp * rng.uniform(-1, 1, N)
    u = u_amp * rng.uniform(-1, 1, (3, N))
    g = g_amp * rng.uniform(-1, 1, (3, N))
    if dim == 2:
        u[2] = 0
        g[2] = 0
    return rho, u, g


def batch_domains(n=512, seed=7494, h_range=(16, 128), l_range=(64, 256),
                  tau_range=(0.55, 1.5), g_range=(1e-7, 1e-5), umax=0.1):
    """Uneven D2Q9 domains: half channels (walls in y, uniform g_x), half periodic
    Kolmogorov boxes (g_x = amp sin(2 pi y / H)).  Domains whose continuum peak
    velocity exceeds umax (g H^2 / (8 nu) for a channel, amp H^2/(4 pi^2 nu) for a
    box) are redrawn from the same stream.  Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        kind = int(rng.integers(0, 2))
        H = int(rng.integers(h_range[0], h_range[1] + 1))
        Lx = int(rng.integers(l_range[0], l_range[1] + 1))
        tau2 = float(rng.uniform(*tau_range))
        amp = math.exp(rng.uniform(math.log(g_range[0]), math.log(g_range[1])))
        nu = (tau2 - 0.5) / 3
        peak = amp * H * H / (8 * nu) if kind == 0 else amp * H * H / (4 * math.pi ** 2 * nu)
        if peak > umax:
            continue
        out.append(dict(kind=kind, nx=Lx, ny=H, tau2=tau2, g=amp, peak=peak))
    return out


def batch_domain_dicts(specs):
    """lbm.Batch domain dicts of batch_domains' specs: channels with walls in y and a
    uniform g_x, periodic boxes with the profile g_x = amp sin(2 pi y / H)."""
    doms = []
    for s in specs:
        nx, ny = s["nx"], s["ny"]
        tau = (s["tau2"], 1.0, 1.0)
        if s["kind"] == 0:
            doms.append(dict(shape=(nx, ny, 1), walls=(0, 1, 0), tau=tau, g=(s["g"], 0, 0)))
        else:
            table = np.zeros((3, ny))
            table[0] = s["g"] * np.sin(2 * math.pi * np.arange(ny) / ny)
            doms.append(dict(shape=(nx, ny, 1), walls=(0, 0, 0), tau=tau, g_profile=(1, table)))
    return doms


def mlp_init_params(widths, seed: int) -> np.ndarray:
    """Seeded initial network parameters (flat, W_0, b_0, W_1, b_1, ...; W row-major
    out x in): weights uniform in +-sqrt(6 / (in + out)), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(len(widths) - 1):
        k, n = widths[l], widths[l + 1]
        bound = math.sqrt(6.0 / (k + n))
        parts.append(rng.uniform(-bound, bound, n * k))
        parts.append(np.zeros(n))
    return np.concatenate(parts)


def warmstart_problem(seed: int, box: int = 128, tau_range=(0.55, 1.2), kmax=4,
                      amp_range=(1e-7, 1e-5), umax=0.05, remax=0.5, nmodes=4,
                      family="narrow"):
    """One seeded warm-start problem on a periodic box^3: tau2 uniform in tau_range and
    nmodes Fourier forcing modes (fourier_modes), redrawn until the draw is accepted.

    family "narrow": the summed Stokes amplitude U = sum_j amp_j / (nu K_j^2)
    (K_j = 2 pi |k_j| / box) is at most umax and the Reynolds number U / (nu K_min) at
    most remax.  family "wide": each mode on its own has a Stokes amplitude
    U_j = amp_j / (nu K_j^2) of at most 0.1 and a Reynolds number
    Re_j = amp_j / (nu^2 K_j^3) of at most 1 (the bounds per mode of the configuration's
    sampling; some such problems have no steady state).  Returns dict(tau2, modes, U,
    Re) with U the summed Stokes amplitude and Re the largest Re_j."""
    rng = np.random.default_rng(seed)
    while True:
        tau2 = float(rng.uniform(*tau_range))
        modes = fourier_modes(seed=int(rng.integers(0, 2 ** 31)), nmodes=nmodes, kmax=kmax,
                              amp_range=amp_range)
        nu = (tau2 - 0.5) / 3
        Ks = [2 * math.pi * float(np.linalg.norm(m["k"])) / box for m in modes]
        Uj = [m["amp"] / (nu * K * K) for m, K in zip(modes, Ks)]
        Rej = [m["amp"] / (nu * nu * K ** 3) for m, K in zip(modes, Ks)]
        U = sum(Uj)
        if family == "wide":
            ok = max(Uj) <= 0.1 and max(Rej) <= 1.0
        else:
            ok = U <= umax and U / (nu * min(Ks)) <= remax
        if ok:
            return dict(tau2=tau2, modes=modes, U=U, Re=max(Rej))
