"""Shared test helpers: building matching oracle / library instances and comparing them."""
from __future__ import annotations

import numpy as np

from oracle import Oracle
from oracle import lattice as olat

# storage mode -> (oracle real, shift?, store16?)
EMUL = {"f64": ("f64", False, False), "f32": ("f32", False, False),
        "f32s": ("f32", True, False), "f16s": ("f32", True, True)}


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def oracle_for(lattice, collision, storage, shape, walls, tau, rho0=1.0, force_order=1,
               tau_bulk=0.0, tau_31=0.0, max_order=4):
    real, shifted, s16 = EMUL[storage]
    return Oracle(lattice, collision, shape, walls=walls, tau=tau,
                  shift=rho0 if shifted else 0.0, real=real, store16=s16,
                  force_order=force_order, tau_bulk=tau_bulk, tau_31=tau_31,
                  max_order=max_order)


def to_storage(x: np.ndarray, storage: str) -> np.ndarray:
    """Values as the library stores them, returned in float64."""
    if storage == "f64":
        return np.asarray(x, np.float64)
    if storage == "f16s":
        return np.asarray(x, np.float32).astype(np.float16).astype(np.float64)
    return np.asarray(x, np.float32).astype(np.float64)


def stream_dest(lattice, shape, walls, nodes):
    """For each node x and population i, the (population, node) slot the post-collision
    value f*_i(x) occupies one step later as a pre-collision value: (i, x + e_i) with
    periodic wrap, or (opp(i), x) across a wall."""
    E = np.array(olat.velocities(lattice))
    opp = np.array(olat.opposite(lattice))
    nx, ny, nz = shape
    nodes = np.asarray(nodes, np.int64)
    x = nodes % nx
    y = (nodes // nx) % ny
    z = nodes // (nx * ny)
    Q = len(E)
    pop = np.empty((Q, nodes.size), np.int64)
    dst = np.empty((Q, nodes.size), np.int64)
    dims = (nx, ny, nz)
    for i in range(Q):
        c = [x + E[i, 0], y + E[i, 1], z + E[i, 2]]
        wall = np.zeros(nodes.size, bool)
        for a in range(3):
            out = (c[a] < 0) | (c[a] >= dims[a])
            if walls[a]:
                wall |= out
            c[a] = np.mod(c[a], dims[a])
        d = (c[2] * ny + c[1]) * nx + c[0]
        pop[i] = np.where(wall, opp[i], i)
        dst[i] = np.where(wall, nodes, d)
    return pop, dst


def exact_mismatch(a, b) -> int:
    """Number of entries whose values differ (NaN never equal; -0 == +0)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return int(np.count_nonzero(~(a == b)))
