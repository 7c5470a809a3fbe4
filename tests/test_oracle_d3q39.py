"""Pins of the oracle on the high-order lattice D3Q39 beyond the ones it shares with the
degree-5 lattices (those run on all four lattices in the other oracle test files).

* The paper's reconstruction (the Hermite sum to order 4 after eq:bbd1) rebuilds the
  post-collision state from its moments: anything in the populations that no carried
  moment sees (the null space of the projection, ten dimensions on the 39 velocities) is
  dropped by the SMRT and RMRT collisions and relaxed at rate 1/tau by BGK.
* Kolmogorov flow (periodic, g_x = G sin(2 pi y / n)): the steady amplitude converges at
  second order in 1/n to the incompressible value G / (nu k^2) with the lattice's
  viscosity nu = c_s^2 (tau-hat - 1/2), c_s^2 = 2/3.
"""
import math

import numpy as np
import pytest

from oracle import Oracle
from oracle import lattice as lat

L = "D3Q39"


def _null_space():
    M = np.asarray(lat.tables(L, np.float64)["H"])
    _, sv, vt = np.linalg.svd(M)
    rank = int(np.sum(sv > 1e-10))
    return vt[rank:]


@pytest.mark.parametrize("coll", ["smrt", "rmrt", "bgk"])
@pytest.mark.parametrize("seed", range(3))
def test_moments_blind_part_is_dropped(coll, seed):
    rng = np.random.default_rng(seed)
    o = Oracle(L, coll, (1, 1, 1), tau=(0.7, 0.9 if coll != "bgk" else 0.7, 1.0),
               force_order=3 if coll == "smrt" and seed == 2 else 1)
    u = rng.uniform(-0.08, 0.08, 3)
    g = rng.uniform(-1e-3, 1e-3, 3)
    f = o.init_node(1.0 + 0.05 * rng.uniform(-1, 1), u, g)
    f = f * (1 + 0.02 * rng.uniform(-1, 1, o.Q))
    Z = _null_space()
    assert Z.shape == (10, 39)
    ghost = 1e-3 * (rng.standard_normal(10) @ Z)
    a = o.collide_node(f, g)
    b = o.collide_node(f + ghost, g)
    if coll == "bgk":
        # BGK acts population by population: the blind part relaxes as (1 - omega) ghost
        # (its mass and momentum are zero, so the equilibrium does not see it)
        assert np.max(np.abs((b - a) - (1 - 1 / 0.7) * ghost)) < 1e-15
    else:
        assert np.max(np.abs(b - a)) < 1e-15
        # and the output lies in the range of the reconstruction (columns w_i H_m(e_i)),
        # which is orthogonal to the blind part in the 1/w-weighted product
        w = np.asarray(lat.tables(L, np.float64)["w"])
        assert np.max(np.abs(Z @ (a / w))) < 1e-13


def _kolmogorov_amplitude(n, coll, tau):
    o = Oracle(L, coll, (4, n, 3), tau=(tau, 1.0 if coll != "bgk" else tau, 1.0))
    y = (np.arange(o.N) // 4) % n
    G = 1e-6
    g = np.zeros((3, o.N))
    g[0] = G * np.sin(2 * math.pi * y / n)
    nu = float(lat.cs2(L)) * (tau - 0.5)
    k = 2 * math.pi / n
    steps = int(18 / (nu * k * k))
    f = o.run(o.init(1.0, None, g), g, steps)
    _, u = o.moments(f, g)
    s = np.sin(2 * math.pi * y / n)
    amp = float(u[0] @ s / (s @ s))
    return amp / (G / (nu * k * k))


@pytest.mark.parametrize("coll", ["smrt", "bgk"])
def test_kolmogorov_amplitude_converges_to_continuum(coll):
    r16 = _kolmogorov_amplitude(16, coll, 0.8)
    r32 = _kolmogorov_amplitude(32, coll, 0.8)
    e16, e32 = abs(r16 - 1), abs(r32 - 1)
    assert e32 < 1e-2 and e32 < 0.3 * e16, (r16, r32)  # measured 5.1e-3 (SMRT), 8.2e-3 (BGK)
