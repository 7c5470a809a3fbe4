"""Solid nodes on the GPU against the oracle: random masks (about 15% solid) with and
without wall faces, random state and force field, three steps with force scales: every
fluid node's stored populations equal the oracle's bit for bit; lbm_moments is zero at
solid nodes and equals the oracle at fluid nodes; the monitors' mass is the fluid mass.
(Populations stored at solid nodes are unspecified and not compared.)"""
import numpy as np
import pytest

from oracle import lattice as olat
from paper_2212_07494_amd import inputs
from tests.helpers import exact_mismatch, gpu_available, oracle_for, to_storage

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]

SHAPES = {"D2Q9": (70, 37, 1), "D3Q19": (67, 13, 9), "D3Q27": (67, 11, 7)}
WALLS = {"D2Q9": (0, 1, 0), "D3Q19": (1, 0, 1), "D3Q27": (0, 1, 1)}
TAU = {"bgk": (0.63, 0.63, 1.0), "smrt": (0.58, 0.87, 1.0), "rmrt": (0.58, 0.87, 1.0)}


@pytest.mark.parametrize("storage", ["f64", "f32s", "f16s"])
@pytest.mark.parametrize("coll", ["bgk", "smrt", "rmrt"])
@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19", "D3Q27"])
def test_solid_parity(lat, coll, storage):
    from paper_2212_07494_amd import lbm as L
    L.load()
    shape = SHAPES[lat]
    N = int(np.prod(shape))
    D = 2 if lat == "D2Q9" else 3
    rng = np.random.default_rng(17)
    solid = (rng.uniform(0, 1, N) < 0.15).astype(np.uint8)
    fluid = solid == 0
    g = rng.uniform(-1e-3, 1e-3, (3, N))
    g[D:] = 0
    w = np.array([float(x) for x in olat.weights(lat)])
    for walls in ((0, 0, 0), WALLS[lat]):
        f0 = inputs.random_state(len(w), N, 19, scale=0.05, weights=w)
        if storage != "f64":
            f0 = f0 - w[:, None]
        f0 = to_storage(f0, storage)
        o = oracle_for(lat, coll, storage, shape, walls, TAU[coll])
        o_solid = type(o)(lat, coll, shape, walls=walls, tau=TAU[coll],
                          shift=o._p.shift, real=o.real, store16=bool(o._p.store16),
                          solid=solid)
        scales = [1.0, 0.5, -2.0]
        fo = f0.astype(o_solid.dtype)
        for s in scales:
            fo = o_solid.step(fo, g, s)
        with L.Lattice(lat, coll, storage, shape, walls, TAU[coll], g_field=g,
                       solid=solid) as gpu:
            gpu.set_populations(f0)
            gpu.step(3, g_scale=scales)
            got = gpu.populations()
            assert exact_mismatch(got[:, fluid], fo[:, fluid].astype(np.float64)) == 0, walls
            r, u = gpu.moments(g_scale=-2.0)
            ro, uo = o_solid.moments(fo, g, gscale=-2.0)
            assert np.all(r[~fluid] == 0) and np.all(u[:, ~fluid] == 0)
            assert exact_mismatch(r[fluid], ro[fluid].astype(np.float64)) == 0
            assert exact_mismatch(u[:, fluid], uo[:D, fluid].astype(np.float64)) == 0
            m = gpu.monitors()
            want = float(np.sum(ro[fluid].astype(np.float64)))
            assert abs(m.mass - want) <= 1e-12 * want
