"""The FP64 kernel against the oracle's PLAIN build, element by element.

The bit-exact parity tests compare the library with the oracle's operation-order twin,
which performs the library's roundings in the library's order (fused multiply-adds in
the moment transforms, the transforms folded over opposite velocities).  This file
compares the binary64 kernel with the PLAIN build instead: the step written as the
paper defines it (eq:dft as sum_i f_i H_m(e_i) over all populations in index order,
the Hermite shifts and the inverse transform as plain sums, no fused multiply-add), so
the two differ by rounding only.  Bound: |kernel - plain| <= 1e-14 max |f| after five
steps (the measured distance between the two oracle builds is about 4e-16 max |f|).

Every lattice, collision and boundary set (periodic, walls, solid nodes), plus the
options of the collisions (third-order force, split rates, orders 5-6), at sizes that
span several workgroups with ragged tails.
"""
import numpy as np
import pytest

from oracle import Oracle
from oracle import lattice as olat
from paper_2212_07494_amd import inputs
from tests.helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]

SHAPES = {"D2Q9": (70, 37, 1), "D3Q19": (67, 13, 9), "D3Q27": (67, 11, 7)}
TAU = {"bgk": (0.63, 0.63, 1.0), "smrt": (0.58, 0.87, 1.0), "rmrt": (0.58, 0.87, 1.0)}
BOUND = 1e-14
STEPS = 5


def lbm():
    from paper_2212_07494_amd import lbm as L
    L.load()
    return L


def _case(lat, seed):
    shape = SHAPES[lat]
    N = int(np.prod(shape))
    D = 2 if lat == "D2Q9" else 3
    w = np.array([float(x) for x in olat.weights(lat)])
    f0 = inputs.random_state(len(w), N, seed, scale=0.05, weights=w)
    rng = np.random.default_rng(seed + 1)
    g = rng.uniform(-1e-3, 1e-3, (3, N))
    g[D:] = 0
    return shape, N, f0, g


def _solid(shape, seed):
    rng = np.random.default_rng(seed)
    s = rng.uniform(size=int(np.prod(shape))) < 0.08
    s[0] = False
    return s


def _compare(L, lat, coll, shape, walls, f0, g, solid=None, **opts):
    tau = TAU[coll]
    scales = np.linspace(1.0, -0.5, STEPS)
    o = Oracle(lat, coll, shape, walls=walls, tau=tau, solid=solid, plain=True, **opts)
    fo = f0.copy()
    for s in scales:
        fo = o.step(fo, g, s)
    with L.Lattice(lat, coll, "f64", shape, walls, tau, g_field=g, solid=solid, **opts) as gpu:
        gpu.set_populations(f0)
        gpu.step(STEPS, g_scale=scales)
        got = gpu.populations()
    fluid = slice(None) if solid is None else ~np.asarray(solid, bool)
    diff = np.max(np.abs(got[:, fluid] - fo[:, fluid]))
    scale = np.max(np.abs(fo[:, fluid]))
    assert diff <= BOUND * scale, (lat, coll, walls, opts, diff / scale)
    return diff / scale


@pytest.mark.parametrize("coll", ["bgk", "smrt", "rmrt"])
@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19", "D3Q27"])
def test_fp64_kernel_matches_plain_definition(lat, coll):
    L = lbm()
    shape, N, f0, g = _case(lat, 31)
    walls_sets = [(0, 0, 0), (0, 1, 0)] + ([(1, 0, 1)] if lat != "D2Q9" else [(1, 1, 0)])
    worst = 0.0
    for walls in walls_sets:
        worst = max(worst, _compare(L, lat, coll, shape, walls, f0, g))
    worst = max(worst, _compare(L, lat, coll, shape, (0, 1, 0), f0, g,
                                solid=_solid(shape, 5)))
    print(f"{lat} {coll}: max |kernel - plain| / max |f| = {worst:.2e}")


@pytest.mark.parametrize("lat,opts", [
    ("D2Q9", dict(force_order=3)), ("D3Q19", dict(force_order=3)),
    ("D3Q27", dict(force_order=3)), ("D2Q9", dict(force_order=4)),
    ("D3Q19", dict(force_order=4, tau_bulk=1.3)), ("D3Q27", dict(force_order=4)),
    ("D2Q9", dict(tau_bulk=1.3)),
    ("D3Q19", dict(tau_bulk=1.3)), ("D3Q19", dict(tau_31=1.6)), ("D3Q27", dict(tau_31=0.7)),
    ("D3Q27", dict(max_order=6)), ("D3Q27", dict(max_order=6, force_order=3)),
])
def test_fp64_kernel_options_match_plain_definition(lat, opts):
    L = lbm()
    shape, N, f0, g = _case(lat, 41)
    walls = (0, 1, 0)
    _compare(L, lat, "smrt", shape, walls, f0, g, **opts)
