"""Steps replayed from captured HIP graphs (small lattices) equal single launches.

lbm_step runs n >= 128 steps of a lattice of at most 2^21 nodes as replays of a captured
64-step graph (force factors s(t) read from device memory) plus single launches for the
remainder.  Calls of fewer than 128 steps launch step by step.  Each graph-replayed run is
compared bit for bit with the same steps taken in pieces of fewer than 128, after every
call, with eager work and synchronisation between the calls; per-step force factors and
none; a change of the launch configuration between calls.
"""
import math

import numpy as np
import pytest

from oracle import lattice as olat
from paper_2212_07494_amd import inputs
from tests.helpers import exact_mismatch, gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]


def lbm():
    from paper_2212_07494_amd import lbm as L
    L.load()
    return L


def eager(lat, n, scales=None, piece=100):
    for s in range(0, n, piece):
        k = min(piece, n - s)
        lat.step(k, None if scales is None else scales[s:s + k])


@pytest.mark.parametrize("storage", ["f64", "f32s"])
def test_womersley_graph_replays_equal_single_launches(storage):
    """The Womersley channel (50 x 200, D2Q9 SMRT, uniform force times cos(2 pi t / 1200)),
    three calls of 1000, 300 and 130 steps."""
    L = lbm()
    T = 1200
    s = np.cos(2 * math.pi * np.arange(2000) / T)
    kw = dict(g=(-1e-4, 0.0, 0.0))
    with L.Lattice("D2Q9", "smrt", storage, (50, 200, 1), (0, 1, 0), (0.8, 1.0, 1.0), **kw) as a, \
            L.Lattice("D2Q9", "smrt", storage, (50, 200, 1), (0, 1, 0), (0.8, 1.0, 1.0), **kw) as b:
        t = 0
        for n in (1000, 300, 130):
            a.step(n, s[t:t + n])
            eager(b, n, s[t:t + n])
            t += n
            assert a.time == b.time == t
            assert exact_mismatch(a.populations(), b.populations()) == 0, (n, t)
            a.moments()  # eager work between the calls


def test_graph_without_factors_field_force_and_retuning():
    """D3Q19 SMRT FP32-shifted 40 x 20 x 12 with a y-walled channel and a full force field,
    s(t) = 1: 256 steps (four replays), a different launch configuration, 200 more, then a
    launch held to 4 waves per SIMD (its workgroups reserve LDS inside the graph), 200
    more."""
    L = lbm()
    shape = (40, 20, 12)
    rng = np.random.default_rng(3)
    g = 1e-4 * rng.uniform(-1, 1, (3, int(np.prod(shape))))
    rho, u, _ = inputs.random_fields(shape, seed=4, u_amp=0.02)
    args = ("D3Q19", "smrt", "f32s", shape, (0, 1, 0), (0.6, 0.9, 1.0))
    with L.Lattice(*args, rho=rho, u=u, g_field=g) as a, \
            L.Lattice(*args, rho=rho, u=u, g_field=g) as b:
        a.step(256)
        eager(b, 256, piece=64)
        assert exact_mismatch(a.populations(), b.populations()) == 0
        a.tune(64, 2, 4)
        a.step(200)
        eager(b, 200, piece=64)
        assert exact_mismatch(a.populations(), b.populations()) == 0
        a.tune(128, 2, 26)
        a.step(200)
        eager(b, 200, piece=64)
        assert exact_mismatch(a.populations(), b.populations()) == 0
        w = np.array([float(x) for x in olat.weights("D3Q19")])
        assert np.isfinite(a.populations()).all() and w.size == 19


def test_graph_path_with_factors_does_not_block():
    """With per-step force factors the graph path stages them in pinned memory and uploads
    them asynchronously: the call returns while its 20,000 steps (tens of ms) are still
    running, and a second call right after it (reusing the staging buffer) gives the same
    result as one call of both halves."""
    import torch
    L = lbm()
    s = np.cos(2 * math.pi * np.arange(40_000) / 1200)
    stream = torch.cuda.Stream()
    args = ("D2Q9", "smrt", "f64", (50, 200, 1), (0, 1, 0), (0.8, 1.0, 1.0))
    with L.Lattice(*args, g=(-1e-4, 0.0, 0.0), stream=stream) as a, \
            L.Lattice(*args, g=(-1e-4, 0.0, 0.0), stream=stream) as b:
        a.step(128, s[:128])  # capture the graphs and stage the factors once
        b.step(128, s[:128])
        stream.synchronize()
        a.step(20_000, s[128:20_128])
        pending = not stream.query()
        a.step(19_872, s[20_128:])
        b.step(39_872, s[128:])
        assert exact_mismatch(a.populations(), b.populations()) == 0
        assert pending
