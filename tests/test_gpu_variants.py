"""Every launch configuration of the step (block shapes x memory variants x addressing
paths x block placements, and wave caps on a spread of those) gives bit-identical
results, equal to the oracle's: ragged rows, odd row lengths, block counts that are not
multiples of the XCD count and x/y/z walls are covered."""
import numpy as np
import pytest

from oracle import lattice as olat
from paper_2212_07494_amd import inputs
from tests.helpers import exact_mismatch, gpu_available, oracle_for, to_storage

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]

CASES = {
    "D2Q9": [((134, 9, 1), (0, 0, 0)), ((134, 6, 1), (1, 1, 0)), ((67, 5, 1), (1, 0, 0))],
    "D3Q19": [((70, 5, 4), (0, 0, 0)), ((70, 5, 4), (1, 1, 1)), ((131, 3, 3), (1, 0, 1))],
    "D3Q27": [((70, 4, 3), (0, 0, 0)), ((70, 4, 3), (1, 0, 1)), ((65, 3, 3), (0, 1, 0))],
}
TAU = {"bgk": (0.61, 0.61, 1.0), "smrt": (0.57, 0.91, 1.0), "rmrt": (0.57, 0.91, 1.0)}
# the 12 base variants, then each wave cap (variant // 12 = 1..4) on a spread of bases
VARIANTS = list(range(12)) + [b + 12 * k for k in range(1, 5) for b in (0, 5, 8)]
N_VARIANTS = 60


@pytest.mark.parametrize("storage", ["f64", "f32s", "f16s"])
@pytest.mark.parametrize("coll", ["bgk", "smrt", "rmrt"])
@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19", "D3Q27"])
def test_all_launch_configurations(lat, coll, storage):
    from paper_2212_07494_amd import lbm as L
    L.load()
    w = np.array([float(x) for x in olat.weights(lat)])
    for shape, walls in CASES[lat]:
        N = int(np.prod(shape))
        f0 = inputs.random_state(len(w), N, seed=3, weights=w)
        if storage != "f64":
            f0 = f0 - w[:, None]
        f0 = to_storage(f0, storage)
        rng = np.random.default_rng(4)
        D = 2 if lat == "D2Q9" else 3
        g = rng.uniform(-1e-3, 1e-3, (3, N))
        g[D:] = 0
        o = oracle_for(lat, coll, storage, shape, walls, TAU[coll])
        want = f0.astype(o.dtype)
        for _ in range(3):
            want = o.step(want, g, 1.0)
        want = want.astype(np.float64)
        with L.Lattice(lat, coll, storage, shape, walls, TAU[coll], g_field=g) as gpu:
            for bx in (64, 128, 256):
                for by in (1, 2, 4):
                    if bx * by > 256:
                        continue
                    for v in VARIANTS:
                        L.lbm_set_tuning(gpu.ctx, bx, by, v)
                        gpu.set_populations(f0)
                        gpu.step(3)
                        bad = exact_mismatch(gpu.populations(), want)
                        assert bad == 0, (shape, walls, bx, by, v, bad)
            with pytest.raises(L.LBMError):
                L.lbm_set_tuning(gpu.ctx, 64, 1, N_VARIANTS)
            with pytest.raises(L.LBMError):
                L.lbm_set_tuning(gpu.ctx, 96, 1, 0)
