"""lbm_get_populations_noalloc, the entry point for callers that cannot allocate device
memory: through the C ABI it returns exactly what lbm_get_populations returns, on two
calls in a row (the second with fewer nodes), and refuses requests beyond its fixed
staging array."""
import ctypes as C

import numpy as np
import pytest

from paper_2212_07494_amd import inputs
from tests.helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]


def _call(lib, ctx, nodes, Q):
    idx = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.full((Q, idx.size), np.nan)
    rc = lib.lbm_get_populations_noalloc(ctx, idx.size, idx.ctypes.data_as(C.c_void_p),
                                         out.ctypes.data_as(C.c_void_p))
    return rc, out


@pytest.mark.parametrize("lat,storage", [("D2Q9", "f64"), ("D3Q19", "f32s"), ("D3Q27", "f16s"),
                                         ("D3Q39", "f64")])
def test_noalloc_gather_equals_allocating_gather(lat, storage):
    from paper_2212_07494_amd import lbm as L
    lib = L.load()
    shape = (96, 40, 1) if lat == "D2Q9" else (48, 20, 12)
    N = int(np.prod(shape))
    D = 2 if lat == "D2Q9" else 3
    rho, u, g = inputs.random_fields(shape, seed=2, dim=D)
    rng = np.random.default_rng(4)
    walls = (0, 0, 0) if lat == "D3Q39" else (0, 1, 0)  # D3Q39 runs periodic boxes
    with L.Lattice(lat, "smrt", storage, shape, walls, (0.6, 0.9, 1.0), rho=rho, u=u[:D],
                   g_field=g) as gpu:
        gpu.step(3)
        Q = gpu.Q
        first = rng.integers(0, N, 3000)
        second = rng.integers(0, N, 700)  # a smaller second call
        for nodes in (first, second):
            rc, got = _call(lib, gpu.ctx, nodes, Q)
            assert rc == L.LBM_OK, L.load().lbm_last_error()
            want = gpu.populations(nodes)  # the allocating entry point
            assert np.array_equal(got, want)
        gpu.step(2)
        rc, got = _call(lib, gpu.ctx, second, Q)
        assert rc == L.LBM_OK and np.array_equal(got, gpu.populations(second))
        # beyond the staging array: refused, nothing written
        limit = (4 << 20) // ((Q + 1) * 8)
        big = np.zeros(limit + 1, np.int64)
        rc, got = _call(lib, gpu.ctx, big, Q)
        assert rc == L.LBM_EINVAL and np.isnan(got).all()
        assert b"no-alloc scratch" in lib.lbm_last_error()
        rc, got = _call(lib, gpu.ctx, np.zeros(limit, np.int64), Q)
        assert rc == L.LBM_OK


def test_noalloc_whole_lattice_when_it_fits():
    from paper_2212_07494_amd import lbm as L
    lib = L.load()
    shape = (64, 30, 1)
    with L.Lattice("D2Q9", "bgk", "f64", shape, (0, 0, 0), (0.7, 0.7, 1.0)) as gpu:
        gpu.step(4)
        out = np.empty((9, 64 * 30))
        rc = lib.lbm_get_populations_noalloc(gpu.ctx, 64 * 30, None,
                                             out.ctypes.data_as(C.c_void_p))
        assert rc == L.LBM_OK
        assert np.array_equal(out, gpu.populations())
