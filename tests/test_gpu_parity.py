"""Parity of the HIP library with the CPU oracle, element by element.

FP64 storage: bit-exact against the FP64 oracle.  FP32 / FP32-shifted / FP16-shifted
storage: bit-exact against the oracle's float build, which performs the same binary32
arithmetic in the same order and rounds stores the same way.  Sizes span several
thread blocks with ragged tails in x and y; walls, force profiles, full force fields
and time-dependent force scales are covered.
"""
import numpy as np
import pytest

from oracle import lattice as olat
from paper_2212_07494_amd import inputs
from tests.helpers import exact_mismatch, gpu_available, oracle_for, stream_dest, to_storage

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]

LATS = ["D2Q9", "D3Q19", "D3Q27"]
STORES = ["f64", "f32", "f32s", "f16s"]
SHAPES = {"D2Q9": (70, 37, 1), "D3Q19": (67, 13, 9), "D3Q27": (67, 11, 7)}
WALLS = {"D2Q9": [(0, 0, 0), (0, 1, 0), (1, 1, 0)], "D3Q19": [(0, 0, 0), (1, 0, 1)],
         "D3Q27": [(0, 0, 0), (1, 0, 1)]}
TAU = {"bgk": (0.63, 0.63, 1.0), "smrt": (0.58, 0.87, 1.0), "rmrt": (0.58, 0.87, 1.0)}


def lbm():
    from paper_2212_07494_amd import lbm as L
    L.load()
    return L


def _state(lat, storage, N, seed, rho0=1.0):
    w = np.array([float(x) for x in olat.weights(lat)])
    f = inputs.random_state(len(w), N, seed, scale=0.05, weights=w)
    if storage in ("f32s", "f16s"):
        f = f - w[:, None] * rho0
    return to_storage(f, storage)


def _force(lat, shape, kind, seed):
    N = int(np.prod(shape))
    D = 2 if lat == "D2Q9" else 3
    rng = np.random.default_rng(seed)
    if kind == "field":
        g = rng.uniform(-1e-3, 1e-3, (3, N))
        g[D:] = 0
        return dict(g_field=g), g
    axis = 1
    table = rng.uniform(-1e-3, 1e-3, (3, shape[axis]))
    table[D:] = 0
    return dict(g_profile=(axis, table)), inputs.profile_field(shape, axis, table)


@pytest.mark.parametrize("storage", STORES)
@pytest.mark.parametrize("coll", ["bgk", "smrt", "rmrt"])
@pytest.mark.parametrize("lat", LATS)
def test_step_parity_random_state(lat, coll, storage):
    """Random pre-collision state, random force field, three steps with force scales
    (1, 0.5, -2): every stored value equals the oracle's."""
    L = lbm()
    shape = SHAPES[lat]
    N = int(np.prod(shape))
    for walls in WALLS[lat]:
        for kind in ("field", "profile"):
            kw, g = _force(lat, shape, kind, seed=7)
            f0 = _state(lat, storage, N, seed=11)
            o = oracle_for(lat, coll, storage, shape, walls, TAU[coll])
            with L.Lattice(lat, coll, storage, shape, walls, TAU[coll], **kw) as gpu:
                gpu.set_populations(f0)
                assert exact_mismatch(gpu.populations(), f0) == 0
                scales = [1.0, 0.5, -2.0]
                gpu.step(3, g_scale=scales)
                fo = f0.astype(o.dtype)
                for s in scales:
                    fo = o.step(fo, g, s)
                got = gpu.populations()
                bad = exact_mismatch(got, fo.astype(np.float64))
                assert bad == 0, (walls, kind, bad, np.max(np.abs(got - fo)))


@pytest.mark.parametrize("storage", STORES)
@pytest.mark.parametrize("lat", LATS)
@pytest.mark.parametrize("order,tau_bulk", [(3, 0.0), (3, 1.4), (4, 0.0), (4, 1.4)])
def test_force_content_parity(lat, storage, order, tau_bulk):
    """SMRT with the non-equilibrium force content to third (force_order 3) or fourth
    order (force_order 4), alone and with a separate bulk rate: random state and force
    field, three steps with force scales (1, 0.5, -2), bit-identical to the oracle; and
    the content does change the state against the order below."""
    L = lbm()
    shape = SHAPES[lat]
    N = int(np.prod(shape))
    walls = WALLS[lat][-1]
    kw, g = _force(lat, shape, "field", seed=8)
    f0 = _state(lat, storage, N, seed=12)
    o = oracle_for(lat, "smrt", storage, shape, walls, TAU["smrt"], force_order=order,
                   tau_bulk=tau_bulk)
    scales = [1.0, 0.5, -2.0]
    fo = f0.astype(o.dtype)
    for s in scales:
        fo = o.step(fo, g, s)
    below = 1 if order == 3 else 3
    got = {}
    for fo_ in (below, order):
        with L.Lattice(lat, "smrt", storage, shape, walls, TAU["smrt"], force_order=fo_,
                       tau_bulk=tau_bulk, **kw) as gpu:
            gpu.set_populations(f0)
            gpu.step(3, g_scale=scales)
            got[fo_] = gpu.populations()
    assert exact_mismatch(got[order], fo.astype(np.float64)) == 0
    if storage != "f16s":  # binary16 may round the small change away
        assert exact_mismatch(got[order], got[below]) > 0


@pytest.mark.parametrize("storage", STORES)
@pytest.mark.parametrize("lat", LATS)
def test_bulk_rate_parity(lat, storage):
    """SMRT with its own rate for the trace of the second-order moment (tau_bulk): random
    state, force field and walls, three steps, bit-identical to the oracle; and the state
    differs from the one-rate step."""
    L = lbm()
    shape = SHAPES[lat]
    N = int(np.prod(shape))
    walls = WALLS[lat][-1]
    kw, g = _force(lat, shape, "field", seed=9)
    f0 = _state(lat, storage, N, seed=13)
    o = oracle_for(lat, "smrt", storage, shape, walls, TAU["smrt"], tau_bulk=1.7)
    scales = [1.0, 0.5, -2.0]
    fo = f0.astype(o.dtype)
    for s in scales:
        fo = o.step(fo, g, s)
    got = {}
    for tb in (0.0, 1.7):
        with L.Lattice(lat, "smrt", storage, shape, walls, TAU["smrt"], tau_bulk=tb,
                       **kw) as gpu:
            gpu.set_populations(f0)
            gpu.step(3, g_scale=scales)
            got[tb] = gpu.populations()
    assert exact_mismatch(got[1.7], fo.astype(np.float64)) == 0
    assert exact_mismatch(got[1.7], got[0.0]) > 0


@pytest.mark.parametrize("storage", STORES)
@pytest.mark.parametrize("lat", ["D3Q19", "D3Q27"])
def test_split_rates_parity(lat, storage):
    """SMRT with separate rates for the traces at orders 2 and 3 (tau_bulk, tau_31) and
    for the third-order trace alone: bit-identical to the oracle; each changes the state."""
    L = lbm()
    shape = SHAPES[lat]
    N = int(np.prod(shape))
    walls = WALLS[lat][-1]
    kw, g = _force(lat, shape, "field", seed=10)
    f0 = _state(lat, storage, N, seed=14)
    scales = [1.0, 0.5, -2.0]
    got = {}
    for tb, t31 in ((0.0, 0.0), (0.0, 0.7), (1.7, 0.7)):
        o = oracle_for(lat, "smrt", storage, shape, walls, TAU["smrt"], tau_bulk=tb, tau_31=t31)
        fo = f0.astype(o.dtype)
        for s in scales:
            fo = o.step(fo, g, s)
        with L.Lattice(lat, "smrt", storage, shape, walls, TAU["smrt"], tau_bulk=tb,
                       tau_31=t31, **kw) as gpu:
            gpu.set_populations(f0)
            gpu.step(3, g_scale=scales)
            got[(tb, t31)] = gpu.populations()
        assert exact_mismatch(got[(tb, t31)], fo.astype(np.float64)) == 0, (tb, t31)
    assert exact_mismatch(got[(0.0, 0.7)], got[(0.0, 0.0)]) > 0
    assert exact_mismatch(got[(1.7, 0.7)], got[(0.0, 0.7)]) > 0


@pytest.mark.parametrize("storage", STORES)
@pytest.mark.parametrize("force_order", [1, 3])
def test_high_orders_parity(storage, force_order):
    """D3Q27 SMRT carrying orders 5 and 6 (max_order 6), without and with the third-order
    force content: random state, force field and walls, three steps, bit-identical to
    the oracle; and it changes the state."""
    L = lbm()
    lat = "D3Q27"
    shape = SHAPES[lat]
    N = int(np.prod(shape))
    walls = WALLS[lat][-1]
    kw, g = _force(lat, shape, "field", seed=11)
    f0 = _state(lat, storage, N, seed=15)
    o = oracle_for(lat, "smrt", storage, shape, walls, TAU["smrt"], max_order=6,
                   force_order=force_order)
    scales = [1.0, 0.5, -2.0]
    fo = f0.astype(o.dtype)
    for s in scales:
        fo = o.step(fo, g, s)
    got = {}
    for mo in (4, 6):
        with L.Lattice(lat, "smrt", storage, shape, walls, TAU["smrt"], max_order=mo,
                       force_order=force_order, **kw) as gpu:
            gpu.set_populations(f0)
            gpu.step(3, g_scale=scales)
            got[mo] = gpu.populations()
    assert exact_mismatch(got[6], fo.astype(np.float64)) == 0
    if storage != "f16s":  # binary16 may round the small change away
        assert exact_mismatch(got[6], got[4]) > 0


@pytest.mark.parametrize("storage", STORES)
@pytest.mark.parametrize("coll", ["bgk", "smrt", "rmrt"])
@pytest.mark.parametrize("lat", LATS)
def test_init_and_moments_parity(lat, coll, storage):
    """lbm_init from (rho, u, g) fields and lbm_moments match the oracle exactly."""
    L = lbm()
    shape = SHAPES[lat]
    D = 2 if lat == "D2Q9" else 3
    rho, u, _ = inputs.random_fields(shape, seed=5, dim=D)
    kw, g = _force(lat, shape, "field", seed=9)
    walls = WALLS[lat][-1]
    o = oracle_for(lat, coll, storage, shape, walls, TAU[coll])
    with L.Lattice(lat, coll, storage, shape, walls, TAU[coll], rho=rho, u=u[:D], **kw) as gpu:
        fo = o.init(rho, u, g)
        assert exact_mismatch(gpu.populations(), fo.astype(np.float64)) == 0
        r_g, u_g = gpu.moments()
        r_o, u_o = o.moments(fo, g)
        assert exact_mismatch(r_g, r_o.astype(np.float64)) == 0
        assert exact_mismatch(u_g, u_o[:D].astype(np.float64)) == 0
        gpu.step(4)
        fo = o.run(fo, g, 4)
        assert exact_mismatch(gpu.populations(), fo.astype(np.float64)) == 0
        r_g, u_g = gpu.moments(g_scale=0.25)
        r_o, u_o = o.moments(fo, g, 0.25)
        assert exact_mismatch(u_g, u_o[:D].astype(np.float64)) == 0


def test_poiseuille_channel_config():
    """64 x 32 force-driven channel, D2Q9 BGK, tau-hat 0.8, g = 1e-6, FP64, 10,000 steps:
    bit-exact with the oracle; profile within the known transient of the closed form."""
    from oracle import closed_forms as cf
    L = lbm()
    w = inputs.poiseuille_channel()
    o = oracle_for("D2Q9", "bgk", "f64", w.shape, w.walls, w.tau)
    with L.Lattice("D2Q9", "bgk", "f64", w.shape, w.walls, w.tau, g=(1e-6, 0, 0)) as gpu:
        gpu.step(w.steps)
        fo = o.run(o.init(w.rho, w.u, w.g), w.g, w.steps)
        assert exact_mismatch(gpu.populations(), fo) == 0
        _, u = gpu.moments()
    want = cf.poiseuille_profile(32, 1e-6, 0.8, 0.8)
    err = np.max(np.abs(u[0].reshape(32, 64) - want[:, None])) / want.max()
    assert err < 2e-4


def _sampled_step_parity(gpu, o, lat, shape, walls, g, nodes, storage):
    """One step on the GPU at full size versus the oracle's collision at sampled nodes."""
    pre = gpu.populations(nodes)
    gpu.step(1)
    pop, dst = stream_dest(lat, shape, walls, nodes)
    flat = np.unique(dst)
    post_all = gpu.populations(flat)
    pos = np.searchsorted(flat, dst)
    got = post_all[pop, pos]
    bad = 0
    for j, n in enumerate(nodes):
        want = o.collide_node(pre[:, j].astype(o.dtype), g[:, n])
        want = to_storage(want, storage)
        bad += exact_mismatch(got[:, j], want)
    return bad


def _sample_nodes(shape, k, seed):
    N = int(np.prod(shape))
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    corners = [0, nx - 1, (ny - 1) * nx, N - 1, N - nx, (nz - 1) * nx * ny]
    return np.unique(np.concatenate([rng.integers(0, N, k), corners]))


@pytest.mark.parametrize("storage", ["f64", "f32s"])
def test_kolmogorov_full_size_sampled(storage):
    """1024 x 1024 periodic D2Q9 SMRT shear flow at full size: one step matches the
    oracle's collision at sampled nodes exactly."""
    L = lbm()
    w = inputs.kolmogorov_box()
    o = oracle_for("D2Q9", "smrt", storage, w.shape, w.walls, w.tau)
    with L.Lattice("D2Q9", "smrt", storage, w.shape, w.walls, w.tau, rho=w.rho, u=w.u[:2],
                   g_profile=w.g_profile) as gpu:
        gpu.step(3)
        nodes = _sample_nodes(w.shape, 300, 1)
        g = w.g.astype(o.dtype)
        assert _sampled_step_parity(gpu, o, "D2Q9", w.shape, w.walls, g, nodes, storage) == 0


@pytest.mark.parametrize("variant", [1, 5, 13, 14])
@pytest.mark.parametrize("storage", ["f64", "f32s", "f16s"])
def test_taylor_green_256_sampled(storage, variant):
    """D3Q19 SMRT 256^3 Taylor-Green + sin(z) force (the benchmark workload), at the
    launch configurations the tuner picks for it (256 x 1, general addressing, at most 5
    waves per SIMD, with non-temporal stores or non-temporal loads and stores: variants 13
    and 14), without the wave cap, and with the scalar-base addressing path: one step
    matches the oracle's collision at sampled nodes exactly."""
    L = lbm()
    w = inputs.taylor_green_3d(n=256)
    o = oracle_for("D3Q19", "smrt", storage, w.shape, w.walls, w.tau)
    with L.Lattice("D3Q19", "smrt", storage, w.shape, w.walls, w.tau, rho=w.rho, u=w.u,
                   g_profile=w.g_profile) as gpu:
        gpu.tune(256, 1, variant)
        gpu.step(2)
        nodes = _sample_nodes(w.shape, 200, 2)
        g = w.g.astype(o.dtype)
        assert _sampled_step_parity(gpu, o, "D3Q19", w.shape, w.walls, g, nodes, storage) == 0


@pytest.mark.parametrize("storage", ["f64", "f32s"])
def test_d3q27_fourier_128_sampled(storage):
    """D3Q27 SMRT 128^3 periodic box forced by four seeded Fourier modes (the warm-start
    workload), tuned launch: one step matches the oracle's collision at sampled nodes
    exactly."""
    L = lbm()
    p = inputs.warmstart_problem(2022, box=128)
    shape = (128, 128, 128)
    tau = (p["tau2"], 1.0, 1.0)
    g = inputs.fourier_force(shape, p["modes"])
    o = oracle_for("D3Q27", "smrt", storage, shape, (0, 0, 0), tau)
    rng = np.random.default_rng(5)
    N = int(np.prod(shape))
    rho = 1.0 + 1e-3 * rng.uniform(-1, 1, N)
    u = 0.02 * rng.uniform(-1, 1, (3, N))
    with L.Lattice("D3Q27", "smrt", storage, shape, (0, 0, 0), tau, rho=rho, u=u,
                   g_field=g) as gpu:
        gpu.tune(autotune_steps=5)
        gpu.step(2)
        nodes = _sample_nodes(shape, 200, 3)
        assert _sampled_step_parity(gpu, o, "D3Q27", shape, (0, 0, 0), g.astype(o.dtype), nodes,
                                    storage) == 0


def test_monitors_match_oracle_sums():
    L = lbm()
    shape = (40, 24, 1)
    rho, u, _ = inputs.random_fields(shape, seed=3, dim=2)
    o = oracle_for("D2Q9", "smrt", "f64", shape, (0, 1, 0), TAU["smrt"])
    g = np.array([1e-5, 0, 0])
    with L.Lattice("D2Q9", "smrt", "f64", shape, (0, 1, 0), TAU["smrt"], rho=rho, u=u[:2],
                   g=g) as gpu:
        gpu.step(9)
        m0 = gpu.monitors()  # records u(9)
        gpu.step(1)
        m = gpu.monitors()   # compares u(10) with u(9)
        fo = o.run(o.init(rho, u, g), g, 10)
        r, uu = o.moments(fo, g)
        f9 = o.run(o.init(rho, u, g), g, 9)
        _, u9 = o.moments(f9, g)
    assert m0.step == 9 and m.step == 10
    assert abs(m.mass - r.sum()) <= 1e-12 * r.sum()
    for a in range(2):
        assert abs(m.mom[a] - (r * uu[a]).sum()) <= 1e-12 * np.abs(r * uu[a]).sum()
    assert abs(m.umax - np.sqrt((uu[:2] ** 2).sum(0)).max()) <= 1e-15
    res = np.sqrt(((uu[:2] - u9[:2]) ** 2).sum() / (uu[:2] ** 2).sum())
    assert abs(m.resid - res) <= 1e-10 * res
    assert m.nonfinite == 0


def test_buffers_beyond_4gib_sampled():
    """D3Q19 SMRT 512^3 in FP32-shifted storage: 10.2 GB a population buffer, so slot
    offsets pass 2^32 bytes (64-bit addressing) while each plane stays small enough for
    the scalar-base path.  A smooth field varying along every axis, a z-profile force;
    after two steps, one more step matches the oracle's collision at sampled nodes (the
    first and last nodes of the lattice among them) exactly, at the tuned launch and
    with the scalar-base addressing path."""
    L = lbm()
    n = 512
    shape = (n, n, n)
    k = 2 * np.pi / n
    c = np.arange(n)
    sx, cx = np.sin(k * c), np.cos(k * c)
    u = np.empty((3, n, n, n))  # (component, z, y, x)
    u[0] = 0.02 * sx[None, None, :] * cx[None, :, None] * cx[:, None, None]
    u[1] = -0.02 * cx[None, None, :] * np.sin(2 * k * c)[None, :, None] * cx[:, None, None]
    u[2] = 0.01 * np.cos(3 * k * c)[None, None, :] * sx[:, None, None]
    u = u.reshape(3, -1)
    rho = (1.0 + 1e-3 * cx[None, :, None] * np.sin(3 * k * c)[:, None, None]
           * np.ones(n)[None, None, :]).reshape(-1)
    table = np.zeros((3, n))
    table[0] = 1e-6 * np.sin(k * c)
    table[1] = 5e-7 * np.cos(2 * k * c)
    tau = (0.56, 1.0, 1.0)
    o = oracle_for("D3Q19", "smrt", "f32s", shape, (0, 0, 0), tau)
    with L.Lattice("D3Q19", "smrt", "f32s", shape, (0, 0, 0), tau, rho=rho, u=u,
                   g_profile=(2, table)) as gpu:
        del rho, u
        gpu.tune(256, 1, 13)
        gpu.step(2)
        nodes = _sample_nodes(shape, 300, 7)
        z = nodes // (n * n)
        g = np.zeros((3, n ** 3), o.dtype)  # only the sampled nodes' entries are read
        g[:, nodes] = table[:, z].astype(o.dtype)
        assert _sampled_step_parity(gpu, o, "D3Q19", shape, (0, 0, 0), g, nodes, "f32s") == 0
        gpu.tune(256, 1, 5)
        assert _sampled_step_parity(gpu, o, "D3Q19", shape, (0, 0, 0), g, nodes, "f32s") == 0
