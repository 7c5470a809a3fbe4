"""Population waves: the device synthesis of lbm_set_waves against its definition, and the
steady response of lbm_ws_lattice_waves against the converged lattice itself -- to first
order the steady state's error is second order in the forcing, to second order it is
third order, which a wrong factor, sign or conjugation in any second-order wave breaks."""
import copy
import math

import numpy as np
import pytest

from oracle import lattice as olat
from paper_2212_07494_amd import inputs
from tests.helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]


def _weights(lat):
    return np.array([olat.to_f64(w) for w in olat.weights(lat)])


def _synth(lat, shape, k, phase, amp, rho0):
    """w_i rho0 + sum_w Re[A_wi exp(i theta_w(x))], written out (Q x N, binary64)."""
    nx, ny, nz = shape
    n = np.arange(nx * ny * nz)
    x, y, z = n % nx, (n // nx) % ny, n // (nx * ny)
    f = np.repeat((_weights(lat) * rho0)[:, None], n.size, axis=1)
    for kw, ph, a in zip(k, phase, amp):
        th = 2 * math.pi * (kw[0] * x / nx + kw[1] * y / ny + kw[2] * z / nz) + ph
        f += np.outer(a.real, np.cos(th)) - np.outer(a.imag, np.sin(th))
    return f


SHAPES = {"D2Q9": (24, 20, 1), "D3Q19": (12, 10, 9), "D3Q27": (10, 8, 7)}


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("storage", ["f64", "f32s", "f16s"])
def test_set_waves_matches_definition(lat, storage):
    from paper_2212_07494_amd import lbm as L
    L.load()
    shape = SHAPES[lat]
    Q = L.QOF[lat]
    rng = np.random.default_rng(11)
    nw = 7
    # wavevectors beyond the box and negative ones exercise the integer reduction
    k = rng.integers(-40, 41, size=(nw, 3)).astype(np.int32)
    phase = rng.uniform(-7.0, 7.0, size=nw)
    amp = (rng.normal(size=(nw, Q)) + 1j * rng.normal(size=(nw, Q))) * 1e-3
    rho0 = 1.25
    shift = rho0 if storage.endswith("s") else 0.0
    want = _synth(lat, shape, k, phase, amp, rho0) - (_weights(lat) * shift)[:, None]
    with L.Lattice(lat, "smrt", storage, shape, (0, 0, 0), (0.8, 1.0, 1.0), rho0=rho0) as lt:
        lt.set_waves(k, phase, amp)
        got = lt.populations()
        assert lt.time == 0
        if storage == "f64":
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)
        else:
            # one rounding of the binary64 value: within one unit of the last place
            eps = 2.0 ** -23 if storage == "f32s" else 2.0 ** -10
            assert np.all(np.abs(got - want) <= eps * np.maximum(np.abs(want), 2.0 ** -14))
        # no waves: the rest state
        lt.set_waves(np.zeros((0, 3), np.int32), np.zeros(0), np.zeros((0, Q)))
        rest = lt.populations()
        np.testing.assert_array_equal(rest, np.repeat(((_weights(lat) * (rho0 - shift))
                                                       .astype(np.float64))[:, None],
                                                      rest.shape[1], axis=1)
                                      if storage == "f64" else np.zeros_like(rest))


@pytest.mark.parametrize("storage", ["f64", "f32s"])
def test_set_waves_with_walls_and_solids_places_values_like_set_populations(storage):
    """With walls and solid nodes the synthesis still gives the definition at every fluid
    node, and it fills the same slots as lbm_set_populations: two steps from either are
    identical."""
    from paper_2212_07494_amd import lbm as L
    L.load()
    lat, shape = "D3Q19", (12, 10, 9)
    N = int(np.prod(shape))
    rng = np.random.default_rng(23)
    solid = (rng.uniform(0, 1, N) < 0.1).astype(np.uint8)
    fluid = solid == 0
    k = rng.integers(-5, 6, size=(5, 3)).astype(np.int32)
    phase = rng.uniform(-3.0, 3.0, size=5)
    amp = (rng.normal(size=(5, 19)) + 1j * rng.normal(size=(5, 19))) * 1e-3
    shift = 1.0 if storage == "f32s" else 0.0
    want = _synth(lat, shape, k, phase, amp, 1.0) - (_weights(lat) * shift)[:, None]
    g = np.zeros((3, N))
    g[0] = 1e-5
    with L.Lattice(lat, "smrt", storage, shape, (0, 1, 1), (0.8, 1.0, 1.0), g_field=g,
                   solid=solid) as lt:
        lt.set_waves(k, phase, amp)
        p1 = lt.populations()
        if storage == "f64":
            np.testing.assert_allclose(p1[:, fluid], want[:, fluid], rtol=0, atol=1e-15)
        else:
            assert np.all(np.abs(p1[:, fluid] - want[:, fluid])
                          <= 2.0 ** -23 * np.abs(want[:, fluid]) + 1e-30)
        lt.step(2)
        s1 = lt.populations()
        lt.set_populations(p1)
        lt.step(2)
        s2 = lt.populations()
    np.testing.assert_array_equal(s1[:, fluid], s2[:, fluid])


def _problem(lat, scale):
    """Two interacting shear waves (p_1 . k_2 and p_2 . k_1 nonzero) on a 16-periodic box,
    velocity amplitude about 2e-3 at scale 1."""
    nu = (0.8 - 0.5) / 3.0
    K = 2 * math.pi / 16
    a = 2e-3 * nu * K * K * scale
    if lat == "D2Q9":
        modes = [dict(k=[1, 0, 0], p=[0, 1, 0], amp=a, phase=0.3),
                 dict(k=[1, 2, 0], p=[2 / math.sqrt(5), -1 / math.sqrt(5), 0], amp=0.7 * a,
                      phase=-1.1)]
    else:
        modes = [dict(k=[1, 0, 0], p=[0, 1, 0], amp=a, phase=0.3),
                 dict(k=[0, 1, 1], p=[1, 0, 0], amp=0.7 * a, phase=-1.1)]
    return dict(tau2=0.8, modes=modes)


@pytest.mark.parametrize("lat,coll", [("D3Q27", "smrt"), ("D2Q9", "bgk"), ("D3Q19", "smrt"),
                                      ("D3Q27", "rmrt")])
def test_second_order_waves_are_the_steady_state_to_third_order(lat, coll):
    from paper_2212_07494_amd import lbm as L
    L.load()
    box = 16
    shape = (box, box, 1) if lat == "D2Q9" else (box, box, box)
    errs = {}
    for scale in (1.0, 0.5):
        prob = _problem(lat, scale)
        k, ph, A = L.lbm_ws_lattice_waves(prob, box, order=2, lattice=lat, collision=coll)
        n = len(prob["modes"])
        assert len(k) == n + n * (n + 1)
        g = inputs.fourier_force(shape, prob["modes"])
        with L.Lattice(lat, coll, "f64", shape, (0, 0, 0), (0.8, 1.0, 1.0), g_field=g) as lt:
            lt.set_waves(k[:n], ph[:n], A[:n])
            f1 = lt.populations()
            lt.set_waves(k, ph, A)
            f2 = lt.populations()
            lt.step(6000)
            prev = lt.populations()
            lt.step(500)
            fss = lt.populations()
        rest = _weights(lat)[:, None]
        e1 = np.abs(fss - f1).max()
        e2 = np.abs(fss - f2).max()
        # converged far below the third-order error
        assert np.abs(fss - prev).max() < 1e-3 * e2, (np.abs(fss - prev).max(), e2)
        errs[scale] = (e1, e2, np.abs(fss - rest).max())
    (e1a, e2a, da), (e1b, e2b, db) = errs[1.0], errs[0.5]
    print(lat, coll, errs)
    assert 3.5 < e1a / e1b < 4.5, errs       # first order misses a second-order term
    assert 6.5 < e2a / e2b < 9.5, errs       # second order misses a third-order term
    assert e2a < 0.05 * e1a and e1a < 0.05 * da, errs


@pytest.mark.parametrize("lat,coll", [("D3Q27", "smrt"), ("D2Q9", "bgk"), ("D3Q19", "smrt"),
                                      ("D3Q19", "rmrt")])
def test_third_order_waves_are_the_steady_state_to_fourth_order(lat, coll):
    """Order 3 (cross and cubic terms): its error against the converged lattice falls
    16-fold per halving of the forcing, and is far below order 2's."""
    from paper_2212_07494_amd import lbm as L
    L.load()
    box = 16
    shape = (box, box, 1) if lat == "D2Q9" else (box, box, box)
    errs = {}
    for scale in (2.5, 1.25):
        prob = _problem(lat, scale)
        k3, ph3, A3 = L.lbm_ws_lattice_waves(prob, box, order=3, lattice=lat, collision=coll)
        k2, ph2, A2 = L.lbm_ws_lattice_waves(prob, box, order=2, lattice=lat, collision=coll)
        assert len(k2) < len(k3) <= L.load().lbm_ws_max_waves(2, 3)
        g = inputs.fourier_force(shape, prob["modes"])
        with L.Lattice(lat, coll, "f64", shape, (0, 0, 0), (0.8, 1.0, 1.0), g_field=g) as lt:
            lt.set_waves(k2, ph2, A2)
            f2 = lt.populations()
            lt.set_waves(k3, ph3, A3)
            f3 = lt.populations()
            lt.step(6000)
            prev = lt.populations()
            lt.step(500)
            fss = lt.populations()
        e2 = np.abs(fss - f2).max()
        e3 = np.abs(fss - f3).max()
        assert np.abs(fss - prev).max() < 1e-2 * e3, (np.abs(fss - prev).max(), e3)
        errs[scale] = (e2, e3)
    (e2a, e3a), (e2b, e3b) = errs[2.5], errs[1.25]
    print(lat, coll, errs)
    assert 6.5 < e2a / e2b < 9.5, errs
    assert 12.0 < e3a / e3b < 20.0, errs
    assert e3a < 0.1 * e2a, errs


@pytest.mark.parametrize("lat,coll", [("D3Q27", "smrt"), ("D2Q9", "bgk")])
def test_fourth_order_waves_are_the_steady_state_to_fifth_order(lat, coll):
    """Order 4 (D2 of orders 1 and 3, of 2 and 2, D3 of 1, 1, 2 and D4 of order 1): its
    error against the converged lattice falls 32-fold per halving of the forcing."""
    from paper_2212_07494_amd import lbm as L
    L.load()
    box = 16
    shape = (box, box, 1) if lat == "D2Q9" else (box, box, box)
    errs = {}
    for scale in (2.5, 1.25):
        prob = _problem(lat, scale)
        k3, ph3, A3 = L.lbm_ws_lattice_waves(prob, box, order=3, lattice=lat, collision=coll)
        k4, ph4, A4 = L.lbm_ws_lattice_waves(prob, box, order=4, lattice=lat, collision=coll)
        assert len(k3) < len(k4) <= L.load().lbm_ws_max_waves(2, 4)
        g = inputs.fourier_force(shape, prob["modes"])
        with L.Lattice(lat, coll, "f64", shape, (0, 0, 0), (0.8, 1.0, 1.0), g_field=g) as lt:
            lt.set_waves(k3, ph3, A3)
            f3 = lt.populations()
            lt.set_waves(k4, ph4, A4)
            f4 = lt.populations()
            lt.step(6000)
            prev = lt.populations()
            lt.step(500)
            fss = lt.populations()
        e3 = np.abs(fss - f3).max()
        e4 = np.abs(fss - f4).max()
        assert np.abs(fss - prev).max() < 1e-2 * e4, (np.abs(fss - prev).max(), e4)
        errs[scale] = (e3, e4)
    (e3a, e4a), (e3b, e4b) = errs[2.5], errs[1.25]
    print(lat, coll, errs)
    assert 12.0 < e3a / e3b < 20.0, errs
    assert 24.0 < e4a / e4b < 40.0, errs
    assert e4a < 0.1 * e3a, errs


def test_lattice_waves_first_order_matches_lattice_response():
    """Order 1 of lbm_ws_lattice_waves carries the same linear response that
    lbm_ws_lattice_response reports as mode coefficients: relative to the Stokes amplitude
    s_j, the wave's density is c_6, c_7 and its physical velocity (momentum plus half the
    force) is (p_j + c_0..2) on the sine and c_3..5 on the cosine."""
    from paper_2212_07494_amd import lbm as L
    L.load()
    box = 32
    prob = copy.deepcopy(inputs.warmstart_problem(701, box=box))
    k, ph, A = L.lbm_ws_lattice_waves(prob, box, order=1)
    coef = L.lbm_ws_lattice_response(prob, box)
    nu = (prob["tau2"] - 0.5) / 3.0
    for j, m in enumerate(prob["modes"]):
        assert np.array_equal(k[j], np.asarray(m["k"]))
        assert ph[j] == m["phase"]
        s = m["amp"] / (nu * (2 * math.pi * np.linalg.norm(m["k"]) / box) ** 2)
        rho = A[j].sum()
        assert abs(-rho.imag / s - coef[j, 6]) < 1e-12 and abs(rho.real / s - coef[j, 7]) < 1e-12
        E = np.array(olat.velocities("D3Q27"), np.float64)
        u = E.T @ A[j] + 0.5 * (-1j) * m["amp"] * np.asarray(m["p"])
        np.testing.assert_allclose(-u.imag / s - np.asarray(m["p"]), coef[j, 0:3], atol=1e-12)
        np.testing.assert_allclose(u.real / s, coef[j, 3:6], atol=1e-12)
        assert np.abs(u).max() > 0.5 * s
