"""The batched engine: many uneven domains in one persistent launch per step.

* Every domain matches the oracle run on that domain alone, bit for bit (binary32
  emulation for the shifted storage), after init and after steps.
* Replays of the captured graph equal eager steps, checked after every replay with
  eager work and synchronisation in between.
* All launch configurations give identical results.
* Run to convergence, channel and shear-box domains reach their closed-form profiles.
"""
import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from paper_2212_07494_amd import inputs
from tests.helpers import exact_mismatch, gpu_available, oracle_for

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]


def lbm():
    from paper_2212_07494_amd import lbm as L
    L.load()
    return L


def d2_domains(n, seed=7494, h_range=(16, 128), l_range=(64, 256)):
    """Seeded channel / shear-box domains of the batched workload (as dicts for
    lbm.Batch) and their force fields."""
    specs = inputs.batch_domains(n, seed=seed, h_range=h_range, l_range=l_range)
    return specs, inputs.batch_domain_dicts(specs)


def g_field_of(dom):
    shape = dom["shape"]
    N = int(np.prod(shape))
    if "g_profile" in dom:
        return inputs.profile_field(shape, *dom["g_profile"])
    if "g_field" in dom:
        return np.asarray(dom["g_field"])
    g = np.zeros((3, N))
    for a in range(3):
        g[a] = dom.get("g", (0, 0, 0))[a]
    return g


@pytest.mark.parametrize("storage", ["f64", "f32s"])
def test_batch_matches_oracle_per_domain(storage):
    L = lbm()
    specs, doms = d2_domains(10)
    with L.Batch(doms, "D2Q9", "smrt", storage) as b:
        b.advance(6)
        for d, dom in enumerate(doms):
            o = oracle_for("D2Q9", "smrt", storage, dom["shape"], dom["walls"], dom["tau"])
            g = g_field_of(dom)
            fo = o.run(o.init(1.0, None, g), g, 6)
            assert exact_mismatch(b.populations(d), fo.astype(np.float64)) == 0, d
            r, u = b.moments(d)
            ro, uo = o.moments(fo, g)
            assert exact_mismatch(u, uo[:2].astype(np.float64)) == 0, d


@pytest.mark.parametrize("tile_bx", [0, 1])
def test_batch_d3q27_field_forced_boxes(tile_bx):
    """Periodic D3Q27 boxes of different sizes with full Fourier force fields and
    initial velocity fields (the warm-start data generator's setting), with the default
    tiles and with linear tiles (layers of 306-460 nodes, so tiles end inside rows)."""
    L = lbm()
    doms = []
    for k, n in enumerate((16, 12, 20)):
        shape = (n, n + 2, n - 3)
        modes = inputs.fourier_modes(seed=100 + k, amp_range=(1e-5, 1e-4))
        g = inputs.fourier_force(shape, modes)
        rho, u, _ = inputs.random_fields(shape, seed=k, u_amp=0.01)
        doms.append(dict(shape=shape, tau=(0.7, 0.9, 1.0), g_field=g, rho=rho, u=u))
    with L.Batch(doms, "D3Q27", "smrt", "f32s") as b:
        b.tune(tile_bx, 4, 1)
        b.advance(4)
        for d, dom in enumerate(doms):
            o = oracle_for("D3Q27", "smrt", "f32s", dom["shape"], (0, 0, 0), dom["tau"])
            fo = o.run(o.init(dom["rho"], dom["u"], dom["g_field"]), dom["g_field"], 4)
            assert exact_mismatch(b.populations(d), fo.astype(np.float64)) == 0, d


def test_graph_replays_equal_eager_steps():
    L = lbm()
    specs, doms = d2_domains(24, seed=11)
    with L.Batch(doms, "D2Q9", "smrt", "f32s") as g, L.Batch(doms, "D2Q9", "smrt", "f32s") as e:
        for rep in range(4):
            # one replay of a 10-step interval (tol 0 and a huge stall count: nobody stops)
            steps, resid, status = g.run(10, 0.0, check_every=10, stall_checks=10 ** 6)
            e.advance(10)
            assert np.all(steps == 10 * (rep + 1)) and np.all(status == L.DOM_RUNNING)
            for d in range(len(doms)):
                assert exact_mismatch(g.populations(d), e.populations(d)) == 0, (rep, d)
            # eager work between replays
            g.moments(0)


def test_launch_configurations_identical():
    L = lbm()
    specs, doms = d2_domains(16, seed=3)
    with L.Batch(doms, "D2Q9", "smrt", "f32s") as ref:
        ref.advance(5)
        want = [ref.populations(d) for d in range(len(doms))]
    for tbx in (0, 1, 64, 256):
        for bpc in (0, 1, 8):
            for v in (0, 2):
                with L.Batch(doms, "D2Q9", "smrt", "f32s") as b:
                    b.tune(tbx, bpc, v)
                    b.advance(5)
                    for d in range(len(doms)):
                        assert exact_mismatch(b.populations(d), want[d]) == 0, (tbx, bpc, v, d)


def test_run_to_convergence_closed_forms():
    """FP64 channels and shear boxes run to resid < 1e-10: channels reach the exact
    discrete Poiseuille profile, boxes the exact discrete Kolmogorov amplitude."""
    L = lbm()
    doms, kinds = [], []
    for k, (H, tau2, g) in enumerate([(16, 0.8, 1e-6), (24, 1.2, 5e-7), (20, 0.6, 1e-6)]):
        doms.append(dict(shape=(64, H, 1), walls=(0, 1, 0), tau=(tau2, 1.0, 1.0), g=(g, 0, 0)))
        kinds.append(("channel", H, tau2, g))
    for k, (H, tau2, A) in enumerate([(32, 0.7, 2e-7), (16, 1.0, 1e-6)]):
        table = np.zeros((3, H))
        table[0] = A * np.sin(2 * math.pi * np.arange(H) / H)
        doms.append(dict(shape=(64, H, 1), walls=(0, 0, 0), tau=(tau2, 1.0, 1.0),
                         g_profile=(1, table)))
        kinds.append(("box", H, tau2, A))
    with L.Batch(doms, "D2Q9", "smrt", "f64") as b:
        steps, resid, status = b.run(200_000, 1e-10, check_every=200, stall_checks=50)
        assert np.all(status == L.DOM_CONVERGED), (status, resid)
        assert np.all(resid < 1e-10)
        for d, (kind, H, tau2, g) in enumerate(kinds):
            _, u = b.moments(d)
            ux = u[0].reshape(H, 64)
            assert np.ptp(ux, axis=1).max() < 1e-12 * np.abs(ux).max()
            if kind == "channel":
                want = cf.poiseuille_profile(H, g, tau2, 1.0)
                err = np.max(np.abs(ux[:, 0] - want)) / want.max()
            else:
                k = 2 * math.pi / H
                U = cf.kolmogorov_amplitude(g, k, tau2, 1.0)
                err = np.max(np.abs(ux[:, 0] - U * np.sin(k * np.arange(H)))) / U
            # converged to resid 1e-10 per step: the remaining error is that of the slowest
            # mode, resid / (decay rate per step)
            assert err < 1e-5, (d, kind, err)
    assert steps.min() > 0
