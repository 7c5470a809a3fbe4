"""Monitors, failure detection and the NaN-poison debug pass.

* Monitor records computed inside lbm_step (monitor_every = K) equal the two-call path
  (record at t - 1, compare at t) bit for bit, for K = 1 and K > 1.
* The FP64 sums (mass, sum rho u, J = sum j, max |u|, residual) against the oracle's
  fields on 2-D and 3-D lattices, reduced storage and several block shapes.
* A NaN injected into the state from the host: the in-step monitors see it, the next
  synchronising call returns LBM_ENONFINITE, lbm_step refuses to advance until the
  state is replaced.
* The Mach guard's warning.
* With every buffer a step writes first filled with NaN, results stay bit-identical
  (every slot a step pulls was written by the step before it).
* lbm_batch_step, the boundary's batched call, on the batched workload's domains.
"""
import warnings

import numpy as np
import pytest

from oracle import lattice as olat
from paper_2212_07494_amd import inputs
from tests.helpers import exact_mismatch, gpu_available, oracle_for, to_storage

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]

TAU = (0.58, 0.87, 1.0)


def lbm():
    from paper_2212_07494_amd import lbm as L
    L.load()
    return L


def _fields(shape, dim, seed):
    rho, u, g = inputs.random_fields(shape, seed=seed, dim=dim)
    return rho, u[:dim], g


@pytest.mark.parametrize("lat,storage,K", [("D2Q9", "f64", 1), ("D2Q9", "f64", 4),
                                           ("D3Q19", "f32s", 1), ("D3Q19", "f32s", 3),
                                           ("D3Q27", "f16s", 5), ("D3Q39", "f32s", 2)])
def test_in_step_monitors_equal_two_call_path(lat, storage, K):
    L = lbm()
    shape = (70, 21, 1) if lat == "D2Q9" else (40, 13, 9)
    dim = 2 if lat == "D2Q9" else 3
    rho, u, g = _fields(shape, dim, 4)
    walls = (0, 0, 0) if lat in olat.HIGH_ORDER else (0, 1, 0)
    n = 4 * K
    with L.Lattice(lat, "smrt", storage, shape, walls, TAU, rho=rho, u=u, g_field=g,
                   monitor_every=K) as a, \
            L.Lattice(lat, "smrt", storage, shape, walls, TAU, rho=rho, u=u, g_field=g) as b:
        a.step(n)
        ma = a.monitors()
        b.step(n - 1)
        b.monitors()       # records u(n - 1)
        b.step(1)
        mb = b.monitors()  # compares u(n) with u(n - 1)
        assert ma.step == mb.step == n
        for k in ("mass", "umax", "resid", "nonfinite"):
            assert getattr(ma, k) == getattr(mb, k), (k, getattr(ma, k), getattr(mb, k))
        assert list(ma.mom) == list(mb.mom) and list(ma.j) == list(mb.j)
        assert ma.resid > 0
        # a second read at the same time returns the same record
        ma2 = a.monitors()
        assert ma2.resid == ma.resid and ma2.mass == ma.mass
        # the same states: the in-step passes change nothing
        assert exact_mismatch(a.populations(), b.populations()) == 0


@pytest.mark.parametrize("lat,storage,tunings", [
    ("D2Q9", "f64", [(64, 4, 0), (256, 1, 4)]),
    ("D3Q19", "f32s", [(64, 1, 1), (128, 2, 0), (256, 1, 5)]),
    ("D3Q27", "f64", [(64, 4, 2), (128, 1, 3)]),
    ("D3Q39", "f64", [(64, 2, 1), (256, 1, 5)]),
])
def test_monitor_sums_against_oracle(lat, storage, tunings):
    L = lbm()
    shape = (90, 24, 1) if lat == "D2Q9" else (70, 11, 6)
    dim = 2 if lat == "D2Q9" else 3
    rho, u, g = _fields(shape, dim, 9)
    walls = (0, 0, 0) if lat in olat.HIGH_ORDER else (0, 1, 0)
    o = oracle_for(lat, "smrt", storage, shape, walls, TAU)
    gg = g.astype(o.dtype)
    u3 = np.zeros((3, u.shape[1]))
    u3[:dim] = u
    f9 = o.run(o.init(rho, u3, g), g, 9)
    f10 = o.run(f9, g, 1)
    _, u9 = o.moments(f9, gg)
    r, uu = o.moments(f10, gg)
    r, uu, u9 = (np.asarray(v, np.float64) for v in (r, uu, u9))
    E = np.array(olat.velocities(lat))
    # j = sum_i d_i e_i per node, accumulated in the arithmetic type in population order
    # from -0.0 (the shift w_i rho0 carries no momentum)
    J = np.zeros((3, f10.shape[1]), o.dtype)
    for a in range(3):
        acc = np.full(f10.shape[1], -0.0, o.dtype)
        for i in range(len(E)):
            if E[i, a] == 1:
                acc = acc + f10[i]
            elif E[i, a] == -1:
                acc = acc + (-f10[i])
            elif E[i, a] != 0:  # the longer links of D3Q39
                acc = acc + o.dtype(E[i, a]) * f10[i]
        J[a] = acc
    J = J.astype(np.float64)
    tol_id = 1e-9 if storage == "f64" else 1e-5
    for bx, by, var in tunings:
        with L.Lattice(lat, "smrt", storage, shape, walls, TAU, rho=rho, u=u, g_field=g) as gpu:
            gpu.tune(bx, by, var)
            gpu.step(9)
            gpu.monitors()
            gpu.step(1)
            m = gpu.monitors()
        assert m.step == 10
        assert abs(m.mass - r.sum()) <= 1e-12 * r.sum()
        for a in range(dim):
            ref = (r * uu[a]).sum()
            assert abs(m.mom[a] - ref) <= 1e-11 * np.abs(r * uu[a]).sum(), (a, m.mom[a], ref)
            assert abs(m.j[a] - J[a].sum()) <= 1e-11 * np.abs(J[a]).sum(), (a, m.j[a])
        # J = sum rho u - sum F/2 with F = rho g (eq:half_F)
        for a in range(dim):
            want = (r * uu[a]).sum() - 0.5 * (r * gg[a].astype(np.float64)).sum()
            assert abs(m.j[a] - want) <= tol_id * np.abs(r * uu[a]).sum()
        umax = np.sqrt((uu[:dim] ** 2).sum(0)).max()
        assert abs(m.umax - umax) <= 1e-15
        res = np.sqrt(((uu[:dim] - u9[:dim]) ** 2).sum() / (uu[:dim] ** 2).sum())
        assert abs(m.resid - res) <= 1e-9 * res
        assert m.nonfinite == 0


def test_nonfinite_state_is_reported_and_stops_stepping():
    L = lbm()
    shape = (64, 16, 1)
    w = np.array([float(x) for x in olat.weights("D2Q9")])
    f = inputs.random_state(9, 64 * 16, 3, weights=w)
    with L.Lattice("D2Q9", "smrt", "f64", shape, (0, 1, 0), TAU, monitor_every=2) as gpu:
        gpu.step(4)
        assert gpu.monitors().nonfinite == 0
        bad = f.copy()
        bad[3, 100] = np.nan  # injected from the host
        gpu.set_populations(bad)
        gpu.step(2)  # the in-step check at t = 2 sees it; step itself only enqueues
        with pytest.raises(L.LBMError) as e:
            gpu.moments()  # the next synchronising call
        assert e.value.status == L.LBM_ENONFINITE
        with pytest.raises(L.LBMError) as e:
            gpu.step(1)  # refuses to advance a non-finite state
        assert e.value.status == L.LBM_ENONFINITE
        assert gpu.time == 2
        m = gpu.monitors()
        assert m.nonfinite >= 1
        # replacing the state clears it
        gpu.set_populations(f)
        gpu.step(2)
        rho, u = gpu.moments()
        assert np.isfinite(rho).all() and np.isfinite(u).all()
        assert gpu.monitors().nonfinite == 0


def test_nonfinite_seen_by_step_without_synchronising():
    """lbm_step reads a completed in-step record itself: after the stream drains, the
    next lbm_step call returns LBM_ENONFINITE."""
    import torch
    L = lbm()
    shape = (64, 16, 1)
    w = np.array([float(x) for x in olat.weights("D2Q9")])
    f = inputs.random_state(9, 64 * 16, 3, weights=w)
    f[0, 5] = np.inf
    with L.Lattice("D2Q9", "bgk", "f64", shape, (0, 1, 0), (0.7, 0.7, 1.0),
                   monitor_every=1) as gpu:
        gpu.set_populations(f)
        gpu.step(1)
        torch.cuda.synchronize()
        with pytest.raises(L.LBMError) as e:
            gpu.step(1)
        assert e.value.status == L.LBM_ENONFINITE


def test_mach_guard_warns():
    L = lbm()
    shape = (32, 8, 1)
    N = 32 * 8
    u = np.zeros((2, N))
    u[0] = 0.08  # Ma = 0.08 / sqrt(1/3) = 0.139
    with L.Lattice("D2Q9", "smrt", "f64", shape, (0, 0, 0), TAU, u=u, mach_limit=0.1,
                   monitor_every=1) as gpu:
        with pytest.warns(L.MachWarning):
            gpu.monitors()
        gpu.step(1)
        with pytest.warns(L.MachWarning):
            gpu.moments()  # reads the in-step record of t = 1
    with L.Lattice("D2Q9", "smrt", "f64", shape, (0, 0, 0), TAU, u=u, mach_limit=0.2) as gpu:
        with warnings.catch_warnings():
            warnings.simplefilter("error")
            gpu.monitors()  # below the limit: no warning


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19", "D3Q27"])
@pytest.mark.parametrize("storage", ["f64", "f16s"])
def test_poisoned_buffers_change_nothing(lat, storage):
    """Every buffer a step writes is filled with NaN first: with walls, solid nodes and
    a force field the results stay bit-identical to the unpoisoned run, so no step reads
    a slot the previous step did not write."""
    L = lbm()
    shape = (70, 13, 1) if lat == "D2Q9" else (40, 11, 7)
    dim = 2 if lat == "D2Q9" else 3
    N = int(np.prod(shape))
    rho, u, g = _fields(shape, dim, 5)
    solid = np.random.default_rng(2).uniform(size=N) < 0.1
    solid[0] = False
    out = []
    for poison in (False, True):
        for coll in ("bgk", "smrt"):
            walls = (0, 1, 0) if lat == "D2Q9" else (0, 1, 1)
            with L.Lattice(lat, coll, storage, shape, walls, TAU, rho=rho, u=u, g_field=g,
                           solid=solid, debug_poison=poison) as gpu:
                gpu.step(7)
                r, uu = gpu.moments()
                out.append((r, uu))
    for (ra, ua), (rb, ub) in zip(out[:2], out[2:]):
        assert np.isfinite(ra).all() and np.isfinite(ua).all()
        assert exact_mismatch(ra, rb) == 0 and exact_mismatch(ua, ub) == 0


def test_batch_step_symbol_runs_the_batched_workload():
    """lbm_batch_step on 40 of the batched workload's domains (FP64): every domain ends
    CONVERGED, its reported steps are multiples of the check interval, and the states
    equal lbm_batch_run's with the same interval."""
    L = lbm()
    specs = inputs.batch_domains(40, seed=7494, h_range=(16, 32), l_range=(64, 96))
    doms = inputs.batch_domain_dicts(specs)
    with L.Batch(doms, "D2Q9", "smrt", "f64") as a, L.Batch(doms, "D2Q9", "smrt", "f64") as b:
        sa, ra, st = a.step(400_000, 1e-9)
        sb, rb, stb = b.run(400_000, 1e-9, check_every=100, stall_checks=10)
        assert np.all(st == L.DOM_CONVERGED), (st, ra)
        assert np.all(ra < 1e-9) and np.all(sa % 100 == 0)
        assert np.array_equal(sa, sb) and np.array_equal(ra, rb) and np.array_equal(st, stb)
        for d in range(len(doms)):
            assert exact_mismatch(a.populations(d), b.populations(d)) == 0
