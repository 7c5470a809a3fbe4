"""Womersley flow (paper Sec. III.B) on the GPU: a 50 x 200 D2Q9 channel (periodic in x,
halfway bounce-back plates in y) driven by the uniform force -A_p cos(2 pi t / T),
T = 1200, nu = 0.1 (tau2 = 0.8), A_p = 1e-4, from rest, with the per-step force factor of
lbm_step.  Checked against the oracle (exact, first period), against the exact odd-sector
recursion of the lattice (20 periods), and against the continuum solution at 16 phases
of the 20th period (the paper's comparison; what remains is the slow transient of the
static start, 2.7% of the profile at the phases where it is smallest)."""
import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from tests.helpers import exact_mismatch, gpu_available, oracle_for

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]

NX, NY, T, NU, AP = 50, 200, 1200, 0.1, 1e-4
TAU = (3 * NU + 0.5, 1.0, 1.0)
G = (-AP, 0.0, 0.0)


def scales(k):
    """Force factors s_0 .. s_k; s_0 = 1, so the rest state lbm_init builds with the force
    at factor 1 is the static start."""
    return np.cos(2 * math.pi * np.arange(k + 1) / T)


@pytest.mark.parametrize("coll", ["smrt", "bgk"])
def test_first_period_matches_oracle(coll):
    from paper_2212_07494_amd import lbm as L
    L.load()
    k = T
    s = scales(k)
    o = oracle_for("D2Q9", coll, "f64", (NX, NY, 1), (0, 1, 0), TAU)
    g = np.array(G)
    f = o.run(o.init(1.0, None, g * s[0]), g, k, gscale=s[:k])
    with L.Lattice("D2Q9", coll, "f64", (NX, NY, 1), (0, 1, 0), TAU, g=G) as gpu:
        gpu.step(k, g_scale=s[:k])
        assert exact_mismatch(gpu.populations(), f) == 0


@pytest.mark.parametrize("coll", ["smrt", "bgk"])
def test_twenty_periods(coll):
    from paper_2212_07494_amd import lbm as L
    L.load()
    k = 20 * T
    s = scales(k + T)
    om = 2 * math.pi / T
    want = cf.odd_sector_evolve(np.full(NY, -AP), s[:k + 1], TAU[0], TAU[1], coll, walls=True)
    with L.Lattice("D2Q9", coll, "f64", (NX, NY, 1), (0, 1, 0), TAU, g=G) as gpu:
        gpu.step(k, g_scale=s[:k])
        rho, u = gpu.moments(g_scale=s[k])
        ux = u[0].reshape(NY, NX)
        # the lattice's own dynamics, to FP64 accumulation over 24,000 steps
        assert np.max(np.abs(ux - want[:, None])) < 1e-9 * np.abs(want).max()
        assert np.max(np.abs(u[1])) < 1e-12 * np.abs(want).max()
        # the paper's comparison: phases n T / 16 of the 20th period against the continuum
        errs = []
        t = k - T
        with L.Lattice("D2Q9", coll, "f64", (NX, NY, 1), (0, 1, 0), TAU, g=G) as gp2:
            gp2.step(t, g_scale=s[:t])
            for n in range(16):
                _, u2 = gp2.moments(g_scale=s[t])
                uc = cf.womersley_profile(NY, NU, AP, om, t)
                errs.append(np.linalg.norm(u2[0].reshape(NY, NX)[:, 0] - uc) / np.linalg.norm(uc))
                gp2.step(T // 16, g_scale=s[t:t + T // 16])
                t += T // 16
        print(coll, "E2 against the continuum by phase", np.round(errs, 4).tolist())
        assert max(errs) < 3.5e-2 and np.median(errs) < 1e-2, errs


def test_fp32_shifted_storage():
    """FP32-shifted storage over 20 periods against FP64 storage."""
    from paper_2212_07494_amd import lbm as L
    L.load()
    k = 20 * T
    s = scales(k)
    out = {}
    for st in ("f64", "f32s"):
        with L.Lattice("D2Q9", "smrt", st, (NX, NY, 1), (0, 1, 0), TAU, g=G) as gpu:
            gpu.step(k, g_scale=s[:k])
            out[st] = gpu.moments(g_scale=s[k])[1][0]
    e2 = np.linalg.norm(out["f32s"] - out["f64"]) / np.linalg.norm(out["f64"])
    print("FP32-shifted vs FP64, E2", e2)
    assert e2 < 1e-5, e2
