"""The learned warm start (paper_2212_07494_amd/resum.py) with the committed network.

* Its forward pass on the features of held-out problems equals the FP64 reference
  network (oracle/mlp.py) with the GPU's BF16 roundings emulated, element by element.
* On 12 held-out problems of the wide forcing family (per-mode Stokes amplitude <= 0.1
  and Reynolds number <= 1, expansions whose series ratio sigma is at least 1e-3; seeds
  disjoint from the training and validation sets), D3Q27 SMRT on 128^3 in FP64, the
  total steps to a per-step residual below 1e-8 from the learned start are at most 0.9 of
  those from the same expansion without the network (order 3, or 4 where the series
  converges slowly).  The converged lattice decides: every run ends at resid < 1e-8.
"""
import numpy as np
import pytest

from oracle import mlp
from tests.helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]


def test_network_forward_matches_reference():
    from paper_2212_07494_amd import lbm as L
    from paper_2212_07494_amd import resum as R
    L.load()
    rs = R.ResumStart(weights=R.WEIGHTS)
    try:
        feats = np.array([ex[4] for _, ex in R.problems(R.TEST_SEED, 6)], np.float32)
        y = rs.predict_y(feats)
        params = rs.net.params().astype(np.float64)
    finally:
        rs.close()
    y_e, _ = mlp.forward(params, R.WIDTHS, feats, bf16=True)
    y_e = y_e * rs.scale.astype(np.float64)
    ch = list(R.LEARNED)  # the other outputs are scaled to zero
    rms = np.sqrt(np.mean(y_e[:, ch] ** 2, axis=0))
    err = np.max(np.abs(y[:, ch] - y_e[:, ch]), axis=0) / rms
    assert np.all(err <= 2e-2), err


def test_learned_start_beats_the_expansion_on_held_out_problems():
    from paper_2212_07494_amd import lbm as L
    from paper_2212_07494_amd import resum as R
    L.load()
    res = R.evaluate(R.WEIGHTS, 12, plain=False)
    tot = res["totals"]
    print({k: v for k, v in res.items() if k != "problems"})
    assert tot["learned"] <= 0.9 * tot["waves"], tot
