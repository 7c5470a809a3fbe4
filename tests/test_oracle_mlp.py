"""Pins of the FP64 network reference (oracle/mlp.py) against finite differences,
torch's bfloat16 conversion and the closed form of Adam's first step."""
import numpy as np
import pytest

from oracle import mlp
from paper_2212_07494_amd import inputs


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(5000) * 10.0 ** rng.integers(-8, 8, 5000)).astype(np.float32)
    x = np.concatenate([x, np.float32([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 65504.0])])
    want = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), want)
    assert mlp.bf16_round(1.0 + 2 ** -8) == 1.0            # tie to even
    assert mlp.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def test_gelu_gradient_finite_difference():
    z = np.linspace(-6, 6, 1001)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(z))) < 1e-8


def test_loss_gradient_finite_difference():
    widths = [5, 7, 6, 3]
    p = inputs.mlp_init_params(widths, seed=1)
    p[p == 0] = 0.01  # non-zero biases
    rng = np.random.default_rng(2)
    x = rng.standard_normal((11, 5))
    t = rng.standard_normal((11, 3))
    w = np.array([1.0, 0.5, 2.0])
    loss, g = mlp.loss_and_grad(p, widths, x, t, w)
    h = 1e-6
    for idx in rng.choice(p.size, 40, replace=False):
        e = np.zeros_like(p)
        e[idx] = h
        lp, _ = mlp.loss_and_grad(p + e, widths, x, t, w)
        lm, _ = mlp.loss_and_grad(p - e, widths, x, t, w)
        assert abs((lp - lm) / (2 * h) - g[idx]) < 1e-7 * max(1.0, abs(g[idx]))
    assert g.size == mlp.num_params(widths) == p.size


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([3.0, -0.2, 1e-3, 0.0])
    p1, m, v = mlp.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-12)
    assert np.allclose(p1[:3], -0.01 * np.sign(g[:3]), rtol=1e-9)
    assert p1[3] == 0.0
