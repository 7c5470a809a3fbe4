"""The warm-start network's GPU kernels against the FP64 reference (oracle/mlp.py).

The reference with bf16=True rounds exactly the operands the GPU rounds, so forward
outputs and gradients agree to FP32 accumulation error (checked at 1e-3 relative L2, with
occasional one-ulp BF16 flips of re-rounded activations); against the unrounded FP64
reference the agreement is at BF16 precision (reported, checked at 2e-2)."""
import math

import numpy as np
import pytest

from oracle import mlp
from paper_2212_07494_amd import inputs
from tests.helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("widths,rows", [([64, 64], 64), ([34, 96], 1000), ([130, 70], 777),
                                         ([34, 128, 96, 4], 1000), ([34, 512, 512, 512, 512, 4], 4096)])
def test_forward_and_gradients(widths, rows):
    import torch
    from paper_2212_07494_amd import lbm as L
    L.load()
    p = inputs.mlp_init_params(widths, seed=3)
    rng = np.random.default_rng(4)
    p += 0.01 * rng.standard_normal(p.size)  # non-zero biases
    p32 = p.astype(np.float32).astype(np.float64)
    x = rng.standard_normal((rows, widths[0])).astype(np.float32)
    t = rng.standard_normal((rows, widths[-1])).astype(np.float32)
    w = np.linspace(0.5, 2.0, widths[-1]).astype(np.float32)
    net = L.MLP(widths, max_rows=rows)
    try:
        net.set_params(p32)
        assert np.array_equal(net.params(), p32.astype(np.float32))
        xd = torch.tensor(x, device="cuda")
        yd = torch.empty((rows, widths[-1]), device="cuda")
        td = torch.tensor(t, device="cuda")
        net.forward(xd, yd)
        net.zero_grads()
        loss = net.loss_backward(td, w)
        y = yd.cpu().numpy()
        g = net.grads()
    finally:
        net.close()
    y_e, _ = mlp.forward(p32, widths, x, bf16=True)
    l_e, g_e = mlp.loss_and_grad(p32, widths, x, t, w, bf16=True)
    y_f, _ = mlp.forward(p32, widths, x, bf16=False)
    l_f, g_f = mlp.loss_and_grad(p32, widths, x, t, w, bf16=False)
    assert rel(y, y_e) < 1e-3, rel(y, y_e)
    assert abs(loss - l_e) < 1e-3 * l_e
    assert rel(g, g_e) < 1e-3, rel(g, g_e)
    assert rel(y, y_f) < 2e-2 and rel(g, g_f) < 2e-2, (rel(y, y_f), rel(g, g_f))


def test_adam_step():
    import torch
    from paper_2212_07494_amd import lbm as L
    L.load()
    widths = [34, 64, 4]
    p = inputs.mlp_init_params(widths, seed=5).astype(np.float32)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((300, 34)).astype(np.float32)
    t = rng.standard_normal((300, 4)).astype(np.float32)
    net = L.MLP(widths, max_rows=300)
    try:
        net.set_params(p)
        xd, td = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
        yd = torch.empty((300, 4), device="cuda")
        pr = p.astype(np.float64)
        m = np.zeros_like(pr)
        v = np.zeros_like(pr)
        for step in (1, 2, 3):
            net.forward(xd, yd)
            net.zero_grads()
            net.loss_backward(td)
            g = net.grads().astype(np.float64)
            net.adam(1e-3, step)
            pr, m, v = mlp.adam(pr, g, m, v, step, 1e-3)
            got = net.params().astype(np.float64)
            assert np.max(np.abs(got - pr)) < 1e-6, step
    finally:
        net.close()


def test_features_and_upsampling():
    import torch
    from paper_2212_07494_amd import lbm as L
    L.load()
    prob = inputs.warmstart_problem(seed=8, box=64)
    n, box = 16, 64
    xd = torch.empty((n ** 3, L.WS_FEATURES), device="cuda")
    U = L.lbm_ws_features(prob, n, box, xd)
    x = xd.cpu().numpy().astype(np.float64)
    nu = (prob["tau2"] - 0.5) / 3
    Ks = [2 * math.pi * np.linalg.norm(m["k"]) / box for m in prob["modes"]]
    s = [m["amp"] / (nu * K * K) for m, K in zip(prob["modes"], Ks)]
    assert math.isclose(U, sum(s), rel_tol=1e-12)
    pos = np.stack(inputs.coords((n, n, n)), 1) * (box / n)
    for j, m in enumerate(prob["modes"]):
        th = 2 * math.pi * pos @ np.asarray(m["k"], np.float64) / box + m["phase"]
        assert np.max(np.abs(x[:, 8 * j: 8 * j + 3] - np.outer(np.sin(th), m["p"]))) < 2e-5
        assert np.max(np.abs(x[:, 8 * j + 3: 8 * j + 6] - np.outer(np.cos(th), m["p"]))) < 2e-5
        assert np.allclose(x[:, 8 * j + 6], s[j] / U, rtol=1e-6)
        assert np.allclose(x[:, 8 * j + 7], Ks[j], rtol=1e-6)
    assert np.allclose(x[:, 32], prob["tau2"] - 0.5, rtol=1e-6)
    assert np.allclose(x[:, 33], U / (nu * min(Ks)), rtol=1e-5)
    # upsampling: a periodic field sampled on 8^3 and interpolated to 32^3
    nc, nf = 8, 32
    c = np.random.default_rng(1).standard_normal((2, nc ** 3)).astype(np.float32)
    fd = torch.empty((2, nf ** 3), device="cuda")
    L.lbm_upsample_periodic(torch.tensor(c, device="cuda"), nc, 2, fd, nf)
    f = fd.cpu().numpy().reshape(2, nf, nf, nf)
    cc = c.reshape(2, nc, nc, nc).astype(np.float64)
    r = nc / nf
    for (z, y, xx) in [(0, 0, 0), (5, 17, 31), (31, 2, 9), (12, 30, 30)]:
        fx, fy, fz = xx * r, y * r, z * r
        x0, y0, z0 = int(fx), int(fy), int(fz)
        ax, ay, az = fx - x0, fy - y0, fz - z0
        want = 0.0
        for dz, wz in ((0, 1 - az), (1, az)):
            for dy, wy in ((0, 1 - ay), (1, ay)):
                for dx, wx in ((0, 1 - ax), (1, ax)):
                    want = want + wz * wy * wx * cc[:, (z0 + dz) % nc, (y0 + dy) % nc, (x0 + dx) % nc]
        assert np.allclose(f[:, z, y, xx], want, atol=1e-5)
    assert np.allclose(f[:, ::4, ::4, ::4].reshape(2, -1), c, atol=1e-6)


@pytest.mark.parametrize("point_major", [0, 1])
def test_reset_fields_equals_init(point_major):
    import torch
    from paper_2212_07494_amd import lbm as L
    L.load()
    shape = (12, 10, 8)
    N = int(np.prod(shape))
    rng = np.random.default_rng(9)
    U = 0.02
    if point_major:
        net_out = rng.uniform(-1, 1, (N, 4)).astype(np.float32)
        rho = 1.0 + U * U * net_out[:, 3].astype(np.float64)
        u = (U * net_out[:, :3].astype(np.float64)).T
        dev = torch.tensor(net_out, device="cuda")
    else:
        rho = (1.0 + 0.01 * rng.uniform(-1, 1, N)).astype(np.float32).astype(np.float64)
        u = (0.02 * rng.uniform(-1, 1, (3, N))).astype(np.float32).astype(np.float64)
        dev = torch.tensor(np.concatenate([rho, u.ravel()]).astype(np.float32), device="cuda")
    g = inputs.fourier_force(shape, inputs.fourier_modes(seed=3))
    with L.Lattice("D3Q27", "smrt", "f32s", shape, (0, 0, 0), (0.7, 1.0, 1.0), rho=rho, u=u,
                   g_field=g) as a, \
         L.Lattice("D3Q27", "smrt", "f32s", shape, (0, 0, 0), (0.7, 1.0, 1.0), g_field=g) as b:
        b.step(3)
        L.lbm_reset_fields(b.ctx, dev, point_major, U)
        assert b.time == 0
        assert np.array_equal(a.populations(), b.populations())
