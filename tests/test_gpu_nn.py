"""The warm-start network's GPU kernels against the FP64 reference (oracle/mlp.py).

The reference with bf16=True rounds exactly the operands the GPU rounds, so forward
outputs and gradients agree to FP32 accumulation error, apart from occasional one-ulp
BF16 flips of re-rounded activations.  Checked element by element: every output and
every gradient entry within 2e-2 of the RMS of its layer block (a wrong tile edge or
row would be off by about the RMS), plus 1e-3 relative L2 over each array; against the
unrounded FP64 reference the agreement is at BF16 precision (checked at 2e-2 L2)."""
import math

import numpy as np
import pytest

from oracle import closed_forms, mlp
from paper_2212_07494_amd import inputs
from tests.helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def elementwise(a, b, blocks, bound=2e-2):
    """Largest |a - b| over each block (slices of the flat arrays), in units of the RMS of
    b over that block; asserts it is within bound."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    worst = 0.0
    for sl in blocks:
        rms = float(np.sqrt(np.mean(b[sl] ** 2))) or 1e-300
        e = float(np.max(np.abs(a[sl] - b[sl]))) / rms
        worst = max(worst, e)
        assert e <= bound, (sl, e)
    return worst


def param_blocks(widths):
    out, off = [], 0
    for l in range(len(widths) - 1):
        n, k = widths[l + 1], widths[l]
        out.append(slice(off, off + n * k))
        out.append(slice(off + n * k, off + n * k + n))
        off += n * k + n
    return out


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
    # element by element: each output column, each weight matrix and bias vector
    ey = elementwise(y, y_e, [slice(c, None, widths[-1]) for c in range(widths[-1])])
    eg = elementwise(g, g_e, param_blocks(widths))
    print(f"{widths} x {rows}: worst element error {ey:.1e} (outputs), {eg:.1e} (gradients) "
          "of the block RMS")
    assert rel(y, y_f) < 2e-2 and rel(g, g_f) < 2e-2, (rel(y, y_f), rel(g, g_f))


def test_forward_with_addend():
    """y = network(x) + a: the loss against t is the plain network's loss against t - a."""
    import torch
    from paper_2212_07494_amd import lbm as L
    L.load()
    widths, rows = [34, 96, 96, 4], 700
    p = inputs.mlp_init_params(widths, seed=11).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(12)
    x = rng.standard_normal((rows, 34)).astype(np.float32)
    t = rng.standard_normal((rows, 4)).astype(np.float32)
    a = rng.standard_normal((rows, 4)).astype(np.float32)
    net = L.MLP(widths, max_rows=rows)
    try:
        net.set_params(p)
        xd, td, ad = (torch.tensor(v, device="cuda") for v in (x, t, a))
        y0 = torch.empty((rows, 4), device="cuda")
        y1 = torch.empty((rows, 4), device="cuda")
        net.forward(xd, y0)
        net.forward(xd, y1, ad)
        assert np.array_equal(y1.cpu().numpy(), y0.cpu().numpy() + a)
        net.zero_grads()
        loss = net.loss_backward(td)
        g = net.grads()
    finally:
        net.close()
    t_res = t.astype(np.float64) - a.astype(np.float64)
    l_e, g_e = mlp.loss_and_grad(p, widths, x, t_res, None, bf16=True)
    assert abs(loss - l_e) < 1e-3 * l_e
    assert rel(g, g_e) < 1e-3, rel(g, g_e)


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


def test_features():
    import torch
    from paper_2212_07494_amd import lbm as L
    L.load()
    prob = inputs.warmstart_problem(seed=8, box=64)
    n, box = 16, 64
    xd = torch.empty((n ** 3, L.WS_FEATURES), device="cuda")
    bd = torch.empty((n ** 3, 4), device="cuda")
    bd2 = torch.empty((n ** 3, 4), device="cuda")
    U = L.lbm_ws_features(prob, n, box, xd, bd, base_order=1)
    U2 = L.lbm_ws_features(prob, n, box, xd, bd2, base_order=2)
    assert U2 == U
    x = xd.cpu().numpy().astype(np.float64)
    base = bd.cpu().numpy().astype(np.float64)
    base2 = bd2.cpu().numpy().astype(np.float64)
    # the perturbative steady solutions on the lattice, sampled at the grid points
    sub = (slice(None), slice(None, None, box // n), slice(None, None, box // n),
           slice(None, None, box // n))
    for b, order in ((base, 1), (base2, 2)):
        rho_c, u_c = closed_forms.fourier_perturbative_steady(box, prob["tau2"], prob["modes"], order)
        want_u = (u_c.reshape(3, box, box, box)[sub].reshape(3, -1) / U).T
        want_r = ((rho_c - 1.0).reshape(1, box, box, box)[sub].reshape(-1)) / U
        assert np.max(np.abs(b[:, :3] - want_u)) < 1e-4 * max(1.0, np.abs(want_u).max())
        assert np.max(np.abs(b[:, 3] - want_r)) < 1e-4 * max(1e-3, np.abs(want_r).max())
    nu = (prob["tau2"] - 0.5) / 3
    Ks = [2 * math.pi * np.linalg.norm(m["k"]) / box for m in prob["modes"]]
    s = [m["amp"] / (nu * K * K) for m, K in zip(prob["modes"], Ks)]
    assert math.isclose(U, sum(s), rel_tol=1e-12)
    pos = np.stack(inputs.coords((n, n, n)), 1) * (box / n)
    for j, m in enumerate(prob["modes"]):
        th = 2 * math.pi * pos @ np.asarray(m["k"], np.float64) / box + m["phase"]
        assert np.max(np.abs(x[:, 11 * j: 11 * j + 3] - np.outer(np.sin(th), m["p"]))) < 2e-5
        assert np.max(np.abs(x[:, 11 * j + 3: 11 * j + 6] - np.outer(np.cos(th), m["p"]))) < 2e-5
        assert np.allclose(x[:, 11 * j + 6], s[j] / U, rtol=1e-6)
        assert np.allclose(x[:, 11 * j + 7], Ks[j], rtol=1e-6)
        khat = np.asarray(m["k"], np.float64) / np.linalg.norm(m["k"])
        assert np.max(np.abs(x[:, 11 * j + 8: 11 * j + 11] - khat)) < 1e-6
    assert np.all(base[:, 3] == 0)
    assert np.allclose(x[:, 44], prob["tau2"] - 0.5, rtol=1e-6)
    assert np.allclose(x[:, 45], U / (nu * min(Ks)), rtol=1e-5)


@pytest.mark.parametrize("layout", [0, 1, 2])
def test_reset_fields_equals_init(layout):
    import torch
    from paper_2212_07494_amd import lbm as L
    L.load()
    shape = (12, 10, 8)
    N = int(np.prod(shape))
    rng = np.random.default_rng(9)
    U = 0.02
    if layout:
        net_out = rng.uniform(-1, 1, (N, 4)).astype(np.float32)
        rho = 1.0 + U * net_out[:, 3].astype(np.float64)
        u = (U * net_out[:, :3].astype(np.float64)).T
        arr = net_out if layout == 1 else np.ascontiguousarray(net_out.T)
        dev = torch.tensor(arr, device="cuda")
    else:
        rho = (1.0 + 0.01 * rng.uniform(-1, 1, N)).astype(np.float32).astype(np.float64)
        u = (0.02 * rng.uniform(-1, 1, (3, N))).astype(np.float32).astype(np.float64)
        dev = torch.tensor(np.concatenate([rho, u.ravel()]).astype(np.float32), device="cuda")
    g = inputs.fourier_force(shape, inputs.fourier_modes(seed=3))
    with L.Lattice("D3Q27", "smrt", "f32s", shape, (0, 0, 0), (0.7, 1.0, 1.0), rho=rho, u=u,
                   g_field=g) as a, \
         L.Lattice("D3Q27", "smrt", "f32s", shape, (0, 0, 0), (0.7, 1.0, 1.0), g_field=g) as b:
        b.step(3)
        L.lbm_reset_fields(b.ctx, dev, layout, U)
        assert b.time == 0
        assert np.array_equal(a.populations(), b.populations())


def lowpass_periodic(a, axis):
    """The 7-point periodic filter with transfer 1 - sin^6(k/2), by its definition."""
    c = (11 / 16, 15 / 64, -3 / 32, 1 / 64)
    out = c[0] * a
    for o in (1, 2, 3):
        out = out + c[o] * (np.roll(a, o, axis) + np.roll(a, -o, axis))
    return out


@pytest.mark.parametrize("walls", [(0, 0, 0), (0, 1, 0)])
def test_reset_fields_filter_and_projection(walls):
    """Filtered (periodic axes only) and projected onto mass N rho0 and zero momentum,
    then the same state as lbm_init of those fields; checked against numpy."""
    import torch
    from paper_2212_07494_amd import lbm as L
    L.load()
    shape = (12, 10, 6)   # includes an axis shorter than the filter
    nx, ny, nz = shape
    N = nx * ny * nz
    rng = np.random.default_rng(21)
    U = 0.03
    rows = rng.uniform(-1, 1, (N, 4)).astype(np.float32)
    rows[:, :3] += 0.2   # a net momentum and mass to remove
    rows[:, 3] += 0.1
    rho = 1.0 + U * rows[:, 3].astype(np.float64)
    u = U * rows[:, :3].astype(np.float64).T
    planes = np.concatenate([rho[None], u]).reshape(4, nz, ny, nx)
    for ax, w in enumerate(walls):      # array axes are (plane, z, y, x)
        if not w:
            planes = lowpass_periodic(planes, 3 - ax)
    planes = planes.reshape(4, N)
    rho_f, u_f = planes[0], planes[1:]
    delta = (N * 1.0 - rho_f.sum()) / N
    rho_p = rho_f + delta
    c = (rho_p * u_f).sum(1) / rho_p.sum()
    u_p = u_f - c[:, None]
    g = inputs.fourier_force(shape, inputs.fourier_modes(seed=3))
    with L.Lattice("D3Q27", "smrt", "f64", shape, walls, (0.7, 1.0, 1.0), rho=rho_p, u=u_p,
                   g_field=g) as a, \
         L.Lattice("D3Q27", "smrt", "f64", shape, walls, (0.7, 1.0, 1.0), g_field=g) as b:
        b.step(2)
        flags = L.RESET_FILTER | L.RESET_MASS | L.RESET_MOMENTUM
        L.lbm_reset_fields(b.ctx, torch.tensor(rows, device="cuda"), 1, U, flags=flags)
        fa, fb = a.populations(), b.populations()
        assert np.max(np.abs(fa - fb)) < 1e-15
        m = b.monitors()
        assert abs(m.mass - N) < 1e-12 * N
        assert max(abs(v) for v in m.mom) < 1e-14 * N
        # the checkerboard along every periodic axis is gone
        r_b, u_b = b.moments()
        for ax, w in enumerate(walls):
            if w:
                continue
            sign = (-1.0) ** np.asarray(inputs.coords(shape)[ax])
            assert abs(np.sum(u_b * sign)) < 1e-13 * N


def test_output_scale_and_loss_grad():
    """With an output scale S the network is S * net; its gradients are those of the
    reference network whose last layer is multiplied by S.  loss_grad gives the weighted
    mean-square loss of any array and its gradient."""
    import torch
    from paper_2212_07494_amd import lbm as L
    L.load()
    widths, rows = [34, 64, 4], 500
    p = inputs.mlp_init_params(widths, seed=13).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(14)
    p += 0.01 * rng.standard_normal(p.size)
    p = p.astype(np.float32).astype(np.float64)
    x = rng.standard_normal((rows, 34)).astype(np.float32)
    t = rng.standard_normal((rows, 4)).astype(np.float32)
    S = np.array([0.5, 2.0, 0.125, 1.0], np.float32)
    w = np.array([1.0, 0.5, 2.0, 1.5], np.float32)
    net = L.MLP(widths, max_rows=rows)
    try:
        net.set_params(p)
        net.set_output_scale(S)
        xd, td = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
        yd = torch.empty((rows, 4), device="cuda")
        net.forward(xd, yd)
        net.zero_grads()
        loss = net.loss_backward(td, w)
        g = net.grads()
        dy = torch.empty_like(yd)
        loss2 = net.loss_grad(yd, td, dy, w)
        y = yd.cpu().numpy().astype(np.float64)
    finally:
        net.close()
    # reference: scale the last layer's weights and bias by S (exact in BF16 for these S)
    ps = p.copy()
    nW = 4 * 64
    ps[-(nW + 4):-4] = (p[-(nW + 4):-4].reshape(4, 64) * S[:, None]).ravel()
    ps[-4:] = p[-4:] * S
    y_e, _ = mlp.forward(ps, widths, x, bf16=True)
    l_e, g_e = mlp.loss_and_grad(ps, widths, x, t, w, bf16=True)
    assert rel(y, y_e) < 1e-3
    assert abs(loss - l_e) < 1e-3 * l_e and abs(loss2 - loss) < 1e-9 * loss
    # chain rule back to the unscaled parameters: d/dW_last = S * d/d(S W_last)
    g_e = g_e.copy()
    g_e[-(nW + 4):-4] = (g_e[-(nW + 4):-4].reshape(4, 64) * S[:, None]).ravel()
    g_e[-4:] *= S
    assert rel(g, g_e) < 1e-3, rel(g, g_e)
    d = y - t
    want = 2 * w * d / d.size
    assert np.max(np.abs(dy.cpu().numpy() - want)) < 1e-6 * np.abs(want).max()
