"""Checkpoint / resume: n steps, save, load into a fresh context, n steps equals 2n steps
bit for bit, in every storage mode; mismatched parameters, truncated and foreign files are
rejected with LBM_EINVAL and leave the context as it was."""
import numpy as np
import pytest

from paper_2212_07494_amd import inputs
from tests.helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]

SHAPE = (40, 12, 9)


def make(L, storage, tau=(0.6, 0.9, 1.0), coll="smrt", force_order=1):
    g = inputs.fourier_force(SHAPE, inputs.fourier_modes(seed=4))
    rng = np.random.default_rng(2)
    N = int(np.prod(SHAPE))
    return L.Lattice("D3Q19", coll, storage, SHAPE, (0, 1, 0), tau,
                     rho=1 + 1e-3 * rng.uniform(-1, 1, N), u=0.02 * rng.uniform(-1, 1, (3, N)),
                     g_field=g, force_order=force_order)


@pytest.mark.parametrize("storage", ["f64", "f32", "f32s", "f16s"])
def test_resume_is_bit_exact(tmp_path, storage):
    from paper_2212_07494_amd import lbm as L
    L.load()
    path = tmp_path / "state.ckpt"
    with make(L, storage) as a:
        a.step(40)
        want = a.populations()
        t_want = a.time
    with make(L, storage) as b:
        b.step(20)
        b.save(path)
    with make(L, storage) as c:
        c.load(path)
        assert c.time == 20
        c.step(20)
        assert c.time == t_want
        assert np.array_equal(c.populations(), want)


def test_mismatches_are_rejected(tmp_path):
    from paper_2212_07494_amd import lbm as L
    L.load()
    path = tmp_path / "state.ckpt"
    with make(L, "f32s") as a:
        a.step(3)
        a.save(path)
    data = path.read_bytes()
    (tmp_path / "short.ckpt").write_bytes(data[: len(data) // 2])
    (tmp_path / "junk.ckpt").write_bytes(b"not a checkpoint at all")
    cases = [(dict(storage="f32"), path, "storage"),
             (dict(storage="f32s", tau=(0.61, 0.9, 1.0)), path, "parameters"),
             (dict(storage="f32s", force_order=3), path, "parameters"),
             (dict(storage="f32s"), tmp_path / "short.ckpt", "truncated"),
             (dict(storage="f32s"), tmp_path / "junk.ckpt", "not a checkpoint"),
             (dict(storage="f32s"), tmp_path / "missing.ckpt", "cannot open")]
    for kw, p, frag in cases:
        with make(L, **kw) as b:
            before = b.populations()
            with pytest.raises(L.LBMError) as ei:
                b.load(p)
            assert ei.value.status == L.LBM_EINVAL and frag in str(ei.value), (kw, str(ei.value))
            assert np.array_equal(b.populations(), before) and b.time == 0


def test_resume_is_bit_exact_on_d3q39(tmp_path):
    """The same on the high-order lattice (periodic box, FP32-shifted)."""
    from paper_2212_07494_amd import lbm as L
    L.load()
    path = tmp_path / "state39.ckpt"
    shape = (24, 12, 6)
    rho, u, g = inputs.random_fields(shape, seed=8)

    def mk():
        return L.Lattice("D3Q39", "smrt", "f32s", shape, (0, 0, 0), (0.7, 0.9, 1.0), rho=rho,
                         u=u, g_field=g)
    with mk() as a:
        a.step(40)
        want = a.populations()
    with mk() as b:
        b.step(20)
        b.save(path)
    with mk() as c:
        c.load(path)
        c.step(20)
        assert c.time == 40 and np.array_equal(c.populations(), want)
