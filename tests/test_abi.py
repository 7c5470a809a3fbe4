"""CPU-side checks of the C-ABI library: it loads, exports every declared entry point,
and rejects invalid parameters before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


@pytest.mark.parametrize("header", ["lbm.h", "lbm_batch.h", "lbm_nn.h"])
def test_library_exports_every_declared_symbol(header):
    from paper_2212_07494_amd import lbm
    lib = lbm.load()
    names = _declared(header)
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), n
    # the binding covers the same names
    assert set(names) <= set(lbm.EXPORTS)


def test_version_and_strerror():
    from paper_2212_07494_amd import lbm
    lib = lbm.load()
    assert lib.lbm_version() == 100
    assert lib.lbm_strerror(-1) == b"invalid argument"


@pytest.mark.parametrize("change,fragment", [
    (dict(tau=(0.5, 0.8, 1.0)), "tau[2]"),
    (dict(collision="smrt", tau=(0.8, 0.8, 0.9)), "tau[4]"),
    (dict(collision="smrt", tau=(0.8, 0.4, 1.0)), "tau[3]"),
    (dict(shape=(8, 8, 2)), "nz == 1"),
    (dict(shape=(0, 8, 1)), "positive"),
    (dict(rho0=0.0), "rho0"),
    (dict(lattice="D3Q19", shape=(2048, 2048, 1024)), "2^31"),
    (dict(force_order=2), "force_order"),
    (dict(force_order=3), "SMRT"),
    (dict(force_order=4), "SMRT"),
    (dict(collision="rmrt", force_order=4), "SMRT"),
    (dict(force_order=5), "1, 3 or 4"),
    (dict(lattice="D3Q39", shape=(8, 8, 8), collision="smrt", force_order=4),
     "fourth-order moments"),
    (dict(lattice="D3Q27", shape=(8, 8, 8), collision="smrt", force_order=4, max_order=6),
     "not combined with max_order 6"),
    (dict(lattice="D3Q19", shape=(8, 8, 8), collision="smrt", tau_31=0.7, force_order=4),
     "not combined with force_order 4"),
    (dict(tau_bulk=1.2), "tau_bulk needs the SMRT"),
    (dict(collision="rmrt", tau_bulk=1.2), "tau_bulk needs the SMRT"),
    (dict(collision="smrt", tau_bulk=0.5), "must exceed 1/2"),
    (dict(collision="smrt", tau_bulk=float("nan")), "must exceed 1/2"),
    (dict(lattice="D3Q19", shape=(8, 8, 8), tau_31=0.7), "tau_31 needs the SMRT"),
    (dict(collision="smrt", tau_31=0.7), "D2Q9 carries no"),
    (dict(lattice="D3Q19", shape=(8, 8, 8), collision="smrt", tau_31=0.7, force_order=3),
     "not combined with force_order 3"),
    (dict(lattice="D3Q27", shape=(8, 8, 8), collision="smrt", tau_31=0.4), "must exceed 1/2"),
    (dict(lattice="D3Q27", shape=(8, 8, 8), collision="smrt", max_order=5), "4 (default) or 6"),
    (dict(lattice="D3Q19", shape=(8, 8, 8), collision="smrt", max_order=6), "SMRT on D3Q27"),
    (dict(lattice="D3Q27", shape=(8, 8, 8), max_order=6), "SMRT on D3Q27"),
    (dict(mach_limit=-0.1), "mach_limit"),
    (dict(mach_limit=float("nan")), "mach_limit"),
    (dict(rho0=float("nan")), "rho0"),
    (dict(lattice="D3Q39", shape=(8, 8, 2)), "extent >= 3"),
    (dict(lattice="D3Q39", shape=(8, 8, 8), bc=(0, 1, 0)), "periodic boxes only"),
    (dict(lattice="D3Q39", shape=(8, 8, 8), solid=np.zeros(512, np.uint8)), "solid"),
    (dict(lattice="D3Q39", shape=(8, 8, 8), collision="smrt", tau_31=0.7), "D_aaa"),
    (dict(lattice="D3Q39", shape=(8, 8, 8), collision="smrt", max_order=6), "SMRT on D3Q27"),
])
def test_invalid_parameters_rejected(change, fragment):
    from paper_2212_07494_amd import lbm
    kw = dict(lattice="D2Q9", collision="bgk", storage="f64", shape=(8, 8, 1),
              tau=(0.8, 0.8, 1.0), rho0=1.0)
    kw.update(change)
    p, keep = lbm.make_params(**kw)
    with pytest.raises(lbm.LBMError) as ei:
        lbm.lbm_init(p)
    assert ei.value.status == lbm.LBM_EINVAL
    assert fragment in str(ei.value)


def test_unknown_enums_and_null_arguments():
    from paper_2212_07494_amd import lbm
    lib = lbm.load()
    p, keep = lbm.make_params()
    p.storage = 9
    out = C.c_void_p()
    assert lib.lbm_init(C.byref(p), None, None, None, C.byref(out)) == lbm.LBM_EINVAL
    assert out.value is None
    assert lib.lbm_init(None, None, None, None, C.byref(out)) == lbm.LBM_EINVAL
    p, keep = lbm.make_params()
    p.g_kind = lbm.G_FIELD  # field without data
    assert lib.lbm_init(C.byref(p), None, None, None, C.byref(out)) == lbm.LBM_EINVAL
    # calls on a NULL context report a state error
    assert lib.lbm_step(None, 1, None) == lbm.LBM_ESTATE
    assert lib.lbm_free(None) == lbm.LBM_ESTATE
    assert lib.lbm_copy_probe(None, None, 16, 1, 256, 0, None) == lbm.LBM_EINVAL


def test_batch_rejects_invalid_domains():
    from paper_2212_07494_amd import lbm
    with pytest.raises(lbm.LBMError) as ei:
        lbm.Batch([dict(shape=(8, 8, 1)), dict(shape=(8, 8, 1), tau=(0.4, 0.8, 1.0))],
                  lattice="D2Q9", collision="bgk", storage="f32s")
    assert ei.value.status == lbm.LBM_EINVAL and "domain 1" in str(ei.value)
    with pytest.raises(lbm.LBMError):
        lbm.Batch([dict(shape=(8, 8, 1), tau=(0.8, 0.8, 0.5))], collision="smrt")
    with pytest.raises(lbm.LBMError):
        lbm.Batch([dict(shape=(8, 8, 2))], lattice="D2Q9")
    lib = lbm.load()
    assert lib.lbm_batch_advance(None, 1) == lbm.LBM_ESTATE
    assert lib.lbm_batch_free(None) == lbm.LBM_ESTATE
    # the boundary's batched step and the status read, through ctypes
    steps = np.zeros(4, np.int64)
    resid = np.zeros(4)
    assert lib.lbm_batch_step(None, 100, 1e-8, steps.ctypes.data, resid.ctypes.data) == \
        lbm.LBM_ESTATE
    assert lib.lbm_batch_status(None, None) == lbm.LBM_ESTATE


def test_status_codes_and_warning():
    """The warning code is positive and named; the monitor record carries J."""
    from paper_2212_07494_amd import lbm
    lib = lbm.load()
    assert lbm.LBM_WMACH > 0
    assert b"Mach" in lib.lbm_strerror(lbm.LBM_WMACH)
    assert lib.lbm_strerror(lbm.LBM_ENONFINITE) == b"non-finite value in the state"
    names = [f[0] for f in lbm.lbm_monitors._fields_]
    assert names == ["step", "mass", "mom", "j", "umax", "resid", "nonfinite"]
    # lbm_monitors as declared in the header: field order
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    decl = re.search(r"typedef struct \{\s*int64_t step;\s*double (.*?);\s*int64_t nonfinite;",
                     text, flags=re.S)
    assert decl and decl.group(1).replace(" ", "") == "mass,mom[3],j[3],umax,resid"


def test_generated_tables_are_current():
    """lbm_tables.h is what gen_tables.py produces (the build regenerates it)."""
    import importlib.util
    path = os.path.join(ROOT, "paper_2212_07494_amd", "csrc", "gen_tables.py")
    spec = importlib.util.spec_from_file_location("gen_tables", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    tmp = os.path.join(ROOT, "_build", "lbm_tables_check.h")
    os.makedirs(os.path.dirname(tmp), exist_ok=True)
    mod.generate(tmp)
    cur = os.path.join(ROOT, "paper_2212_07494_amd", "csrc", "lbm_tables.h")
    assert open(tmp).read() == open(cur).read()


def test_library_constants_equal_oracle_rationals():
    """The library's independently derived tables equal the oracle's exact rationals."""
    import importlib.util
    from oracle import lattice as olat
    path = os.path.join(ROOT, "paper_2212_07494_amd", "csrc", "gen_tables.py")
    spec = importlib.util.spec_from_file_location("gen_tables", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    for name in olat.ALL_LATTICES:
        vel, w, ms = mod.lattice(name)
        assert mod.sound_speed2(name) == olat.cs2(name)
        _, minv = mod.reconstruction(vel, w, ms, mod.sound_speed2(name))
        assert vel == olat.velocities(name)
        assert w == olat.weights(name)
        assert ms == olat.index_set(name)
        assert [list(r) for r in olat.reconstruction(name)] == minv
        assert np.all(np.isfinite(np.array([[float(x) for x in r] for r in minv])))


def test_checkpoint_calls_validate_arguments(tmp_path):
    """lbm_save / lbm_load reject a NULL or foreign context before touching the GPU."""
    from paper_2212_07494_amd import lbm
    lib = lbm.load()
    assert lib.lbm_save(None, str(tmp_path / "x").encode()) == lbm.LBM_ESTATE
    assert lib.lbm_load(None, str(tmp_path / "x").encode()) == lbm.LBM_ESTATE


def test_lattice_response_rejects_bad_arguments():
    """lbm_ws_lattice_response validates its arguments before creating any context."""
    from paper_2212_07494_amd import lbm
    lib = lbm.load()
    params, keep = lbm.make_params("D3Q27", "smrt", "f64", (1, 1, 1), tau=(0.8, 1.0, 1.0))
    prob = lbm.ws_problem_struct(dict(tau2=0.8, modes=[]))
    out = np.zeros(64)
    assert lib.lbm_ws_lattice_response(None, C.byref(prob), 32, out.ctypes.data) == lbm.LBM_EINVAL
    assert lib.lbm_ws_lattice_response(C.byref(params), C.byref(prob), 32,
                                       out.ctypes.data) == lbm.LBM_EINVAL  # no modes
    assert b"nmodes" in lib.lbm_last_error()
    prob1 = lbm.ws_problem_struct(dict(tau2=0.8, modes=[dict(k=[1, 0, 0], p=[0, 1, 0],
                                                              amp=1e-6, phase=0.0)]))
    assert lib.lbm_ws_lattice_response(C.byref(params), C.byref(prob1), 0,
                                       out.ctypes.data) == lbm.LBM_EINVAL  # box < 1


def test_lattice_waves_rejects_bad_arguments():
    """lbm_ws_lattice_waves validates its arguments before creating any context."""
    from paper_2212_07494_amd import lbm
    lib = lbm.load()
    params, keep = lbm.make_params("D3Q27", "smrt", "f64", (1, 1, 1), tau=(0.8, 1.0, 1.0))
    modes = [dict(k=[1, 0, 0], p=[0, 1, 0], amp=1e-6, phase=0.0),
             dict(k=[0, 2, 0], p=[0, 0, 1], amp=1e-6, phase=0.5)]
    prob = lbm.ws_problem_struct(dict(tau2=0.8, modes=modes))
    k = np.zeros((8, 3), np.int32)
    ph = np.zeros(8)
    amp = np.zeros((8, 27, 2))
    n = C.c_int32()
    args = (k.ctypes.data, ph.ctypes.data, amp.ctypes.data, C.byref(n))
    assert lib.lbm_ws_lattice_waves(C.byref(params), C.byref(prob), 32, 5, 8,
                                    *args) == lbm.LBM_EINVAL
    assert b"order" in lib.lbm_last_error()
    # the bound: n, n + n (n + 1), plus 2 n^2 (n + 1) + C(2n + 2, 3) at order 3
    assert [lib.lbm_ws_max_waves(2, o) for o in (1, 2, 3)] == [2, 8, 8 + 24 + 20]
    assert lib.lbm_ws_max_waves(0, 1) == 0 and lib.lbm_ws_max_waves(4, 5) == 0
    # order 4 adds 2n * 2 n3 + C(2 n2 + 1, 2) + C(2n + 1, 2) * 2 n2 + C(2n + 3, 4) for
    # n2 = n (n + 1) second-order and n3 = 2 n n2 + C(2n + 2, 3) third-order waves
    assert lib.lbm_ws_max_waves(2, 4) == 52 + 4 * 2 * 44 + 78 + 10 * 12 + 35
    frac = lbm.ws_problem_struct(dict(tau2=0.8, modes=[dict(k=[0.5, 0, 0], p=[0, 1, 0],
                                                             amp=1e-6, phase=0.0)]))
    assert lib.lbm_ws_lattice_waves(C.byref(params), C.byref(frac), 32, 1, 8,
                                    *args) == lbm.LBM_EINVAL
    assert b"integer" in lib.lbm_last_error()
    # two modes to second order give 2 + 2 * 3 = 8 waves
    assert lib.lbm_ws_lattice_waves(C.byref(params), C.byref(prob), 32, 2, 7,
                                    *args) == lbm.LBM_EINVAL
    assert b"max_waves" in lib.lbm_last_error()
    assert lib.lbm_ws_lattice_waves(C.byref(params), C.byref(prob), 32, 2, 8,
                                    None, *args[1:]) == lbm.LBM_EINVAL
    bad = lbm.ws_problem_struct(dict(tau2=0.8, modes=[dict(k=[0, 0, 0], p=[0, 1, 0],
                                                            amp=1e-6, phase=0.0)]))
    assert lib.lbm_ws_lattice_waves(C.byref(params), C.byref(bad), 32, 1, 8,
                                    *args) == lbm.LBM_EINVAL
    assert b"k = 0" in lib.lbm_last_error()


def test_set_waves_rejects_invalid_context():
    from paper_2212_07494_amd import lbm
    lib = lbm.load()
    assert lib.lbm_set_waves(None, 0, None, None, None) == lbm.LBM_ESTATE


def test_set_waves_binding_checks_shapes():
    """The binding rejects arrays whose shapes would make the library read past them."""
    from paper_2212_07494_amd import lbm
    k = np.zeros((2, 3), np.int32)
    with pytest.raises(ValueError):
        lbm.lbm_set_waves(None, 19, k, np.zeros(2), np.zeros((2, 9), complex))
    with pytest.raises(ValueError):
        lbm.lbm_set_waves(None, 19, np.zeros((2, 2), np.int32), np.zeros(2),
                          np.zeros((2, 19), complex))
    with pytest.raises(ValueError):
        lbm.lbm_set_waves(None, 19, np.full((2, 3), 0.5), np.zeros(2),
                          np.zeros((2, 19), complex))


def test_lattice_info_matches_oracle_tables():
    """lbm_lattice_info (host only) returns each lattice's velocities and weights in the
    population order of the oracle's tables, D3Q39 included."""
    from oracle import lattice as olat
    from paper_2212_07494_amd import lbm
    lib = lbm.load()
    for name in olat.ALL_LATTICES:
        D, Q = C.c_int32(), C.c_int32()
        e = np.zeros(3 * 39, np.int32)
        w = np.zeros(39)
        assert lib.lbm_lattice_info(lbm.LATTICES[name], C.byref(D), C.byref(Q),
                                    e.ctypes.data_as(C.c_void_p),
                                    w.ctypes.data_as(C.c_void_p)) == 0
        assert Q.value == len(olat.velocities(name)) == lbm.QOF[name]
        assert D.value == olat.dim(name)
        assert [tuple(v) for v in e[:3 * Q.value].reshape(-1, 3)] == olat.velocities(name)
        assert list(w[:Q.value]) == [float(x) for x in olat.weights(name)]
    assert lib.lbm_lattice_info(4, None, None, None, None) == lbm.LBM_EINVAL


def test_warm_start_expansion_rejects_d3q39():
    from paper_2212_07494_amd import lbm
    prob = dict(tau2=0.8, modes=[dict(k=(1, 0, 0), p=(0, 1, 0), amp=1e-6, phase=0.0)] * 4)
    for call in (lbm.lbm_ws_lattice_response, lbm.lbm_ws_lattice_waves):
        with pytest.raises(lbm.LBMError) as ei:
            call(prob, 32, lattice="D3Q39")
        assert "covers D2Q9, D3Q19 and D3Q27" in str(ei.value)
