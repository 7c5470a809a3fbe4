"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle: lbm_oracle.c in its three builds (binary64, binary32 emulation, plain
  order), compiled with -fsanitize=address,undefined into a standalone driver
  (oracle/sanitize_driver.c) that runs every whole-lattice entry point, collision,
  boundary set and option of every lattice.
* The library's host side: the runtime units compiled for the host only (no device
  code) with the same sanitizers, linked into a driver that calls the C ABI without a
  GPU: parameter validation, lattice tables, error paths of context creation, the
  warm-start features and order scaling, checkpoint arguments.

The sanitizers abort on the first error (-fno-sanitize-recover=all); the executables
run as child processes, so nothing sanitized is loaded into the test process.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import lattice as lat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")


def _table_file(path, L, real):
    t = lat.tables(L, real)
    with open(path, "wb") as fh:
        fh.write(np.array([t["D"], t["Q"], t["NM"]], np.int32).tobytes())
        for k in ("e", "opp", "mi"):
            fh.write(np.ascontiguousarray(t[k], np.int32).tobytes())
        for k in ("w", "H", "Minv"):
            fh.write(np.ascontiguousarray(t[k], real).tobytes())
        fh.write(np.array([t["ics2"]], np.float64).tobytes())


@pytest.mark.parametrize("build", ["f64", "f32", "plain"])
def test_oracle_under_sanitizers(build, tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = tmp_path / f"san_oracle_{build}"
    defs = {"f64": ["-DREAL=double"], "f32": ["-DREAL=float"],
            "plain": ["-DREAL=double", "-DPLAIN"]}[build]
    src = os.path.join(ROOT, "oracle", "sanitize_driver.c")
    subprocess.run(["gcc", "-std=c11", "-fopenmp", "-ffp-contract=off", *SAN, *defs, src, "-o",
                    str(exe), "-lm"], check=True, capture_output=True, text=True)
    real = np.float32 if build == "f32" else np.float64
    for L in lat.ALL_LATTICES:
        tf = tmp_path / f"{L}_{build}.bin"
        _table_file(tf, L, real)
        r = subprocess.run([str(exe), str(tf)], capture_output=True, text=True, env=ENV,
                           timeout=600)
        assert r.returncode == 0 and "runtime error" not in r.stderr, (L, r.stdout, r.stderr[-3000:])
        assert "0 with non-finite" in r.stdout, r.stdout


RUNTIME_UNITS = ("lbm_runtime", "lbm_aux", "lbm_batch_runtime", "lbm_nn", "lbm_ws_expansion",
                 "lbm_d2q9", "lbm_d3q19", "lbm_d3q27", "lbm_d3q39")


HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _hipcc(args):
    r = subprocess.run([HIPCC, *args], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]


def test_library_host_code_under_sanitizers(tmp_path):
    """Every runtime unit built as for the library, with the host pass instrumented
    (the device code is compiled normally and never runs here), linked with
    tests/native/sanitize_runtime.c and run with no GPU present."""
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    import concurrent.futures as cf
    csrc = os.path.join(ROOT, "paper_2212_07494_amd", "csrc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", csrc]
    common = ["-O1", "-g", "-fPIC", "-fno-omit-frame-pointer", "-ffp-contract=off",
              "-Xarch_host", "-fsanitize=address,undefined",
              "-Xarch_host", "-fno-sanitize-recover=all"]
    device = ["-std=c++20", "--offload-arch=gfx950",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

    def unit(name):
        obj = str(tmp_path / f"{name}.o")
        _hipcc([*device, *common, *inc, "-c", os.path.join(csrc, f"{name}.hip"), "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(unit, RUNTIME_UNITS))
    drv = str(tmp_path / "driver.o")
    _hipcc(["-x", "c", "-std=c11", *common, *inc, "-c",
            os.path.join(ROOT, "tests", "native", "sanitize_runtime.c"), "-o", drv])
    exe = str(tmp_path / "san_runtime")
    _hipcc(["--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address,undefined",
            drv, *objs, "-o", exe])
    env = dict(ENV, HIP_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr, (r.stdout, r.stderr[-3000:])
    assert "0 failures" in r.stdout, r.stdout
