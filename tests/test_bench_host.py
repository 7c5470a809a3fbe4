"""Host-side logic of bench.py, on the CPU: the hash of the step kernel's sources, the
lookup of the committed HBM counters that fills the bench line's roofline.traffic, and
the refusal of runs on more than one GPU."""
import json
import os
import re
import shutil
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2212_07494_amd", "csrc")
COUNTERS = os.path.join(ROOT, "profiles", "step_d3q19_smrt_f32s_256_counters.json")


def _copy_sources(tmp_path):
    dst = tmp_path / "paper_2212_07494_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in bench.STEP_SOURCES:
        shutil.copy(os.path.join(CSRC, f), dst / f)
    return dst


def test_source_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    here = bench.kernel_source_hash()
    dst = _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == here
    node = dst / "lbm_node.h"
    text = node.read_text()
    node.write_text("// a reworded comment\n/* and a block\n   comment */\n\n" + text)
    assert bench.kernel_source_hash() == here
    node.write_text(text.replace("T(0.5) * M.F[a]", "T(0.25) * M.F[a]", 1))
    assert bench.kernel_source_hash() != here


def test_traffic_is_taken_only_for_the_current_sources_and_variant():
    with open(COUNTERS) as fh:
        d = json.load(fh)
    h = d["kernel_source_hash"]
    for variant, nbytes in d["hbm_bytes_by_memory_variant"].items():
        assert bench.measured_traffic(h, "f32s", variant) == nbytes
    assert bench.measured_traffic("0" * 16, "f32s", "nt-store") is None
    assert bench.measured_traffic(h, "f32s", "no-such-variant") is None
    assert bench.measured_traffic(h, "f8", "nt-store") is None
    # every variant the bench line can name has counters
    assert set(bench.MEMORY_VARIANTS) <= set(d["hbm_bytes_by_memory_variant"])


def test_committed_profiles_were_taken_on_the_current_sources():
    """Each profile summary quotes the kernel-source hash it was taken on; a change to the
    step's code without new profiles fails here (and the bench line then reports no
    counter traffic)."""
    here = bench.kernel_source_hash()
    quoted = {}
    for name in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            text = fh.read()
        for m in re.finditer(r"\b([0-9a-f]{16})\b", text):
            if "hash" in text[max(0, m.start() - 200):m.start()]:
                quoted[name] = m.group(1)
    assert "step_d3q19_smrt_f32s_256_counters.json" in quoted
    assert {n: h for n, h in quoted.items() if h != here} == {}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
