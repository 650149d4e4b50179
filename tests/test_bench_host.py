"""Host-side logic of bench.py (CPU, no GPU calls)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_source_hash_covers_every_hip_file(tmp_path, monkeypatch):
    h0 = bench.kernel_source_hash()
    assert h0 == bench.kernel_source_hash() and len(h0) == 64
    # a copy of the sources with one header byte changed hashes differently
    src = os.path.join(ROOT, "paper_2508_04076_amd", "csrc")
    dst = tmp_path / "paper_2508_04076_amd" / "csrc"
    dst.mkdir(parents=True)
    names = sorted(f for f in os.listdir(src) if f.endswith((".hip", ".h")))
    assert any(f.endswith(".h") for f in names) and any(f.endswith(".hip") for f in names)
    for f in names:
        (dst / f).write_bytes(open(os.path.join(src, f), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == h0
    h = dst / names[0]
    h.write_bytes(h.read_bytes() + b"\n")
    assert bench.kernel_source_hash() != h0


def test_counters_of_other_sources_are_not_used(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "hbm_counters_plate_fp64_stress_sums.json").write_text(json.dumps(
        {"workload": "plate", "precision": "fp64", "layout": "stress_sums",
         "kernel_source_sha256": "0" * 64, "kernels": {}}))
    (prof / "hbm_counters_block_mixed_terms.json").write_text(json.dumps(
        {"workload": "block", "precision": "mixed", "layout": "terms",
         "kernel_source_sha256": "1" * 64, "kernels": {}}))
    live = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counters_for(live, "plate", "fp64", "stress_sums") is None
    assert bench.counters_for("0" * 64, "plate", "fp64", "stress_sums")["workload"] == "plate"
    # another layout, precision or workload is not used
    assert bench.counters_for("0" * 64, "plate", "fp64", "terms") is None
    assert bench.counters_for("0" * 64, "plate", "mixed", "stress_sums") is None
    assert bench.counters_for("1" * 64, "block", "mixed", "terms")["workload"] == "block"
    assert bench.counters_for("1" * 64, "block", "fp64", "terms") is None
    assert bench.counters_for("1" * 64, "hex", "mixed", "terms") is None
