"""Host-side pieces of bench.py and the committed measurement files (no GPU).

* The DRAM traffic of the lookup kernel is taken from the committed counter
  file only while its kernel digest matches the kernel sources; otherwise
  the roofline has no measured bytes.
* --gpus other than 1 exits with a message before anything touches a GPU.
* The committed autotuner cache holds well-formed lines (signature, launch
  shapes in range, best time).
"""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_follows_the_kernel_digest(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic() is None  # no file
    f.write_text(json.dumps({"kernel_digest": bench.kernel_source_digest(), "dram_bytes_per_lookup": 123.0}))
    assert bench.measured_traffic()["dram_bytes_per_lookup"] == 123.0
    f.write_text(json.dumps({"kernel_digest": "0" * 16, "dram_bytes_per_lookup": 123.0}))
    assert bench.measured_traffic() is None
    f.write_text("not json")
    assert bench.measured_traffic() is None


def test_committed_traffic_file_is_well_formed():
    path = os.path.join(ROOT, "profiles", "lookup_traffic_c3.json")
    if not os.path.exists(path):
        pytest.skip("no counter file committed yet")
    with open(path) as fh:
        d = json.load(fh)
    assert len(d["kernel_digest"]) == 16
    # DRAM-side bytes per lookup: read sectors plus written sectors (32 B each)
    # over the lookups of the profiled batch, and the copy calibration's check
    # that those counters count true bytes
    assert d["dram_bytes_per_lookup"] == pytest.approx(
        d["dram_read_bytes_per_lookup"] + d["dram_write_bytes_per_lookup"], rel=1e-9)
    assert 0 < d["dram_bytes_per_lookup"] < 36 + 56 * 300 * 8
    for k in ("dram_read", "dram_write", "read_by_size"):
        assert d["copy_scale"][k] == pytest.approx(1.0, abs=0.01)
    assert os.path.exists(os.path.join(ROOT, d["source"]))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_tuning_cache_lines():
    with open(os.path.join(ROOT, "paper_2403_12345_amd", "tuning_cache.txt")) as fh:
        lines = [ln.split() for ln in fh if ln.strip()]
    assert lines
    sigs = set()
    for f in lines:
        # signature, lookup_ilp, tail, sort_min, in_flight, set tile, set grid, best ms, collide_sort_min, loops
        assert len(f) in (8, 10)
        assert f[0].startswith("single-") or f[0].startswith("set-")
        assert f[0] not in sigs
        sigs.add(f[0])
        assert int(f[1]) in (1, 2, 4)
        assert int(f[4]) > 0 and int(f[4]) <= 1 << 24
        assert float(f[7]) > 0
        if len(f) == 10:
            assert 0 <= int(f[9]) <= 4
