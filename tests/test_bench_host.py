"""Host-side parts of bench.py: the one-GPU guard, the roofline arithmetic and
the rule that counter traffic is reported only for the kernel sources it was
measured on.  No GPU is touched."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_roofline_arithmetic():
    # 8e9 B in 1 ms is 8000 GB/s: the whole HBM peak
    r = bench.roofline_of("k", 8e9, 1.0, 4e9)
    assert r["achieved"] == pytest.approx(8000.0)
    assert r["frac"] == pytest.approx(1.0)
    assert r["peak"] == 8000.0 and r["unit"] == "GB/s" and r["bound"] == "hbm"
    assert r["traffic_frac"] == pytest.approx(0.5)
    r = bench.roofline_of("k", 1e9, 2.0, None)
    assert r["frac"] == pytest.approx(1e9 / 2e-3 / 1e9 / 8000.0)
    assert r["traffic"] is None and "traffic_frac" not in r
    assert bench.roofline_of("k", 1e9, 0.0, None)["achieved"] == 0.0


def test_traffic_only_for_the_sources_it_was_measured_on(tmp_path):
    sha = bench.kernel_source_sha("sample.hip")
    good = {"kernels": {"sample_kernel": {"source": "sample.hip", "source_sha": sha,
                                          "hbm_bytes_per_launch": 123}}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(good))
    assert bench.load_traffic(str(p), "sample_kernel") == 123
    assert bench.load_traffic(str(p), "level_kernel") is None
    stale = {"kernels": {"sample_kernel": dict(good["kernels"]["sample_kernel"], source_sha="0" * 16)}}
    p.write_text(json.dumps(stale))
    assert bench.load_traffic(str(p), "sample_kernel") is None
    assert bench.load_traffic(str(tmp_path / "missing.json"), "sample_kernel") is None
    p.write_text("not json")
    assert bench.load_traffic(str(p), "sample_kernel") is None


@pytest.mark.parametrize("name", ["large_kernel_traffic.json", "medium_kernel_traffic.json"])
def test_committed_traffic_matches_the_kernels(name):
    """The committed counter summaries were taken on the kernels in the tree,
    so the bench line reports their traffic rather than null."""
    path = os.path.join(ROOT, "profiles", name)
    tr = json.load(open(path))
    for key, k in tr["kernels"].items():
        assert k["source_sha"] == bench.kernel_source_sha(k.get("source", "sample.hip")), key
        assert bench.load_traffic(path, key) == k["hbm_bytes_per_launch"]
