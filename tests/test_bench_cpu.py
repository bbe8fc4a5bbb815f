"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
byte model and the rule that HBM counters are reported only for the kernel
sources, workload and launch shape they were taken on."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_launch():
    # stats: occupied samples, allocated corners gathered, gradient corners, valid rays
    stats = (10, 40, 30, 5)
    assert bench.alg_bytes(stats, 7, 2, 2) == 44 * 7 + 32 * 10 + 112 * 40 + 24 * 2
    assert bench.alg_bytes(stats, 7, 2, 3) == 44 * 7 + 32 * 10 + 112 * 40 + 24 * 2 + 224 * 30


def _profile(tmp_path, sha, workload="wl", block=64, variant=1, traffic="123456"):
    p = tmp_path / "traffic.md"
    p.write_text("# counters\n\n"
                 f"- workload: `{workload}`\n- block: `{block}`\n- variant: `{variant}`\n"
                 f"- sources_sha256: `{sha}`\n- traffic_bytes_per_launch: `{traffic}`\n"
                 "- fetch_kib_per_launch: `10`\n- write_kib_per_launch: `100`\n"
                 "- fetch_scale: `0.5`\n- write_scale: `1.0`\n")
    return p.name


def test_traffic_only_for_matching_sources_workload_and_launch(tmp_path, monkeypatch):
    sha = bench.sources_sha256()
    monkeypatch.setattr(bench, "PROFILES_DIR", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILES", {"wl": _profile(tmp_path, sha),
                                                    "other": "missing.md"})
    t = bench.measured_traffic("wl", 64, 1)
    assert t["bytes"] == 123456.0 and t["read_bytes"] == 20 * 1024 and t["write_bytes"] == 100 * 1024
    assert bench.measured_traffic("other", 64, 1) is None
    assert bench.measured_traffic("unknown", 64, 1) is None
    assert bench.measured_traffic("wl", 128, 1) is None
    assert bench.measured_traffic("wl", 64, 0) is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILES", {"wl": _profile(tmp_path, "0" * 64)})
    assert bench.measured_traffic("wl", 64, 1) is None


def test_roofline_fraction_is_measured_traffic_over_peak():
    tr = {"bytes": 2.0e9, "read_bytes": 0.5e9, "write_bytes": 1.5e9}
    r = bench.roofline(40.0e9, 0.25e9, 4.0, tr, "k", "c2_room256_1200x680_mapping")
    assert r["bound"] == "latency" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(500.0) and r["frac"] == pytest.approx(500.0 / 8000.0)
    assert r["frac"] <= 1.0 and r["traffic"] == 2.0e9
    assert r["traffic_over_compulsory"] == pytest.approx(8.0)
    assert r["gather_issue"]["gbs"] == pytest.approx(10000.0)
    none = bench.roofline(40.0e9, 0.25e9, 4.0, None, "k", "c2_room256_1200x680_mapping")
    assert none["achieved"] is None and none["frac"] is None and none["traffic"] is None


def test_sources_digest_covers_the_kernel_sources():
    # the fused kernel's translation unit: render.hip and every header it includes
    files = set(bench.KERNEL_SOURCES)
    csrc = os.path.join(ROOT, "paper_2307_03404_amd", "csrc")
    pending = ["render.hip"]
    seen = set()
    while pending:
        f = pending.pop()
        if f in seen:
            continue
        seen.add(f)
        with open(os.path.join(csrc, f)) as fh:
            src = fh.read()
        pending += re.findall(r'^#include "([^"]+)"', src, re.M)
    assert {"paper_2307_03404_amd/csrc/" + f for f in seen} == files
    d = bench.sources_sha256()
    assert len(d) == 64 and d == bench.sources_sha256()
