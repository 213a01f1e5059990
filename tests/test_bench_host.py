"""Host-side logic of bench.py: the one-GPU contract, the algorithmic bytes and
flops per site it reports against, and the rule that a stored HBM traffic
figure counts only for the kernel sources it was measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("nv", [1, 4, 12])
def test_algorithmic_bytes_per_site(nv):
    # FP32 (8-byte complex words): each link read once, the input read once,
    # the output written once; compressed links keep two of three rows
    assert bench.site_bytes("staggered", nv, 8) == 288 + 48 * nv
    assert bench.site_bytes("wilson", nv, 8) == 288 + 192 * nv
    assert bench.site_bytes("brillouin", nv, 8) == 2880 + 192 * nv
    assert bench.site_bytes("wilson", nv, 8, compressed=True) == 192 + 192 * nv
    assert bench.site_bytes("staggered", nv, 8, compressed=True) == 192 + 48 * nv
    # FP64 doubles, 16-bit storage halves
    assert bench.site_bytes("wilson", nv, 16) == 2 * bench.site_bytes("wilson", nv, 8)
    assert bench.site_bytes("wilson", nv, 4) * 2 == bench.site_bytes("wilson", nv, 8)


def test_headline_bytes_and_flops():
    # 16^3 x 32, N_v = 12: 2592 B/site, 339.7 MB and 2.076 Gflop per application
    vol = 16 * 16 * 16 * 32
    assert bench.site_bytes("wilson", 12, 8) == 2592
    assert bench.site_bytes("wilson", 12, 8) * vol == 339_738_624
    assert bench.FLOPS["wilson"] * vol * 12 == 2_076_180_480
    # the staggered and Wilson conventions: 8 hops of an SU(3) product on 3 or
    # (spin-projected) 6 components plus the accumulation
    assert bench.FLOPS["staggered"] == 570
    assert bench.FLOPS["wilson"] == 1320


def test_stored_traffic_counts_only_for_its_sources(tmp_path, monkeypatch):
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    with open(path) as f:
        data = json.load(f)
    ent = data["wilson_16^3x32_nv12_fp32"]
    assert ent["bytes_per_launch"] > ent["algorithmic_bytes"] > 0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: ent["source_hash"])
    assert bench.measured_traffic("wilson_16^3x32_nv12_fp32") == ent["bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("wilson_16^3x32_nv12_fp32") is None
    assert bench.measured_traffic("no such workload") is None
