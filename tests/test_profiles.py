"""The committed measurement records belong to the committed sources (no GPU).

bench.py reports the direct sum's HBM traffic only from a record whose source hash matches
direct.hip; a stale record would silently drop it from the benchmark line.
"""
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_record_matches_source():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["k_direct"]
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    assert rec["source_sha256"] == hashlib.sha256(src).hexdigest()
    cal = rec["copy_calibration"]
    want = 1024 * (rec["fetch_kib_per_dispatch"] * cal["fetch_scale"] + rec["write_kib_per_dispatch"] * cal["write_scale"])
    assert abs(rec["hbm_bytes_per_launch"] / want - 1) < 1e-3
    # a 1 GiB copy reads and writes 1 GiB once each after calibration
    assert abs(cal["fetch_kib"] * cal["fetch_scale"] * 1024 / cal["bytes"] - 1) < 1e-6
    assert abs(cal["write_kib"] * cal["write_scale"] * 1024 / cal["bytes"] - 1) < 1e-6


def test_profile_summaries_present():
    for name in ("k_direct_paper-1e5lens-4096sq.md", "default-bench_all-kernels.md", "farfield_1e6lens-8192sq.md",
                 "farfield_1e7lens-32768sq.md", "k_direct_isa_mix.json", "traffic.json"):
        assert os.path.getsize(os.path.join(ROOT, "profiles", name)) > 0, name
