"""Host-side logic of bench.py (no GPU): the one-GPU guard and the rule that
the HBM traffic figure is reported only for the kernel sources its counters
were taken with."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert res.returncode != 0
    line = json.loads(res.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def _sources_hash():
    h = hashlib.sha256()
    for f in bench.TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def _profile(tmp_path, traffic, source_hash):
    p = tmp_path / "traffic.md"
    p.write_text("# counters\n\nmachine-readable:\n"
                 f"traffic_bytes_per_launch = {traffic}\nsource_hash = {source_hash}\n")
    return str(p)


def test_traffic_reported_only_for_matching_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _profile(tmp_path, 123456789, _sources_hash()))
    assert bench.measured_traffic() == 123456789.0
    # counters taken with other sources: no figure
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _profile(tmp_path, 123456789, "0" * 16))
    assert bench.measured_traffic() is None


def test_traffic_missing_or_malformed_profile_gives_none(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.md"))
    assert bench.measured_traffic() is None
    bad = tmp_path / "bad.md"
    bad.write_text(f"traffic_bytes_per_launch = many\nsource_hash = {_sources_hash()}\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(bad))
    assert bench.measured_traffic() is None


def test_committed_traffic_profile_names_its_sources():
    """The committed profile carries a figure and a 16-digit hash of the
    forward kernel's sources (whether it matches depends on whether the
    counters were re-taken after the last kernel change)."""
    vals = {}
    for line in open(os.path.join(ROOT, "profiles", "hbm_traffic_headline_bf16.md")):
        if " = " in line:
            k, v = line.strip().split(" = ", 1)
            vals[k] = v
    assert float(vals["traffic_bytes_per_launch"]) > 0
    assert len(vals["source_hash"]) == 16 and int(vals["source_hash"], 16) >= 0
