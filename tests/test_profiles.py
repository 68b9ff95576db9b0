"""The committed profiler summaries describe the kernels as they are: the
HBM traffic the benchmark reports is keyed by a hash of the fused kernels'
source, and a summary taken on other source would be dropped (reported as
null) at run time.  Each summary also names the command that produced it."""
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROF = os.path.join(ROOT, "profiles")


def test_traffic_summary_matches_the_kernel_source():
    with open(os.path.join(PROF, "traffic.json")) as fh:
        doc = json.load(fh)
    h = bench.kernel_source_hash()
    entries = [e for cfg in doc.values() for e in cfg.values()]
    assert entries
    for e in entries:
        assert e["source_hash"] == h, (e["kernel"], e["source_hash"], h)
        assert e["bytes_per_launch"] > 0
        # copy calibration: bytes moved per KiB the counter reports
        assert 1.0 <= e["fetch_factor"] <= 4.0 and 0.5 <= e["write_factor"] <= 2.0


def test_summaries_name_their_command():
    for name in os.listdir(PROF):
        if name.endswith(".md"):
            text = open(os.path.join(PROF, name)).read()
            assert "rocprofv3" in text, name
