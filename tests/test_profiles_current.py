"""The committed counter summaries describe the committed kernels: the
benchmark reports their measured HBM traffic only while the kernel sources
hash to the value recorded with the counters, so a kernel change that is
not re-profiled shows up here (and as traffic null in the bench line)."""
from __future__ import annotations

import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _keys(path):
    import re
    with open(path) as fh:
        return dict(re.findall(r"^- (\w+): `([^`]*)`", fh.read(), flags=re.M))


def test_step_profile_matches_the_step_sources_and_shipped_launch():
    kv = _keys(bench.TRAFFIC_PROFILE)
    assert kv["kernel_source_sha256"] == bench.step_source_hash()
    with open(os.path.join(ROOT, "paper_2311_08927_amd", "data", "autotune_choices.json")) as fh:
        (entry,) = json.load(fh).values()
    launch = "tuned " + ":".join(str(x) for x in entry["choice"])
    assert kv["launch"] == launch
    per = [float(v) for v in kv["traffic_bytes_per_interval"].split(",")]
    assert len(per) >= 20 and all(v > 0 for v in per)
    # the bench line at the benchmark's horizon reads the mean of its intervals
    assert bench.measured_traffic(20, launch) == sum(per[:20]) / 20
    assert bench.measured_traffic(len(per) + 1, launch) is None
    assert bench.measured_traffic(20, "tuned 9:9:9") is None


def test_fixed_profile_matches_the_fixed_sources():
    kv = _keys(bench.FIXED_PROFILE)
    assert kv["kernel_source_sha256"] == bench.step_source_hash(bench.FIXED_SOURCES)
    shape = f"euler|{bench.FIXED_PARTICLES}|10|0.5"
    assert kv["shape"] == shape
    assert bench.fixed_traffic(shape) == float(kv["traffic_bytes_per_launch"])
    assert bench.fixed_traffic(f"rk4|{bench.FIXED_PARTICLES}|10|0.5") is None
