"""bench.py's use of the committed counter summaries (CPU): every traffic
summary names its kernel, class, precision and launch shape, and the bench
takes a traffic figure only for that exact launch shape."""
import glob
import os

import bench

PROFILES = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles")


def _traffic_lines():
    out = []
    for path in sorted(glob.glob(os.path.join(PROFILES, "*_traffic.md"))):
        lines = [ln for ln in open(path) if ln.startswith("traffic:")]
        assert len(lines) >= 1, path
        for ln in lines:
            kv = dict(t.split("=", 1) for t in ln.split()[1:])
            out.append((os.path.basename(path), kv))
    return out


def test_every_traffic_summary_is_complete():
    lines = _traffic_lines()
    assert lines
    for name, kv in lines:
        for key in ("kernel", "class", "precision", "lanes", "trip", "xcd", "bytes_per_launch"):
            assert key in kv, (name, key)
        assert int(kv["bytes_per_launch"]) > 0
        assert name.split("_")[0] in bench.WORKLOADS, name


def test_traffic_only_for_the_measured_launch_shape():
    for name, kv in _traffic_lines():
        wl = name.split("_")[0]
        args = (wl, kv["precision"], kv["class"], int(kv["lanes"]), int(kv["trip"]), int(kv["xcd"]))
        assert bench.measured_traffic(*args) == int(kv["bytes_per_launch"])
        other_lanes = 64 if int(kv["lanes"]) != 64 else 32
        assert bench.measured_traffic(wl, kv["precision"], kv["class"], other_lanes, int(kv["trip"]),
                                      int(kv["xcd"])) is None
        assert bench.measured_traffic(wl, kv["precision"], kv["class"], int(kv["lanes"]), 2 if int(kv["trip"]) == 1 else 1,
                                      int(kv["xcd"])) is None
        assert bench.measured_traffic(wl, "FP64", kv["class"], int(kv["lanes"]), int(kv["trip"]),
                                      int(kv["xcd"])) is None
