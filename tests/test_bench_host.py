"""Host-side logic of bench.py: the roofline's traffic figure is taken only
from counters recorded on the same kernel sources and launch shape (else it
is null), and the byte counts per node update follow the field set and
scheme."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1003_0282_amd import workloads as W  # noqa: E402


def test_traffic_only_for_matching_sources_and_shape(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_hash", lambda: "abc")
    d = {"kernel_hash": "abc", "by_launch": [{"launch": "128,1,0,0,1", "hbm_bytes_per_launch": 7.0},
                                             {"launch": "256,1,0,0,1", "hbm_bytes_per_launch": 5.0}]}
    (prof / "traffic_w.json").write_text(json.dumps(d))
    assert bench.traffic_entry("w", "128,1,0,0,1") == 7.0
    assert bench.traffic_entry("w", "256,1,0,0,1") == 5.0
    assert bench.traffic_entry("w", "64,4,0,0,1") is None
    assert bench.traffic_entry("missing", "128,1,0,0,1") is None
    d["kernel_hash"] = "old"
    (prof / "traffic_w.json").write_text(json.dumps(d))
    assert bench.traffic_entry("w", "128,1,0,0,1") is None


def test_bytes_per_update():
    pipe = W.roofline_pipe()
    assert bench.bytes_per_update(pipe, 0) == 144 and bench.bytes_per_update(pipe, 1) == 72
    assert bench.bytes_per_update(dict(pipe, original=True), 0) == 176
    assert bench.bytes_per_update(W.cavity(16, 24, 100.0), 1) == 104
    assert bench.bytes_per_update(W.melt(10.0, 10.0, 1e3), 1) == 136


def test_traffic_key_covers_device_code_and_layout(tmp_path, monkeypatch):
    """The key of the traffic files changes with the solver's device code and
    with the host code that lays the populations out, and not with the rest
    of the host runtime (the counters depend only on the first two)."""
    src = os.path.join(ROOT, "paper_1003_0282_amd", "csrc")
    text = {f: open(os.path.join(src, f)).read() for f in os.listdir(src) if f.startswith("lbaxi")}
    hip = text["lbaxi.hip"]
    assert "\n// host runtime\n" in hip
    cut = hip.index("\n// host runtime\n")
    a = hip.index("\n// Row-blocked layout", cut)
    b = hip.index("\n// Device workspace", a)
    pkg = tmp_path / "paper_1003_0282_amd" / "csrc"
    pkg.mkdir(parents=True)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))

    def key(h):
        for f, t in text.items():
            (pkg / f).write_text(h if f == "lbaxi.hip" else t)
        return bench.kernel_hash()

    base = key(hip)
    assert key(hip[:cut // 2] + " " + hip[cut // 2:]) != base          # device code
    assert key(hip[:(a + b) // 2] + " " + hip[(a + b) // 2:]) != base  # layout
    assert key(hip[:b + 40] + " " + hip[b + 40:]) == base              # rest of the host runtime
