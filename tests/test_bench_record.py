"""Host checks of bench.py's measurement records (no GPU).

The committed counter record of the finest-level launches
(profiles/traffic_k_stream2d_2048_fp64.json) must carry every key that
bench.measured_traffic compares before it reports `traffic`: the workload, the
hash of the kernel sources it was measured on, the finest level's kernel
configuration and the bytes of each launch class.  A record missing one of
them makes the bench report `traffic: null` whatever the sources.
"""
import json

import bench


def test_traffic_record_has_what_the_bench_compares():
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    assert rec["workload"] == "2d-2048-fp64"
    assert len(rec["source_sha256"]) == 64
    kind, param, blocks = rec["level0_kernel"]
    assert kind in ("strips", "tiles") and param > 0 and blocks > 0
    for cls in ("pre0", "post0"):
        e = rec["launches"][cls]
        assert e["bytes_per_launch"] > e["algorithmic_bytes_per_launch"] > 0


def test_measured_traffic_is_reported_only_for_the_measured_configuration(monkeypatch):
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["source_sha256"])
    lk = rec["level0_kernel"]
    got = bench.measured_traffic("2d-2048-fp64", "post0", tuple(lk))
    assert got == rec["launches"]["post0"]["bytes_per_launch"]
    assert bench.measured_traffic("2d-1024-fp64", "post0", tuple(lk)) is None
    assert bench.measured_traffic("2d-2048-fp64", "post0", ("tiles", 512, 4096)) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic("2d-2048-fp64", "post0", tuple(lk)) is None
