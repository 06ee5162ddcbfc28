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


def test_vcycle_bytes_counts_every_launch_of_the_cycle():
    """2048^2 as the default bench runs it: strips on the finest level, tiles on
    levels 1-5, the one-workgroup tail from 32^2 down; 3D 128^3 per-cell."""
    lk = [("strips", 50, 738)] + [("tiles", 512, 1024)] * 5 + [("tail", 0, 0)] * 5
    n = [2048 * 2048 // 4 ** l for l in range(11)]
    want = (90 + 84) * n[0]
    for l in range(1, 6):
        # pre: 8 reads + 6 writes + 9 coarse values per 4 cells; post: 8 reads,
        # 3 writes, 6 coarse values per 4 cells
        want += 8 * ((8 + 6 + 9 / 4) + (8 + 3 + 6 / 4)) * n[l]
    want += 8 * (9 * n[6] + 2 * sum(n[6:]))
    assert abs(bench.vcycle_bytes(2, (2048, 2048), lk) - want) < 1e-6 * want

    lk3 = [("per-cell", 256, 4096), ("per-cell", 256, 512), ("per-cell", 256, 64),
           ("per-cell", 256, 8)] + [("tail", 0, 0)] * 3
    m = [128 ** 3 // 8 ** l for l in range(7)]
    want3 = 0.0
    for l in range(4):
        launches = [52] * 8 + [8 * (8 + 9 / 8), 8 * (6 + 6 / 8)]
        if l < 3:
            launches.append(8 * 11 / 8)          # right-hand side of the next level
        want3 += sum(launches) * m[l]
    want3 += 8 * (9 * m[4] + 2 * sum(m[4:]))
    assert abs(bench.vcycle_bytes(3, (128,) * 3, lk3) - want3) < 1e-6 * want3
