"""Host checks of bench.py's measurement records (no GPU).

The committed counter records (profiles/traffic.json, one per workload) must
carry every key that bench.measured_traffic compares before it reports
`traffic`: the sources the counters were taken on and their hash, the finest
level's kernel configuration and the bytes of each launch class.  A record
missing one of them makes the bench report `traffic: null` whatever the
sources.
"""
import json
import os

import bench


def _records():
    with open(bench.TRAFFIC_FILE) as fh:
        return json.load(fh)


def test_traffic_records_have_what_the_bench_compares():
    recs = _records()
    assert recs, "no counter record"
    for workload, rec in recs.items():
        assert rec["workload"] == workload
        assert len(rec["source_sha256"]) == 64
        assert rec["sources"] and all(os.path.exists(os.path.join(bench.ROOT, f))
                                      for f in rec["sources"])
        kind, param, blocks = rec["level0_kernel"]
        assert kind in ("strips", "tiles", "zmarch") and param > 0 and blocks > 0
        assert rec["launches"]
        for cls, e in rec["launches"].items():
            assert cls in ("pre0", "post0", "refine")
            assert e["bytes_per_launch"] > 0 and e["algorithmic_bytes_per_launch"] > 0


def test_measured_traffic_is_reported_only_for_the_measured_configuration(monkeypatch):
    recs = _records()
    workload, rec = next(iter(recs.items()))
    cls = next(iter(rec["launches"]))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda sources: rec["source_sha256"])
    lk = rec["level0_kernel"]
    got = bench.measured_traffic(workload, cls, tuple(lk))
    assert got["bytes_per_launch"] == rec["launches"][cls]["bytes_per_launch"]
    assert bench.measured_traffic("no-such-workload", cls, tuple(lk)) is None
    other = "tiles" if lk[0] != "tiles" else "strips"
    assert bench.measured_traffic(workload, cls, (other, 7, 4096)) is None
    # the same kind of finest-level kernel with another autotuned block size
    assert bench.measured_traffic(workload, cls, (lk[0], lk[1] * 2, lk[2])) is not None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda sources: "0" * 64)
    assert bench.measured_traffic(workload, cls, tuple(lk)) is None


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
        # the finest level reads no f_phi, f_p: 44 B per color launch, and its
        # residual + restriction (z marching, 128^3 >= 2^20 cells) 6 values
        launches = ([44] * 8 + [8 * (6 + 9 / 8), 8 * (6 + 6 / 8)] if l == 0
                    else [52] * 8 + [8 * (8 + 9 / 8), 8 * (6 + 6 / 8)])
        if l < 3:
            launches.append(8 * 11 / 8)          # right-hand side of the next level
        want3 += sum(launches) * m[l]
    want3 += 8 * (9 * m[4] + 2 * sum(m[4:]))
    assert abs(bench.vcycle_bytes(3, (128,) * 3, lk3) - want3) < 1e-6 * want3


def test_vcycle_bytes_follow_the_tuned_sweeps():
    """(nu1, nu2) = (1, 2) on the finest level, 3 and 3 below it, bilinear
    prolongation: one pre launch and one post launch on the finest level plus
    the prolongation launch; two of each on the tiled coarse levels."""
    lk = [("strips", 50, 738)] + [("tiles", 512, 1024)] * 5 + [("tail", 0, 0)] * 5
    n = [2048 * 2048 // 4 ** l for l in range(11)]
    want = 8 * ((9 + 9 / 4) + (9 + 6 + 6 / 4)) * n[0]
    for l in range(1, 6):
        want += 8 * ((2 * 11 + 3 + 9 / 4) + (2 * 11 + 6 + 6 / 4)) * n[l]
    want += 8 * (9 * n[6] + 2 * sum(n[6:]))
    got = bench.vcycle_bytes(2, (2048, 2048), lk, (1, 2, 3, 3, 1))
    assert abs(got - want) < 1e-6 * want


def test_traffic_record_from_counter_files(tmp_path, monkeypatch):
    """write_traffic_record: calibration by the 256 MiB copy, the finest-level
    full launches of each pattern (within 2% of the largest counters), the
    counted/algorithmic ratio that the bench applies to its own launches."""
    cells = 1000
    kib = 1024.0
    rows = {"FETCH_SIZE": [], "WRITE_SIZE": []}

    def dispatch(d, name, fetch_bytes, write_bytes, blocks=21):
        # the calibration below reads FETCH_SIZE as half the bytes read
        rows["FETCH_SIZE"].append((d, name, fetch_bytes / 2 / kib, blocks))
        rows["WRITE_SIZE"].append((d, name, write_bytes / kib, blocks))

    dispatch(1, "__amd_rocclr_copyBuffer", bench.COPY_BYTES, bench.COPY_BYTES, 256)
    zero = "void chhs::k_tile2d<float, false, 2, 1, false, true, 512, false, 16, true>(...)"
    full = "void chhs::k_tile2d<float, false, 2, 1, false, true, 512, false, 16, false>(...)"
    dispatch(2, zero, 40 * cells, 12 * cells)           # 52 B counted, 46 algorithmic
    dispatch(3, full, 50 * cells, 12 * cells)           # 62 B counted, 58 algorithmic
    dispatch(4, full, 10 * cells, 3 * cells)            # fewer instances active: not covered
    dispatch(5, full, 90 * cells, 12 * cells, 84)       # another tile height: not covered
    paths = {}
    for name, rs in rows.items():
        f = tmp_path / f"{name}_counter_collection.csv"
        with open(f, "w") as fh:
            fh.write("Dispatch_Id,Kernel_Name,Grid_Size,Workgroup_Size,Counter_Name,Counter_Value\n")
            for d, k, v, b in rs:
                fh.write(f'{d},"{k}",{b * 512},512,{name},{v}\n')
        paths[name] = str(f)
    run = {"config": {"workload": "w", "cells": cells}, "level_kernels": [["tiles", 512, 21]]}
    bj = tmp_path / "bench.json"
    bj.write_text(json.dumps(run) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    bench.write_traffic_record(paths["FETCH_SIZE"], paths["WRITE_SIZE"], str(bj))
    rec = json.loads((tmp_path / "traffic.json").read_text())["w"]
    pre = rec["launches"]["pre0"]
    assert pre["dispatches"] == 2
    assert abs(pre["bytes_per_launch"] - (52 + 62) / 2 * cells) < 1
    assert pre["algorithmic_bytes_per_launch"] == (46 + 58) / 2 * cells
    assert "post0" not in rec["launches"] and "refine" not in rec["launches"]
