"""Host logic of bench.py (CPU): the roofline objects and the oracle
baselines of the bench line are computed from the run's counts as their
definitions state, and the committed counter summaries are read only for the
kernel source and options they were measured with."""
import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _totals(rounds=100, processed=10_000_000, created=4_000_000, fan_windows=100_000):
    return dict(rounds=rounds, processed=processed, created=created, fan_windows=fan_windows, dist_events=300_000,
                angle_events=80_000, tiny=1_000, ich_dropped=50_000, pool_windows=20_000_000, selected=2_000_000,
                scan_fused=2, propagate_launches=25, ms_propagate=2.5, timed_rounds=25, fused_workgroups=768)


def test_single_field_roofline_arithmetic():
    tot = _totals()
    phase = {"select": 0.1, "propagate": 2.5, "organize": 0.2, "events": 0.7}
    wall, steps = 0.05, 2
    roof, phases = bench.roofline_of(tot, phase, 1, wall, steps, traffic=None, counter_flops=None)
    kids = tot["created"] - tot["fan_windows"]
    alg = (bench.PROP_READ_BYTES * tot["processed"] + bench.WINDOW_BYTES * kids
           + bench.DIST_EVENT_BYTES * tot["dist_events"] + bench.ANGLE_EVENT_BYTES * tot["angle_events"]
           + bench.SCAN_BYTES * (tot["pool_windows"] - tot["selected"]))
    per_launch = alg / tot["rounds"]
    launch_s = tot["ms_propagate"] / 1000.0 / tot["propagate_launches"]
    assert roof["alg_bytes_per_launch"] == pytest.approx(per_launch, rel=1e-9)
    assert roof["avg_launch_us"] == pytest.approx(launch_s * 1e6, rel=1e-6)
    assert roof["achieved"] == pytest.approx(per_launch / launch_s / 1e9, rel=1e-4)
    assert roof["frac"] == pytest.approx(roof["achieved"] / bench.HBM_PEAK_GBS, rel=1e-3)
    assert roof["peak"] == 8000.0 and roof["unit"] == "GB/s" and roof["bound"] == "hbm"
    flops = bench.FLOP_PER_WINDOW * tot["processed"] + bench.FLOP_PER_CHILD * (kids + tot["tiny"]
                                                                               + tot["ich_dropped"])
    assert roof["fp64"]["alg_flop_per_launch"] == pytest.approx(flops / tot["rounds"], rel=1e-6)
    assert roof["fp64"]["peak"] == 78.6
    assert sum(phases["share"].values()) == pytest.approx(1.0, abs=1e-3)
    # per-field phase times scale the timed rounds to all rounds
    assert phases["ms_per_field"]["propagate"] == pytest.approx(2.5 / 25 * 100 / 2, rel=1e-3)
    json.dumps(roof)


def test_batch_roofline_arithmetic():
    fs = np.zeros((8, 10), np.int64)
    fs[:, 2] = 1_000_000  # windows processed
    fs[:, 3] = 500_000    # windows created
    opts = {"k": 1, "team_threads": 256, "teams_per_cu": 1, "hops": 1, "gang": 1}  # no committed summary
    r = bench.batch_roofline(fs, 0.01, "c4", opts)
    per_window = bench.PROP_READ_BYTES + bench.WINDOW_BYTES
    assert r["achieved"] == pytest.approx(8e6 * per_window / 0.01 / 1e9, rel=1e-3)
    assert r["lower_bound"] is True
    assert r["traffic"] is None and r["fp64"]["counter_flop_per_launch"] is None
    assert r["fp64"]["alg_flop_per_launch"] == pytest.approx(
        bench.FLOP_PER_WINDOW * 8e6 + bench.FLOP_PER_CHILD * 4e6)


def test_profile_values_follow_source_and_options(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    h = bench.kernel_source_hash()
    (prof / "x.md").write_text(f"kernel_source_sha256_16: {h}\nbench_config_c4: k=1 hops=2\n"
                               "c4_hbm_bytes_per_launch: 123.5\nnote c4_hbm_bytes_per_launch: 9\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    assert bench.profile_value("x.md", "c4_hbm_bytes_per_launch", "k=1 hops=2", "bench_config_c4") == 123.5
    assert bench.profile_value("x.md", "c4_hbm_bytes_per_launch", "k=2 hops=2", "bench_config_c4") is None
    assert bench.profile_value("missing.md", "c4_hbm_bytes_per_launch", "k=1 hops=2") is None
    (prof / "y.md").write_text("kernel_source_sha256_16: 0000000000000000\nbench_config: a\nz: 1\n")
    assert bench.profile_value("y.md", "z", "a") is None  # another kernel source


def test_batched_cpu_baseline_scaling():
    c = {"workers": 4, "wall_s": 3.0, "field_s": [1.0, 2.0, 3.0, 4.0], "processed": [1, 2, 3, 4],
         "fields_per_mesh": 32, "nproc": 6, "cpu_count": 6, "cpu_model": "cpu"}
    b = bench.batched_cpu_baseline(c, batch_ms=100.0)
    assert b["value"] == pytest.approx(1000.0 * 10.0 * 32 / 4)
    assert b["cores"] == 4 and b["kind"] == "oracle"
    assert b["gpu_speedup"] == pytest.approx(800.0)
