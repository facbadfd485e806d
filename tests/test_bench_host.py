"""Host-side logic of bench.py (no GPU): byte models, the counter-record
lookup, the CPU baseline record and the one-GPU guard."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_1803_08601_amd import workloads as wl  # noqa: E402


def test_byte_models_headline_values():
    # power law 1M x 1M, 16M entries, n = 64, float32: A once, B once, C once
    assert bench.bytes_min(1_000_000, 1_000_000, 16_000_000, 64, 4, 4) == 644_000_004
    # every entry gathers its 256-byte B row
    assert bench.bytes_gather(1_000_000, 16_000_000, 64, 4, 4) == 4_484_000_004
    # bf16 values and B halve those terms
    assert bench.bytes_min(10, 20, 30, 8, 2, 2) == 4 * 11 + 6 * 30 + 2 * 20 * 8 + 4 * 10 * 8


def test_counter_lookup_needs_same_shape_and_sources():
    cfg = {"kernel": 2, "vec": 4, "lanes_per_row": 16, "unroll": 2, "items_per_wg": 2048,
           "tile_cols": 0}
    rec = {"config": cfg, "kernel_source_sha": bench.kernel_source_hash(),
           "traffic_bytes": 2_058_240.0, "l2_hit_rate": 0.5, "profile": "x.md"}
    recs = {"w": [dict(rec, config=dict(cfg, unroll=4)), rec]}
    assert bench.counter_record(recs, "w", cfg) is rec
    assert bench.counter_record(recs, "w", dict(cfg, unroll=8)) is None
    assert bench.counter_record(recs, "other", cfg) is None
    stale = {"w": [dict(rec, kernel_source_sha="0" * 16)]}
    assert bench.counter_record(stale, "w", cfg) is None
    # a shape field added after the counters were taken matches only at its default
    assert bench.counter_record(recs, "w", dict(cfg, rows_per_block=0)) is not None
    assert bench.counter_record(recs, "w", dict(cfg, rows_per_block=4)) is None
    f = bench.traffic_fields(recs, "w", cfg, 1_000_000, 4_000_000, 0.5)
    assert f["traffic"] == 2_058_240 and f["traffic_over_bytes_min"] == 2.058
    assert f["bytes_min_frac"] == round(1e6 / 0.5e-3 / 1e9 / 8000, 4)
    assert f["gather_model_frac"] == round(4e6 / 0.5e-3 / 1e9 / 8000, 4)
    none = bench.traffic_fields({}, "w", cfg, 1_000_000, None, 0.5)
    assert none["traffic"] is None and none["gather_model_frac"] is None


def _counter_csv(path, dispatches):
    """A rocprofv3-style counter_collection.csv: dispatches = [(name, {ctr: value})]."""
    import csv
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Correlation_Id", "Dispatch_Id", "Agent_Id", "Kernel_Name", "Counter_Name",
                    "Counter_Value"])
        for i, (name, ctrs) in enumerate(dispatches):
            for c, v in ctrs.items():
                w.writerow([i + 1, i + 1, 1, name, c, v])


def test_record_counters_from_profiler_output(tmp_path):
    """Records and summaries come from the last `steps` dispatches of each of
    a row's kernels (the cold steps), scaled by the copy calibration."""
    import csv
    run = tmp_path / "run"
    copy = [("__amd_rocclr_copyBuffer", {"FETCH_SIZE": 524288.0})] * 3
    _counter_csv(str(run / "copy" / "fetch" / "h" / "c_counter_collection.csv"), copy)
    _counter_csv(str(run / "copy" / "write" / "c_counter_collection.csv"),
                 [("__amd_rocclr_copyBuffer", {"WRITE_SIZE": 1048576.0})] * 3)
    main, fix = "void spmmk::k_merge<spmmk::F32, 4, 2>(int)", "void spmmk::k_merge_fixup<x>(f)"
    # a tuning candidate, then two warm and two cold steps of (main, fix-up)
    seq = [main] + [main, fix] * 4
    vals = {"FETCH_SIZE": [999.0] + [10.0, 1.0, 10.0, 1.0, 20.0, 2.0, 30.0, 3.0],
            "WRITE_SIZE": [999.0] + [5.0, 1.0, 5.0, 1.0, 6.0, 1.0, 8.0, 3.0]}
    rowd = run / "powerlaw-n64-f32"
    for sub, ctr in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        _counter_csv(str(rowd / sub / "r_counter_collection.csv"),
                     [(nm, {ctr: v}) for nm, v in zip(seq, vals[ctr])])
    _counter_csv(str(rowd / "l2" / "r_counter_collection.csv"),
                 [(nm, {"TCC_HIT_sum": 1.0, "TCC_MISS_sum": 3.0,
                        # busy half the time: 256 TAs, GUI_ACTIVE summed over 8 XCDs
                        "TA_TA_BUSY_sum": 0.5 * 256 * 100.0 / 8, "GRBM_GUI_ACTIVE": 100.0})
                  for nm in seq])
    os.makedirs(rowd / "trace")
    with open(rowd / "trace" / "r_kernel_stats.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs",
                    "MaxNs", "StdDev"])
        w.writerow([main, 5, 5000, 1000, 90, 900, 1100, 1])
        w.writerow([fix, 4, 40, 10, 10, 9, 11, 1])
    cfg = {"kernel": 1, "vec": 4}
    (rowd / "manifest.json").write_text(json.dumps([{
        "row": "powerlaw-n64-f32", "config": cfg, "steps": 2,
        "patterns": [r"\bk_merge<", r"\bk_merge_fixup<"], "bytes_min": 100_000,
        "bytes_gather": 400_000, "kernel_ms_cold_mean": 0.5}]))
    (rowd / "cmd.txt").write_text("--quick --no-cpu-baseline --steps 2 --warmup 1")
    key = "0 1 2 3 4 5 6 7 8 9 10 1 1"
    (rowd / "tune.txt").write_text(f"spmm-tune-cache 2\n{key}  2 4 16 2 2048 0 0 0 0  0.5\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    recs = bench.record_counters(str(run), profiles=str(prof))
    # the traced run's autotuner choices are kept for the bench to load
    assert (prof / "bench_tune_cache.txt").read_text().splitlines() == [
        "spmm-tune-cache 2", f"{key}  2 4 16 2 2048 0 0 0 0  0.5"]
    r = recs["powerlaw-n64-f32"][0]
    assert r["fetch_scale"] == 2.0 and r["write_scale"] == 1.0
    assert r["fetch_kib"] == 25.0 + 2.5 and r["write_kib"] == 7.0 + 2.0
    assert r["traffic_bytes"] == 27.5 * 1024 * 2 + 9.0 * 1024
    assert r["l2_hit_rate"] == 0.25 and r["ta_busy"] == 0.5
    assert r["kernel_source_sha"] == bench.kernel_source_hash()
    text = (prof / r["profile"]).read_text()
    assert "python3 bench.py --quick --no-cpu-baseline --steps 2 --warmup 1" in text
    assert "powerlaw-n64-f32" in text
    # a counter pass that planned another shape than the traced run is refused
    (rowd / "fetch.manifest.json").write_text(json.dumps([{
        "row": "powerlaw-n64-f32", "config": {"kernel": 0, "vec": 4}}]))
    with pytest.raises(SystemExit, match="planned"):
        bench.record_counters(str(run), profiles=str(prof))
    assert bench.counter_record(json.load(open(prof / "hbm_counters.json")),
                                "powerlaw-n64-f32", cfg) is not None


def test_committed_counter_records_are_well_formed():
    path = os.path.join(ROOT, "profiles", "hbm_counters.json")
    recs = json.load(open(path))
    assert recs
    for key, lst in recs.items():
        assert isinstance(lst, list) and lst, key
        for r in lst:
            for f in ("config", "kernel_source_sha", "fetch_kib", "write_kib",
                      "fetch_scale", "write_scale", "traffic_bytes", "profile"):
                assert f in r, (key, f)
            assert os.path.exists(os.path.join(ROOT, "profiles", r["profile"]))


def test_cpu_baseline_record():
    A = wl.plain(m=2000, k=2000)
    B = wl.dense(1, A.k, 8)
    out = bench.cpu_baseline(A, B, 8, budget_s=0.2, max_reps=3)
    assert out["kind"] == "oracle" and out["unit"] == "GFLOP/s"
    assert out["cores"] >= 1 and out["value"] > 0
    assert "passes" in out["sample"] and "march=native" in out["sample"]
    assert out["one_thread"]["value"] > 0
    assert out["host"]["affinity_threads"] >= 1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert not r.stdout.strip()


def test_write_summary_table(tmp_path):
    """Sweep records become one markdown table (nested values as JSON) under
    the command that made them."""
    f = tmp_path / "s.md"
    bench.write_summary(str(f), "T", "about", [{"a": 1, "b": {"x": 2}}, {"a": 3, "c": None}])
    text = f.read_text().splitlines()
    assert text[0] == "# T" and text[7].startswith("python3 bench.py")
    assert "| a | b | c |" in text
    assert '| 1 | `{"x":2}` |  |' in text and "| 3 |  |  |" in text
