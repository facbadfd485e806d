"""Host-side logic of bench.py (no GPU): byte models, the counter-record
lookup, the CPU baseline record and the one-GPU guard."""
import json
import os
import subprocess
import sys

import numpy as np

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
    files = ["tiles.hpp", "common.hpp"]
    cfg = {"kernel": 2, "vec": 4, "lanes_per_row": 16, "unroll": 2, "items_per_wg": 2048,
           "tile_cols": 0}
    rec = {"config": cfg, "files": files, "kernel_source_sha": bench.kernel_source_hash(files),
           "fetch_kib": 1000.0, "write_kib": 10.0, "fetch_scale": 2.0, "write_scale": 1.0}
    recs = {"w": [dict(rec, config=dict(cfg, unroll=4)), rec]}
    assert bench.counter_traffic(recs, "w", cfg) == round(1000 * 1024 * 2 + 10 * 1024)
    assert bench.counter_traffic(recs, "w", dict(cfg, unroll=8)) is None
    assert bench.counter_traffic(recs, "other", cfg) is None
    stale = {"w": [dict(rec, kernel_source_sha="0" * 16)]}
    assert bench.counter_traffic(stale, "w", cfg) is None
    # a shape field added after the counters were taken matches only at its default
    assert bench.counter_traffic(recs, "w", dict(cfg, rows_per_block=0)) is not None
    assert bench.counter_traffic(recs, "w", dict(cfg, rows_per_block=4)) is None


def test_committed_counter_records_are_well_formed():
    path = os.path.join(ROOT, "profiles", "hbm_counters.json")
    recs = json.load(open(path))
    assert recs
    for key, lst in recs.items():
        assert isinstance(lst, list) and lst, key
        for r in lst:
            for f in ("config", "files", "kernel_source_sha", "fetch_kib", "write_kib",
                      "fetch_scale", "write_scale", "profile"):
                assert f in r, (key, f)
            assert os.path.exists(os.path.join(ROOT, "profiles", r["profile"]))


def test_cpu_baseline_record():
    A = wl.plain(m=2000, k=2000)
    B = wl.dense(1, A.k, 8)
    out = bench.cpu_baseline(A, B, 8, budget_s=0.2, max_reps=3)
    assert out["kind"] == "oracle" and out["unit"] == "GFLOP/s"
    assert out["cores"] >= 1 and out["value"] > 0
    assert "passes" in out["sample"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert not r.stdout.strip()
