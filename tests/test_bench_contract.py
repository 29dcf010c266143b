"""CPU: the benchmark's helpers that shape its JSON line (no GPU needed)."""
import os

import numpy as np

import bench


def test_recorded_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = bench.kernel_source_sha()
    (prof / "s.md").write_text(f"# x\n\n- source_sha256: {sha}\n- traffic_bytes_per_launch_R32: 123\n")
    (prof / "old.md").write_text("- source_sha256: deadbeef\n- traffic_bytes_per_launch_R32: 5\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: sha)
    assert bench.recorded_traffic("s.md", "traffic_bytes_per_launch_R32") == 123
    assert bench.recorded_traffic("s.md", "traffic_bytes_per_launch_R16") is None
    assert bench.recorded_traffic("old.md", "traffic_bytes_per_launch_R32") is None  # stale counters
    assert bench.recorded_traffic("missing.md", "x") is None


def test_roofline_takes_the_bucket_with_the_most_work():
    m = {"buckets": [{"R": 32, "n_max": 2048, "p_max": 32, "ms_per_launch": 4000.0, "row_updates": 2e12},
                     {"R": 16, "n_max": 1024, "p_max": 32, "ms_per_launch": 4500.0, "row_updates": 5e11}]}
    r = bench.alu_roofline(m)
    assert r["kernel"].startswith("k_wave bucket R=32")
    ops = bench.OPS_PER_ROW_UPDATE * 2e12
    assert abs(r["achieved"] - ops / 4.0 / 1e12) < 1e-9
    assert abs(r["frac"] - ops / 4.0 / bench.PEAK_VALU_LANE_OPS) < 1e-12
    assert r["bound"] == "alu" and r["traffic"] is None


def test_c4_parity_sample_holds_the_largest_problems():
    from paper_2510_15649_amd import workloads as W
    w = W.config4(problems=range(600), path_len=2)
    ids = bench.c4_parity_solves(w, n_uniform=8, n_big=6)
    ns = np.diff(w.row_off)
    big = (ns[ids] > 1024) & (w.p[ids] > 24)
    assert big.sum() >= 6 and len(ids) >= 12 and np.all(np.diff(ids) > 0)


def test_rows_per_lane_buckets():
    assert [bench.rows_per_lane(n) for n in (1, 64, 65, 128, 129, 1024, 1025, 2048)] == [1, 1, 2, 2, 4, 16, 32, 32]
