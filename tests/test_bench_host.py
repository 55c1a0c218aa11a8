"""Host-side checks of the benchmark's contract and its derived figures."""

import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_distance_error_against_float64():
    import bench
    rng = np.random.default_rng(3)
    X = rng.standard_normal((50, 8)).astype(np.float32)
    Q = rng.standard_normal((4, 8)).astype(np.float32)
    ids = np.array([[0, 1, -1], [2, 3, 4], [5, -1, -1], [6, 7, 8]])
    exact = np.zeros(ids.shape, np.float32)
    for qi in range(4):
        for j, i in enumerate(ids[qi]):
            if i >= 0:
                exact[qi, j] = ((X[i].astype(np.float64) - Q[qi]) ** 2).sum()
    assert bench.distance_error(ids, exact, X, Q, "l2") < 1e-7
    bad = exact.copy()
    bad[1, 2] *= 1.001
    assert abs(bench.distance_error(ids, bad, X, Q, "l2") - 1e-3) < 1e-5


def test_coarse_mfma_roofline_is_the_smaller_bound():
    import bench
    from workloads import CONFIGS
    r = dict(coarse="bf16", stage_ms={"coarse": 0.1})
    c4 = bench.coarse_mfma(CONFIGS["c4"], r)     # 164 MB score matrix: HBM-bound
    assert c4["bound"] == "hbm" and c4["peak"] < c4["mfma_peak"]
    assert abs(c4["achieved"] - 2 * 10_000 * 4096 * 96 / 1e-4 / 1e12) < 0.01
    c5 = bench.coarse_mfma(CONFIGS["c5"], dict(coarse="bf16", stage_ms={"coarse": 0.1}))
    assert c5["bound"] == "mfma" and c5["peak"] == 2500.0   # d = 768: compute-bound
    assert bench.coarse_mfma(CONFIGS["c2"], dict(coarse="exact", stage_ms={"coarse": 0.1})) is None


def test_traffic_only_while_sources_match():
    import bench
    for key, rec in bench.TRAFFIC.items():
        config, setting, form = key[:3]
        opts = {"query_order": key[3]} if form == "plain" else \
            {"query_order": key[3], "first_lists": key[4], "rounds": key[5], "list_order": key[6]}
        assert bench.traffic_key(config, setting, form, opts) == key
        t = bench.recorded_traffic(config, setting, form, opts)
        if bench.source_sha(rec["files"]) == rec["sha"]:
            assert t == int(rec["fetch_kib"] * 1024 * 2.0 + rec["write_kib"] * 1024)
        else:
            assert t is None
    # Defaults: longest-first orders, four first lists, one round; another
    # schedule has no record.
    assert bench.traffic_key("c5", "static x0.5", "batched", {"first_lists": 0, "rounds": 0}) == \
        ("c5", "static x0.5", "batched", 0, 4, 1, 0)
    assert bench.recorded_traffic("c5", "static x0.5", "batched",
                                  {"first_lists": 8, "rounds": 5}) is None
    assert bench.recorded_traffic("c5", "static x0.5", "plain", {"query_order": 1}) is None


def test_probe_ladder_settings():
    import torch

    import bench
    from workloads import CONFIGS, scaled
    c2 = CONFIGS["c2"]
    base = torch.full((5,), 32, dtype=torch.int32)
    lad = bench.probe_ladder(c2, base)
    vals = [int(t[0]) for _, t in lad]
    assert vals == list(bench.NPROBE_LADDER) and all(t.dtype == torch.int32 for _, t in lad)
    small = scaled("c2", n=4000, nq=5, L=20, ncomp=20)   # values above L are left out
    assert [int(t[0]) for _, t in bench.probe_ladder(small, base)] == [1, 2, 3, 4, 6, 8, 12, 16]
    c5 = CONFIGS["c5"]
    draws = torch.tensor([4, 7, 100, 256], dtype=torch.int32)
    lad = bench.probe_ladder(c5, draws)
    assert [lbl for lbl, _ in lad][0] == "static x0.0625"
    x16 = dict(lad)["static x0.0625"]
    assert x16.tolist() == [1, 1, 6, 16]          # rounded, clamped to >= 1
    x2 = dict(lad)["static x2"]
    assert x2.tolist() == [8, 14, 200, 512]
    assert all(int(t.max()) <= c5.L for _, t in lad)


def test_cpu_baseline_times_the_oracle_at_the_given_probe_counts():
    import bench
    from workloads import make_workload, scaled, train_index
    cfg = scaled("c1", n=600, nq=4, L=8, ncomp=8)
    X, Q, nprobe = make_workload(cfg)
    index = train_index(X, cfg)
    job = bench.CpuBaseline(X, Q, cfg.k, cfg.R, per_worker=2)
    job.stage(index)
    row = job.run(np.full(cfg.nq, 3, dtype=np.int32))
    assert row["kind"] == "oracle" and row["unit"] == "queries/s" and row["value"] > 0
    assert row["cores"] >= 1 and "queries" in row["sample"]
    assert job.path is None   # staged files removed


def test_batched_scan_points_follow_the_first_pass_rule():
    import bench
    lens = np.array([100, 50, 300, 10, 10, 10, 10, 10, 500])
    probes = np.array([[0, 1, 2, 3, 4, 5, 6, 7, 8],
                       [8, 0, -1, -1, -1, -1, -1, -1, -1],
                       [3, 4, 5, 6, 7, -1, -1, -1, -1]])
    # one list at least, 120 points: row 0 takes lists 0, 1 (100 < 120, then
    # 150); row 1 list 8; row 2 never reaches 120 points and takes them all
    assert bench.batched_scan_points(probes, lens, 120, 1) == (300 + 50 + 500) + 100 + 0
    # four lists at least: row 0 lists 0..3, row 1 both lists, row 2 all
    assert bench.batched_scan_points(probes, lens, 120, 4) == (40 + 500) + 0 + 0
    # a pool of 1000 points outweighs four lists in row 0 (stops after list 8)
    assert bench.batched_scan_points(probes, lens, 1000, 4) == 0
    # pool 10, one list: every row stops after its first list
    assert bench.batched_scan_points(probes, lens, 10, 1) == 900 + 100 + 40
    # 0 means the default, four lists
    assert bench.batched_scan_points(probes, lens, 40, 0) == bench.batched_scan_points(
        probes, lens, 40, 4)
