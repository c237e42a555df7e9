"""Host-side logic that needs no GPU: the bench's roofline accounting and
traffic lookup, the tuner's grid candidates, and the single-GPU guard."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_roofline_hbm_kernel_arithmetic():
    b = load_bench()
    p = dict(n=1_000_000, P=200)
    kernels = {"kick_drift": dict(avg_us=20.0, total_ms=1.0)}
    r = b.kernel_roofline("kick_drift", kernels, None, 0, p, 0)
    # 120 B per particle over 20 us: 6 TB/s of the 8 TB/s peak
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(120 * 1e6 / 20e-6 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["work_per_launch"] == 120 * 1_000_000


def test_roofline_pair_kernel_counts_flops_of_in_cutoff_pairs_only():
    b = load_bench()
    p = dict(n=1000, P=10)
    kernels = {"pair_charged": dict(avg_us=1.0, total_ms=1.0)}
    cnt = {"pair_charged": (10, 20, 5000, 30)}  # coul pairs, lj pairs, candidates, shell members
    r = b.kernel_roofline("pair_charged", kernels, cnt, 0, p, 0)
    # candidates outside the cutoffs and the shell's walk and ranking are overhead, not work
    assert r["work_per_launch"] == b.FLOPS_COUL_PAIR * 10 + b.FLOPS_LJ_PAIR * 20
    assert r["shell_members_per_s"] == pytest.approx(30 / 1e-6)  # reported apart
    assert r["achieved"] == pytest.approx((27 * 10 + 22 * 20) / 1e-6 / 1e12)
    assert r["peak"] == b.PEAK_FP64_TFLOPS
    r32 = b.kernel_roofline("pair_charged", kernels, cnt, 0, p, 1)
    assert r32["peak"] == b.PEAK_FP32_TFLOPS


def test_roofline_fourier_kernels_count_charged_mode_pairs():
    b = load_bench()
    p = dict(n=1000, P=7)
    kernels = {"rho_partial": dict(avg_us=2.0, total_ms=1.0), "gather": dict(avg_us=2.0, total_ms=1.0)}
    r = b.kernel_roofline("rho_partial", kernels, None, 300, p, 0)
    g = b.kernel_roofline("gather", kernels, None, 300, p, 0)
    assert r["work_per_launch"] == b.SLOTS_RHO_IK * 300 * 7
    assert g["work_per_launch"] == b.SLOTS_GATHER_IK * 300 * 7
    assert b.kernel_roofline("sample", {"sample": dict(avg_us=1.0, total_ms=1.0)}, None, 1, p, 0) is None


def test_dominant_kernel_is_the_largest_total_time():
    b = load_bench()
    p = dict(n=100, P=4)
    kernels = {"kick": dict(avg_us=1.0, total_ms=5.0), "kick_drift": dict(avg_us=2.0, total_ms=2.0)}
    dom, every = b.roofline(kernels, None, 0, p, 0)
    assert dom["kernel"] == "kick" and set(every) == {"kick", "kick_drift"}
    assert dom["traffic"] is None  # no workload named: no counter data


def test_measured_traffic_needs_same_sources_and_grid(tmp_path, monkeypatch):
    b = load_bench()
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    import hashlib
    h = hashlib.sha256(b"kernel v1\n").hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"w": {"files": ["k.hip"], "source_sha256": h, "grid": [6, 2, 2],
                 "kinds": {"pair_charged": {"read_bytes": 100.0, "write_bytes": 20.0}}}}
    (prof / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.measured_traffic("w", "pair_charged", [6, 2, 2]) == 120.0
    assert b.measured_traffic("w", "pair_charged", [2, 2, 2]) is None  # another grid
    assert b.measured_traffic("w", "kick", [6, 2, 2]) is None  # kind not counted
    src.write_text("kernel v2\n")
    assert b.measured_traffic("w", "pair_charged", [6, 2, 2]) is None  # sources changed since


def test_measured_traffic_is_per_form(tmp_path, monkeypatch):
    b = load_bench()
    import hashlib
    src = tmp_path / "k.hip"
    src.write_text("kernel\n")
    h = hashlib.sha256(b"kernel\n").hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"w": {"files": ["k.hip"], "source_sha256": h, "grid": [6, 2, 2], "form": "fp32c",
                 "kinds": {"pair_neutral": {"read_bytes": 100.0, "write_bytes": 20.0}}},
           "w:fp64": {"files": ["k.hip"], "source_sha256": h, "grid": [6, 2, 2], "form": "fp64",
                      "kinds": {"pair_neutral": {"read_bytes": 300.0, "write_bytes": 40.0}}}}
    (prof / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.measured_traffic("w", "pair_neutral", [6, 2, 2], "fp32c") == 120.0
    assert b.measured_traffic("w", "pair_neutral", [6, 2, 2], "fp64") == 340.0
    rec.pop("w:fp64")
    (prof / "traffic.json").write_text(json.dumps(rec))
    assert b.measured_traffic("w", "pair_neutral", [6, 2, 2], "fp64") is None  # counted on the other form


def test_tuner_grid_candidates():
    from paper_2609_02694_amd import tune
    g = tune.candidate_grids(30.0, 6.0, edges=(3.0, 3.05, 5.0), xsplits=(1, 2))
    # L // 3.0 = 10 and L // 3.05 = 9, L // 5 = 6; x split multiplies nx only; no duplicates
    assert g == [(10, 10, 10), (20, 10, 10), (9, 9, 9), (18, 9, 9), (6, 6, 6), (12, 6, 6)]
    # grids whose two-species key space would not fit int32 cell tables are skipped
    assert tune.candidate_grids(1000.0, 6.0, edges=(1.0,), xsplits=(1,)) == []


def test_batch_params_split_x():
    from paper_2609_02694_amd import tune
    reps = [(dict(seed=1, stream_seed=5, n=100, L=12.5, alpha=0.3, r_coul=6.0, r_lj=2.5, r_core=0.0, p_shell=0,
                  P=10, dt=0.002, ghost=0.0), None)]
    (pr,) = tune.batch_params(reps, 2.0, 1, xsplit=3)
    assert tuple(pr.ncell) == (18, 6, 6)


def test_tuner_cache_picks_fastest_and_reuses(tmp_path):
    from paper_2609_02694_amd import tune
    preset = dict(n=1000, L=30.0, alpha=0.3, r_coul=6.0, r_lj=2.5, r_core=0.0, p_shell=0, P=10, ghost=0.0)
    calls = []

    def fake_timer(p, s, grid, prec, steps):
        calls.append(grid)
        return abs(grid[0] - 20) + abs(grid[1] - 10)  # fastest at (20, 10, 10)

    path = str(tmp_path / "cache.json")
    g, hit = tune.tune_grid_cached(preset, None, 0, path, edges=(3.0, 5.0), xsplits=(1, 2), timer=fake_timer)
    assert g == (20, 10, 10) and not hit and len(calls) == 4
    g2, hit2 = tune.tune_grid_cached(preset, None, 0, path, edges=(3.0, 5.0), xsplits=(1, 2), timer=fake_timer)
    assert g2 == g and hit2 and len(calls) == 4  # served from the cache, nothing timed
    # another precision is another problem
    _, hit3 = tune.tune_grid_cached(preset, None, 1, path, edges=(3.0, 5.0), xsplits=(1, 2), timer=fake_timer)
    assert not hit3


def test_batch_tuner_cache(tmp_path):
    from paper_2609_02694_amd import tune
    reps = [(dict(n=100, L=12.5, alpha=0.3, r_coul=6.0, r_lj=2.5, r_core=0.0, p_shell=0, P=10, ghost=0.0), None),
            (dict(n=300, L=18.0, alpha=0.3, r_coul=6.0, r_lj=2.5, r_core=0.0, p_shell=0, P=10, ghost=0.0), None)]

    def fake(reps_, cat, off, h, prec, steps, xsplit=1):
        return h + 1.0 / xsplit

    path = str(tmp_path / "c.json")
    best, hit = tune.tune_batch_cached(reps, None, None, 1, path, edges=(2.0, 3.0), xsplits=(1, 3), timer=fake)
    assert best == (2.0, 3) and not hit
    assert tune.tune_batch_cached(reps, None, None, 1, path, edges=(2.0, 3.0), xsplits=(1, 3), timer=fake) == (
        (2.0, 3), True)


def test_roofline_reports_counted_hbm_rate(tmp_path, monkeypatch):
    b = load_bench()
    import hashlib
    src = tmp_path / "k.hip"
    src.write_text("kernel\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"w": {"files": ["k.hip"], "source_sha256": hashlib.sha256(b"kernel\n").hexdigest(), "grid": [4, 2, 2],
                 "kinds": {"kick": {"read_bytes": 3.0e9, "write_bytes": 1.0e9}}}}
    (prof / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    kernels = {"kick": dict(avg_us=1000.0, total_ms=5.0), "kick_drift": dict(avg_us=2.0, total_ms=2.0)}
    dom, every = b.roofline(kernels, None, 0, dict(n=100, P=4), 0, workload="w", grid=[4, 2, 2])
    # 4 GB per launch over 1 ms: 4000 GB/s, half the HBM peak
    assert dom["kernel"] == "kick" and dom["traffic"] == 4.0e9
    assert dom["hbm_gbps"] == pytest.approx(4000.0) and dom["hbm_frac"] == pytest.approx(0.5)
    assert "hbm_gbps" not in every["kick_drift"]  # not counted


def test_repeat_stats_median_min_max():
    b = load_bench()
    r = b.repeat_stats(1000, 10, [0.05, 0.01, 0.02, 0.03, 0.04])
    assert r["repeats"] == 5
    assert r["median_ms"] == pytest.approx(3.0) and r["min_ms"] == pytest.approx(1.0)
    assert r["max_ms"] == pytest.approx(5.0)
    assert r["particle_steps_per_s"] == pytest.approx(1000 / 3.0e-3)


def test_sampled_rows_cover_charged_neutral_faces_and_ends():
    import numpy as np
    b = load_bench()
    n = 5000
    rng = np.random.default_rng(0)
    L = 20.0
    s = dict(x=rng.random(n) * L, q=np.where(np.arange(n) < 500, 1.0, 0.0), L=np.array([L, L, L]))
    rows = b.sampled_rows(s, 64)
    assert len(rows) == len(set(rows.tolist()))
    assert (s["q"][rows] != 0).any() and (s["q"][rows] == 0).any()
    assert n - 1 in rows and 0 in rows
    assert (np.minimum(s["x"][rows], L - s["x"][rows]) < 0.05).sum() >= 8


def test_cpu_info_reports_model_and_threads():
    b = load_bench()
    info = b.cpu_info()
    assert info["oracle_threads"] >= 1 and info["logical_cpus"] >= 1
    assert info["model"]
