"""Host logic of bench.py (no GPU): the one-GPU guard, the counter record it
reads for the roofline's `traffic`, and its latency percentiles."""
import json
import os
import subprocess
import sys

import pytest

import bench
from paper_1601_05448_amd import profile_summary

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line for a run that did not happen


def test_sweep_byte_table():
    # each sweep's FP32 bytes are half its FP64 bytes (every field it moves is
    # one value per cell in the sweep's precision)
    for sw, (b64, b32) in bench.SWEEP_BYTES.items():
        assert b64 == 2 * b32, sw
    # P1 reads rho, p and b and writes the transformed weighted residual
    assert bench.SWEEP_BYTES[1] == (4 * 8, 4 * 4)


def test_traffic_record_matches_the_kernel_sources():
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    assert set(rec) >= {"f32:k_resid_dhtx_z@256", "f64:k_resid_dhtx_z@256"}
    if any(v["source_sha256"] != profile_summary.kernel_source_hash() for v in rec.values()):
        pytest.skip("the counters predate the current kernel sources (bench reports traffic null)")
    n = 256 ** 3
    for key, per_cell in (("f32:k_resid_dhtx_z", 16), ("f64:k_resid_dhtx_z", 32)):
        t = bench.measured_traffic(key, 256)
        assert t is not None
        # measured HBM bytes: at least the algorithmic bytes, and the halo
        # re-reads of the z-marching tiles well under a quarter more
        assert per_cell * n <= t < 1.25 * per_cell * n, (key, t / n)


def test_traffic_is_null_without_a_valid_record(monkeypatch):
    assert bench.measured_traffic("f32:k_resid_dhtx_z", 128) is None  # no record at this size
    assert bench.measured_traffic("f32:no_such_kernel", 256) is None
    monkeypatch.setattr(profile_summary, "kernel_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic("f32:k_resid_dhtx_z", 256) is None  # sources changed since


def test_percentile():
    assert bench.percentile([3.0, 1.0, 2.0], 0.5) == 2.0
    assert bench.percentile([5.0], 0.99) == 5.0
    xs = [float(i) for i in range(101)]  # 0 .. 100
    assert bench.percentile(xs, 0.99) == pytest.approx(99.0)
    assert bench.percentile([0.0, 10.0], 0.25) == pytest.approx(2.5)
    assert bench.percentile([], 0.5) != bench.percentile([], 0.5)  # NaN


def test_profile_stats_by_grid(tmp_path, capsys):
    """The duration summary groups dispatches by kernel name, or by name and
    launch grid, and filters by a name substring."""
    import argparse
    import sqlite3

    db = sqlite3.connect(str(tmp_path / "run_results.db"))
    db.execute("create table kernels (name text, duration integer, grid_x integer, grid_y integer, grid_z integer)")
    rows = [("k_a", 1000, 64, 1, 1), ("k_a", 3000, 64, 1, 1), ("k_a", 8000, 128, 1, 1), ("k_b", 500, 64, 1, 1)]
    db.executemany("insert into kernels values (?, ?, ?, ?, ?)", rows)
    db.commit()
    db.close()
    durs = profile_summary.kernel_durations(str(tmp_path))
    assert sorted(durs["k_a"]) == [1000.0, 3000.0, 8000.0] and durs["k_b"] == [500.0]
    by = profile_summary.kernel_durations(str(tmp_path), by_grid=True)
    assert by["[grid 64x1x1] k_a"] == [1000.0, 3000.0] and by["[grid 128x1x1] k_a"] == [8000.0]
    profile_summary.cmd_stats(argparse.Namespace(dir=str(tmp_path), top=10, match="k_a", by_grid=True))
    out = capsys.readouterr().out.splitlines()
    assert len(out) == 3 and "k_b" not in "".join(out)
    assert out[1].split()[0] == "1" and out[1].endswith("[grid 128x1x1] k_a")  # largest total first
    assert out[2].split()[:3] == ["2", "0.004", "2.0"]  # calls, total ms, mean us


def test_profile_solves_breakdown(tmp_path, capsys):
    """The per-solve breakdown splits the trace at each k_init, reports span,
    time in kernels and gaps, and counts sweep launches shorter than the idle
    limit apart."""
    import argparse
    import sqlite3

    db = sqlite3.connect(str(tmp_path / "run_results.db"))
    db.execute("create table kernels (name text, start integer, end integer)")
    us = 1000
    rows = [("pois::k_init(x)", 0, 2 * us), ("void pois::k_dht_cols<float, 256, 1, 0>(x)", 3 * us, 23 * us),
            ("void pois::k_dht_cols<float, 256, 1, 0>(x)", 25 * us, 29 * us),  # idle: 4 us
            ("pois::k_decide_iter(x)", 30 * us, 37 * us), ("at::other_kernel(x)", 38 * us, 90 * us),
            ("pois::k_init(x)", 100 * us, 101 * us), ("void pois::k_dhtx_update<float, 256, 0, 0>(x)", 101 * us, 131 * us)]
    db.executemany("insert into kernels values (?, ?, ?)", rows)
    db.commit()
    db.close()
    profile_summary.cmd_solves(argparse.Namespace(dir=str(tmp_path), first=0, count=4, idle_us=6.0))
    out = capsys.readouterr().out.splitlines()
    assert out[0] == "solve 0: 4 kernels, span 37.0 us, in kernels 33.0 us, gaps 4.0 us"
    rows0 = {line.split("us  ")[1]: (int(line.split()[0]), float(line.split()[1])) for line in out[1:5]}
    assert rows0 == {"k_dht_cols": (1, 20.0), "k_decide_iter": (1, 7.0), "k_dht_cols (idle)": (1, 4.0),
                     "k_init": (1, 2.0)}
    assert out[5] == "solve 1: 2 kernels, span 31.0 us, in kernels 31.0 us, gaps 0.0 us"


def test_model_bytes_per_cell():
    """The whole-solve byte model: FP64 16 + 104 K + 32; FP32 with refinement
    44 + 48 S + 52 K (see bench.model_bytes_per_cell)."""
    assert bench.model_bytes_per_cell(False, 10, 0) == 16 + 10 * 104 + 32
    # the final check reads rho, p and b and writes nothing
    assert bench.model_bytes_per_cell(True, 10, 3) == 20 + 3 * (32 + 32 + 16 + 20) + (10 - 3) * 52 + 24
    # a step whose end was predicted runs no confirming residual sweep: 16 less
    assert bench.model_bytes_per_cell(True, 10, 3, 9) == bench.model_bytes_per_cell(True, 10, 3) - 16


def test_cpu_baseline_leg_end_to_end():
    """The cpu_baseline leg on small grids: the background oracle solve, the
    reference it continues to, the error of an answer against it, the repeated
    small solves and the concurrent processes."""
    import numpy as np

    import oracle
    from paper_1601_05448_amd import inputs

    prob = inputs.small_problem(shape=(16, 16, 16), lengths=(2 * np.pi,) * 3)
    small = inputs.small_problem(shape=(8, 8, 8), lengths=(2 * np.pi,) * 3, seed=3)
    leg = bench.CpuBaseline(prob, small, 1e-10)
    ans = oracle.solve(prob.rho, prob.b, lengths=prob.lengths, tol=1e-10)["p"]
    base, errors = leg.finish({"oracle_1e-10": ans})
    assert base["kind"] == "oracle" and base["unit"] == "solves/s" and base["value"] > 0
    assert base["cores"] == 1 and base["nproc"] >= 1 and base["cpu_model"]
    assert base["small_32"]["procs"] >= 1 and base["small_32"]["aggregate_solves_per_s"] > 0
    assert base["small_32"]["min_s"] <= base["small_32"]["median_s"]
    e = errors["oracle_1e-10"]
    # an answer at 1e-10 against the 1e-12 reference: small but not zero
    assert 0 < e["rel_l2"] < 1e-8 and e["max_abs"] > 0
