"""Host logic of bench.py (no GPU): the one-GPU guard, the counter summary,
the kernel-trace table, the traffic lookup and the algorithmic cost model."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _csv(path, rows):
    with open(path, "w") as fh:
        fh.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
        for k, (name, counter, value) in enumerate(rows):
            fh.write(f'{k},"{name}","{counter}",{value}\n')


def test_traffic_summary_calibrates_against_the_copy(tmp_path, capsys):
    copy_bytes = 1024 * 1000
    tile = "void lbx::tile_kernel<3, 8, 3, 3, false, 256>(lbx::SysDev const*)"
    sweep = "void lbx::sweep_tile_kernel<3, 8, 3, 3, true, 256>(lbx::StepArgs, int)"
    _csv(tmp_path / "f.csv", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 500.0),
                              ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 2.0),
                              (tile, "FETCH_SIZE", 3000.0), (tile, "FETCH_SIZE", 5000.0),
                              (sweep, "FETCH_SIZE", 6000.0), (sweep, "FETCH_SIZE", 2.0),
                              (sweep, "FETCH_SIZE", 4000.0)])
    _csv(tmp_path / "w.csv", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 1000.0),
                              (tile, "WRITE_SIZE", 700.0), (tile, "WRITE_SIZE", 900.0),
                              (sweep, "WRITE_SIZE", 1500.0), (sweep, "WRITE_SIZE", 0.0),
                              (sweep, "WRITE_SIZE", 500.0)])
    out = tmp_path / "traffic.json"
    bench.traffic_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), copy_bytes, str(out))
    table = json.loads(out.read_text())
    assert table["calibration"]["fetch_factor"] == pytest.approx(2.0)
    assert table["calibration"]["write_factor"] == pytest.approx(1.0)
    rec = table["apply_kernel_forward_ki33"]
    assert rec["fetch_bytes"] == pytest.approx(2.0 * 4000.0 * 1024)
    assert rec["write_bytes"] == pytest.approx(800.0 * 1024)
    assert rec["bytes_per_launch"] == pytest.approx(rec["fetch_bytes"] + rec["write_bytes"])
    assert rec["dispatches"] == [2, 2]
    assert rec["source_sha"] == bench.source_sha(bench.APPLY_SOURCES)
    assert "apply_kernel_adjoint_ki33" not in table
    # the stage sweep averages its executed launches only (the sweep kernel's
    # name must not count as the apply kernel's either)
    sw = table["stage_sweep_c5_ki33"]
    assert sw["dispatches"] == [2, 2]
    assert sw["fetch_bytes"] == pytest.approx(2.0 * 5000.0 * 1024)
    assert sw["write_bytes"] == pytest.approx(1000.0 * 1024)
    # the lookup honours the source hash
    assert bench.measured_traffic("apply_kernel_forward_ki33", bench.APPLY_SOURCES, str(out)) == \
        pytest.approx(rec["bytes_per_launch"])
    assert bench.measured_traffic("apply_kernel_forward_ki33", bench.LDS_SOURCES, str(out)) is None
    assert bench.measured_traffic("no_such_kernel", bench.APPLY_SOURCES, str(out)) is None


def test_kernel_stats_table(tmp_path, capsys):
    # the same table from a results database (kernels view, ns timestamps) and
    # from a kernel_trace.csv; a launch below 5 % of the longest is "other"
    rows = [("void lbx::sweep_tile_kernel<3, 8, 3, 4, false, 256>(int)", 0, 2_000_000),
            ("void lbx::sweep_tile_kernel<3, 8, 3, 4, false, 256>(int)", 3_000_000, 5_000_000),
            ("void lbx::sweep_tile_kernel<3, 8, 3, 4, false, 256>(int)", 6_000_000, 6_010_000),
            ("void lbx::step_count_kernel(lbx::StepArgs)", 7_000_000, 7_005_000)]
    db = tmp_path / "r.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start int, end int)")
    con.executemany("insert into kernels values (?, ?, ?)", rows)
    con.commit()
    con.close()
    csvf = tmp_path / "kernel_trace.csv"
    csvf.write_text("Kernel_Name,Start_Timestamp,End_Timestamp\n" +
                    "".join(f'"{n}",{a},{b}\n' for n, a, b in rows))
    for path in (db, csvf):
        bench.kernel_stats(str(path))
        out = capsys.readouterr().out
        assert "| `lbx::sweep_tile_kernel<3, 8, 3, 4, false, 256>` | 3 | 4.010 | 1.3367 | 99.9 |" in out
        assert "| `lbx::sweep_tile_kernel<3, 8, 3, 4, false, 256>` | 3 | 2 | 2.0000 | 0.0100 |" in out


def test_cost_model_of_the_two_transmon_workload():
    # 62.5 flops per entry per sweep and 62 per entry per adjoint step for
    # two 4-level subsystems (the figures the roofline is priced with).
    sweep, grad = bench.flops_per_entry((4, 4))
    assert sweep == pytest.approx(62.5)
    assert grad == pytest.approx(62.0)
    ctl, jump = bench.neighbour_counts((3,))
    assert ctl == pytest.approx(4 * 2 / 3) and jump == pytest.approx(4 / 9)


def test_window_checkpoints_follow_the_full_horizon():
    from workloads import make_config
    # eight qutrits: every system streams, so the full run's automatic
    # interval ceil(sqrt(5000)) = 71 is made explicit for a window
    assert bench.window_ckpt(make_config(5)) == 71
    # five qutrits carry their own interval
    assert bench.window_ckpt(make_config(4)) == 200
    # the uneven batch mixes LDS-resident systems: automatic
    assert bench.window_ckpt(make_config(3)) == 0


def test_cpu_process_count_respects_share_and_memory():
    info = {"affinity": 64, "mem_available": 200 << 30}
    assert bench.cpu_procs(5, info) == 16
    info = {"affinity": 64, "mem_available": 30 << 30}
    assert bench.cpu_procs(5, info) == 2
    info = {"affinity": 4, "mem_available": None}
    assert bench.cpu_procs(2, info) == 4
    h = bench.host_info()
    assert h["nproc"] >= 1 and h["affinity"] >= 1


def test_oracle_pool_runs_states_in_separate_processes():
    # three two-transmon evaluations over two processes, 20 steps each
    wall = bench.run_oracle_pool(("grad2", 20), [0, 1, 2], 2)
    assert 0.0 < wall < 60.0


def test_traffic_rate_beside_the_algorithmic_rate():
    roof = {"unit": "GB/s", "peak": 8000.0, "traffic": 4e9, "avg_launch_ms": 2.0, "achieved": 1000.0}
    out = bench.with_traffic_rate(dict(roof))
    assert out["traffic_GBps"] == pytest.approx(2000.0)
    assert out["traffic_frac"] == pytest.approx(0.25)
    # no counters (or another unit): unchanged
    assert "traffic_GBps" not in bench.with_traffic_rate(dict(roof, traffic=None))
    assert "traffic_GBps" not in bench.with_traffic_rate(dict(roof, unit="TFLOP/s"))
