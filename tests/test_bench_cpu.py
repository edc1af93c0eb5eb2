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
    tile = "void lbx::tile_kernel<3, 8, 3, 3, false, 0, 256>(lbx::SysDev const*)"
    _csv(tmp_path / "f.csv", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 500.0),
                              ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 2.0),
                              (tile, "FETCH_SIZE", 3000.0), (tile, "FETCH_SIZE", 5000.0)])
    _csv(tmp_path / "w.csv", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 1000.0),
                              (tile, "WRITE_SIZE", 700.0), (tile, "WRITE_SIZE", 900.0)])
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
    # the lookup honours the source hash
    assert bench.measured_traffic("apply_kernel_forward_ki33", bench.APPLY_SOURCES, str(out)) == \
        pytest.approx(rec["bytes_per_launch"])
    assert bench.measured_traffic("apply_kernel_forward_ki33", bench.LDS_SOURCES, str(out)) is None
    assert bench.measured_traffic("no_such_kernel", bench.APPLY_SOURCES, str(out)) is None


def test_kernel_stats_table(tmp_path, capsys):
    db = tmp_path / "r.db"
    con = sqlite3.connect(db)
    con.execute("create table top_kernels (name text, total_calls int, total_duration real, "
                "average real, percentage real)")
    con.execute("insert into top_kernels values ('void lbx::sweep_kernel<false, true>(int)', 4, 2000.0, "
                "500.0, 75.0)")
    con.commit()
    con.close()
    bench.kernel_stats(str(db))
    out = capsys.readouterr().out
    assert "| `lbx::sweep_kernel<false, true>` | 4 | 2.000 | 0.5000 | 75.0 |" in out


def test_cost_model_of_the_two_transmon_workload():
    # 62.5 flops per entry per sweep and 62 per entry per adjoint step for
    # two 4-level subsystems (the figures the roofline is priced with).
    sweep, grad = bench.flops_per_entry((4, 4))
    assert sweep == pytest.approx(62.5)
    assert grad == pytest.approx(62.0)
    ctl, jump = bench.neighbour_counts((3,))
    assert ctl == pytest.approx(4 * 2 / 3) and jump == pytest.approx(4 / 9)
