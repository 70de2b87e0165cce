"""Host logic of the rocprofv3 summary tool: counter CSVs -> bytes per launch
(scaled by the copy calibration), stats table, kernel name mapping."""
import csv

import pytest

from paper_1605_04521_amd import profiling


def write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, v) in enumerate(rows):
            w.writerow([i, name, counter, v])


def test_kernel_key_mapping():
    assert profiling.kernel_key("void mxw::k_lu<float, 32>(float*, ...)") == "lu"
    assert profiling.kernel_key("void mxw::k_local_solve_multi<float, 32, 32>(...)") == "local_solve_multi"
    assert profiling.kernel_key("void mxw::k_local_solve<double, 32>(...)") == "local_solve"
    assert profiling.kernel_key("void mxw::k_spmm<16, 8>(...)") == "spmv"
    assert profiling.kernel_key("void mxw::k_spmv<16>(...)") == "spmv"
    assert profiling.kernel_key("mxw::k_spmm_il(long, int, ...)") == "spmv"
    assert profiling.kernel_key("void mxw::k_lu_queue<float, 32, 8>(float*, ...)") == "lu"
    assert profiling.kernel_key("mxw::k_to_interleaved(long, int, ...)") is None
    assert profiling.kernel_key("mxw::k_dots(...)") is None


def test_traffic_scaled_by_copy(tmp_path):
    # the counter reads half the true bytes: the copy of 1 GiB reads 512 MiB
    gib = 1 << 30
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    write_counters(f, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", gib / 2 / 1024), ("__amd_rocclr_copyBuffer", 1.0),
                                     ("void mxw::k_local_solve<double, 32>", 1000.0),
                                     ("void mxw::k_local_solve<double, 32>", 3000.0)])
    write_counters(w, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", gib / 1024),
                                     ("void mxw::k_local_solve<double, 32>", 10.0),
                                     ("void mxw::k_local_solve<double, 32>", 30.0)])
    res = profiling.traffic(str(f), str(w))
    rec = res["local_solve"]
    assert rec["fetch_bytes"] == pytest.approx(2000.0 * 2 * 1024)
    assert rec["write_bytes"] == pytest.approx(20.0 * 1024)
    assert rec["bytes_per_launch"] == pytest.approx(rec["fetch_bytes"] + rec["write_bytes"])
    assert rec["dispatches"] == [2, 2]
    assert "lu" not in res


def test_traffic_needs_copy(tmp_path):
    f = tmp_path / "f.csv"
    write_counters(f, "FETCH_SIZE", [("void mxw::k_lu<double, 32>", 5.0)])
    with pytest.raises(ValueError):
        profiling.traffic(str(f), str(f))


def test_stats_table(tmp_path):
    p = tmp_path / "s.csv"
    with open(p, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        w.writerow(["a", 2, 4e6, 2e6, 20.0, 1, 3, 0])
        w.writerow(["b", 1, 16e6, 16e6, 80.0, 1, 3, 0])
    t = profiling.stats_table(str(p)).splitlines()
    assert t[2].startswith("| `b` | 1 | 16.00 | 16.0000 | 80.00")
    assert t[3].startswith("| `a` | 2 | 4.00 | 2.0000 | 20.00")
