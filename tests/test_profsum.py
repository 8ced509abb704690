"""Host checks of the rocprofv3 summarizer on synthetic CSV files in the
formats it reads: the per-kernel stats table, the per-launch listing, the
counter averages and the traffic scaling by the device-copy calibration."""
import csv
import io
import json

from paper_2003_01282_amd import profsum as P


def write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_stats_and_calls(tmp_path):
    d = tmp_path / "prof"
    d.mkdir()
    write_csv(d / "x_kernel_stats.csv", [
        {"Name": "void slaq::spmm_rows<0, false, float>(args)", "Calls": 4, "AverageNs": 2500000.0,
         "TotalDurationNs": 1e7, "Percentage": 80.0},
        {"Name": "slaq::update<float>(args)", "Calls": 4, "AverageNs": 625000.0, "TotalDurationNs": 2.5e6,
         "Percentage": 20.0}])
    write_csv(d / "x_kernel_trace.csv", [
        {"Kernel_Name": "slaq::update<float>(a)", "Start_Timestamp": 1000, "End_Timestamp": 3001000,
         "Grid_Size_X": 4096, "Workgroup_Size_X": 256},
        {"Kernel_Name": "void slaq::spmm_rows<0>(a)", "Start_Timestamp": 5000, "End_Timestamp": 7000,
         "Grid_Size_X": 512, "Workgroup_Size_X": 256},
        {"Kernel_Name": "slaq::update<float>(a)", "Start_Timestamp": 9000, "End_Timestamp": 509000,
         "Grid_Size_X": 4096, "Workgroup_Size_X": 256}])
    out = io.StringIO()
    P.stats(str(d), out=out)
    lines = out.getvalue().splitlines()
    assert lines[1].split()[-4:] == ["4", "2500.00", "10.00", "80.00"]
    out = io.StringIO()
    P.calls(str(d), "update", out=out)
    rows = [ln.split() for ln in out.getvalue().splitlines()[1:]]
    assert [r[0] for r in rows] == ["0", "1"] and [r[-1] for r in rows] == ["3.000", "0.500"]


def test_traffic_scaling(tmp_path):
    # the copy of 1 GiB reads as 524,288 KiB of FETCH_SIZE (the counter
    # under-reports by 2) and as 1,048,576 KiB of WRITE_SIZE; the run's later
    # copies (a few bytes, an 8 GiB array, half a GiB) are not the calibration
    fetch, write = tmp_path / "f", tmp_path / "w"
    fetch.mkdir()
    write.mkdir()
    copy = "__amd_rocclr_copyBuffer"
    kern = ["void slaq::spmm_pieces<0>(a)", "void slaq::spmm_rows<0>(a)", "void slaq::spmm_heavy<0>(a)",
            "slaq::update<float>(a)"]
    # another template variant of the light-row kernel: pooled with it
    variant = "void slaq::spmm_rows<0, false, float, true>(a)"
    write_csv(fetch / "c_counter_collection.csv",
              [{"Kernel_Name": copy, "Counter_Name": "FETCH_SIZE", "Counter_Value": v}
               for v in (524288.0, 2.5, 8218193.5, 262144.0)] +
              [{"Kernel_Name": k, "Counter_Name": "FETCH_SIZE", "Counter_Value": v}
               for k, v in zip(kern, (1000.0, 500.0, 100.0, 50.0))] +
              [{"Kernel_Name": kern[0], "Counter_Name": "FETCH_SIZE", "Counter_Value": 3000.0},
               {"Kernel_Name": variant, "Counter_Name": "FETCH_SIZE", "Counter_Value": 100.0}])
    write_csv(write / "c_counter_collection.csv",
              [{"Kernel_Name": copy, "Counter_Name": "WRITE_SIZE", "Counter_Value": v}
               for v in (1048576.0, 16436201.0, 0.0625, 530053.0)] +
              [{"Kernel_Name": k, "Counter_Name": "WRITE_SIZE", "Counter_Value": v}
               for k, v in zip(kern, (10.0, 20.0, 30.0, 40.0))] +
              [{"Kernel_Name": variant, "Counter_Name": "WRITE_SIZE", "Counter_Value": 10.0}])
    out_json = tmp_path / "t.json"
    P.traffic(str(fetch), str(write), float(1 << 30), str(out_json))
    rec = json.loads(out_json.read_text())
    assert abs(rec["FETCH_SIZE_scale"] - 2.0) < 1e-12 and abs(rec["WRITE_SIZE_scale"] - 1.0) < 1e-12
    # spmm_pieces averages its two dispatches: (1000 + 3000) / 2 KiB
    assert rec["kernels"]["spmm_pieces"]["FETCH_SIZE_bytes"] == 2000.0 * 1024 * 2
    assert rec["kernels"]["spmm_rows"]["FETCH_SIZE_bytes"] == 300.0 * 1024 * 2
    stage = (2000 + 300 + 100) * 1024 * 2 + (10 + 15 + 30) * 1024
    assert rec["bytes_per_launch"] == stage
    assert rec["update_bytes_per_launch"] == 50 * 1024 * 2 + 40 * 1024
    assert rec["digest"] == P.kernel_sources_digest()



def test_traffic_calibration_is_the_first_copy_of_its_size():
    import pytest
    assert P.calibration_dispatch([3.0, 524288.0, 8e6, 530000.0], float(1 << 30)) == 524288.0
    with pytest.raises(SystemExit):
        P.calibration_dispatch([8e6, 2.0], float(1 << 30))
