"""Counter summaries (host logic only): calibration of FETCH_SIZE/WRITE_SIZE
by the plain copy and the mapping of kernel instantiations to passes."""
import csv

from paper_2305_10356_amd import profiling


def write_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for kern, val in rows:
            w.writerow({"Kernel_Name": kern, "Counter_Name": counter, "Counter_Value": val})


def test_traffic_calibration_and_pass_mapping(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    x_hc = "void ofm::spmm_kernel<float, 32, 1, false, false, true>(ofm::PassArgs)"
    v_def = "void ofm::spmm_kernel<float, 32, 3, false, false, false>(ofm::PassArgs)"
    chk = "void ofm::spmm_kernel<float, 32, 1, true, false, true>(ofm::PassArgs)"
    upd = "void ofm::dense_kernel<float, 32, 7>(ofm::PassArgs)"
    # the copy reads half of its bytes in FETCH_SIZE units, writes them all
    kib = profiling.COPY_BYTES / 1024.0
    write_csv(tmp_path / "f.csv", "FETCH_SIZE",
              [(copy, kib / 2), (copy, 4.0), (x_hc, 1000.0), (x_hc, 1200.0), (v_def, 500.0),
               (chk, 9999.0), (upd, 300.0)])
    write_csv(tmp_path / "w.csv", "WRITE_SIZE",
              [(copy, kib), (copy, 4.0), (x_hc, 100.0), (x_hc, 100.0), (v_def, 0.0),
               (chk, 1.0), (upd, 200.0)])
    sf, sw, rows = profiling.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    assert sf == 2.0 and sw == 1.0
    by = {r[0]: r for r in rows}
    # the residual-step instantiation (CHECK = true) is not the plain pass
    assert set(by) == {"spmm_x", "spmm_v", "update"}
    assert by["spmm_x"][1] == x_hc
    assert by["spmm_x"][4] == 1024.0 * (1100.0 * 2.0 + 100.0)
    assert by["spmm_v"][4] == 1024.0 * (500.0 * 2.0)
    assert by["update"][4] == 1024.0 * (300.0 * 2.0 + 200.0)
