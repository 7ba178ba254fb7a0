"""The rocprofv3 summaries behind profiles/: kernel-name shortening, the
trace grouped by kernel and grid, the copy calibration of the byte
counters and the shader-clock arithmetic, on small synthetic CSV files
laid out as rocprofv3 writes them.  No GPU is used."""
import csv

import pytest

from paper_2211_07532_amd import profiling as P


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)
    return str(path)


def _table(out):
    return [[c.strip() for c in line.split("|")[1:-1]] for line in out.splitlines() if line.startswith("| ")]


def test_short_name():
    assert P.short_name("void expenc::k_adj_split_sh<2, true, false>(expenc::AdjShArgs)") == \
        "k_adj_split_sh<2, true, false>"
    assert P.short_name("expenc::(anonymous namespace)::k_jacobi(HIP_vector_type<double, 2u>*, int)") == "k_jacobi"
    assert P.short_name("void expenc::k_dwt2_level<8>(HIP_vector_type<float, 2u> const*, int, long)") == \
        "k_dwt2_level<8>"
    assert P.short_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_trace_groups_by_kernel_and_grid(tmp_path, capsys):
    hdr = ["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Start_Timestamp", "End_Timestamp"]
    rows = [["void expenc::k_a<1>(int)", 256, 1, 1, 0, 3000],        # 3 us
            ["void expenc::k_a<1>(int)", 256, 1, 1, 10000, 15000],   # 5 us
            ["void expenc::k_a<1>(int)", 512, 1, 1, 0, 1000],        # another grid
            ["void expenc::k_b(int)", 64, 2, 1, 0, 20000]]           # 20 us, largest total
    P.trace([_write(tmp_path / "t.csv", hdr, rows)])
    t = _table(capsys.readouterr().out)
    assert t[0] == ["kernel", "grid (work-items)", "calls", "avg us", "min us", "max us"]
    body = t[1:]
    assert body[0] == ["k_b", "64x2x1", "1", "20.0", "20.0", "20.0"]
    assert body[1] == ["k_a<1>", "256x1x1", "2", "4.0", "3.0", "5.0"]
    assert body[2] == ["k_a<1>", "512x1x1", "1", "1.0", "1.0", "1.0"]


def test_pmc_means_and_copy_calibration(tmp_path, capsys):
    hdr = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    copy_kib = P.COPY_BYTES / 1024
    rows = [["__amd_rocclr_copyBuffer", 4096, "FETCH_SIZE", copy_kib / 2],   # the counter reads half
            ["__amd_rocclr_copyBuffer", 4096, "WRITE_SIZE", copy_kib],
            ["void expenc::k_x(int)", 1024, "FETCH_SIZE", 1000.0],
            ["void expenc::k_x(int)", 1024, "FETCH_SIZE", 3000.0],
            ["void expenc::k_x(int)", 1024, "WRITE_SIZE", 512.0],
            ["void expenc::k_x(int)", 1024, "SQ_WAVES", 16.0]]
    P.pmc([_write(tmp_path / "c.csv", hdr, rows)])
    out = capsys.readouterr().out
    t = _table(out)
    assert t[0] == ["kernel", "grid", "FETCH_SIZE", "SQ_WAVES", "WRITE_SIZE"]
    kx = [r for r in t if r[0] == "k_x"][0]
    # mean 2000 KiB fetched, x2 calibration -> 3.9 MiB; writes x1 -> 0.5 MiB
    assert kx[2] == "2000 (3.9 MiB scaled)"
    assert kx[3] == "16"
    assert kx[4] == "512 (0.5 MiB scaled)"
    assert "FETCH_SIZE x2.000" in out and "WRITE_SIZE x1.000" in out


def test_clock_from_busy_cycles_and_durations(tmp_path, capsys):
    trace = _write(tmp_path / "t.csv", ["Dispatch_Id", "Start_Timestamp", "End_Timestamp"],
                   [[1, 0, 100000], [2, 200000, 300000], [3, 0, 50000]])      # 100, 100, 50 us
    # GRBM_GUI_ACTIVE summed over 8 XCDs: 2.0 GHz then 2.2 GHz over 100 us
    cnt = _write(tmp_path / "c.csv", ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"],
                 [[1, "void expenc::k_y(int)", 256, "GRBM_GUI_ACTIVE", 8 * 2.0e9 * 100e-6],
                  [2, "void expenc::k_y(int)", 256, "GRBM_GUI_ACTIVE", 8 * 2.2e9 * 100e-6],
                  [2, "void expenc::k_y(int)", 256, "GRBM_COUNT", 1.0],
                  [3, "void expenc::k_z(int)", 64, "GRBM_GUI_ACTIVE", 8 * 1.5e9 * 50e-6]])
    P.clock(cnt, trace)
    t = _table(capsys.readouterr().out)
    assert t[1] == ["k_y", "256", "2", "100.0", "2100", "2200"]
    assert t[2] == ["k_z", "64", "1", "50.0", "1500", "1500"]


@pytest.mark.parametrize("cmd", [["trace"], ["pmc"], ["clock", "a.csv"]])
def test_cli_requires_its_files(cmd):
    with pytest.raises(SystemExit):
        P.main(cmd)
