"""The rocprofv3 table tool (paper_2206_03203_amd/profview.py) on small
hand-written CSV files (CPU): dispatches before the last cache flush are
left out, rows are keyed by kernel (template arguments kept, argument list
dropped) and grid, and the counters table turns FETCH_SIZE / WRITE_SIZE
(KiB per dispatch) into bytes with the given scale factors."""

import csv

from paper_2206_03203_amd import profview


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_kernel_key_keeps_templates_and_drops_arguments():
    name = "void mdp::(anonymous namespace)::spmv_kernel<32, 4, 1, 5, double, double, double>(int, int const*)"
    assert profview.kernel_key(name) == "spmv_kernel<32, 4, 1, 5, double, double, double>"
    assert profview.kernel_key("mdp::dcgs_update_kernel(mdp::Tile const*, int)") == "dcgs_update_kernel"


def test_trace_and_counter_tables(tmp_path, capsys):
    tr = tmp_path / "trace.csv"
    hdr = ["Kernel_Name", "Grid_Size", "Start_Timestamp", "End_Timestamp"]
    _write(tr, hdr, [
        ["dcgs_update_kernel(int)", 131072, 100, 99100],       # before the flush: left out
        ["cache_flush_kernel(double2 const*)", 524288, 200000, 260000],
        ["dcgs_update_kernel(int)", 131072, 300000, 340000],   # 40 us
        ["dcgs_update_kernel(int)", 131072, 400000, 420000],   # 20 us
        ["dcgs_update_kernel(int)", 524288, 500000, 600000],   # another grid: 100 us
    ])
    agg = profview.trace_table(str(tr))
    assert agg[("dcgs_update_kernel", 131072)] == [2, 60.0]
    assert agg[("dcgs_update_kernel", 524288)] == [1, 100.0]
    assert not any("cache_flush" in k for k, _ in agg)

    fetch, write = tmp_path / "fetch.csv", tmp_path / "write.csv"
    chdr = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    _write(fetch, chdr, [[1, "dcgs_update_kernel(int)", 131072, "FETCH_SIZE", 999999.0],
                         [2, "cache_flush_kernel(x)", 524288, "FETCH_SIZE", 1.0],
                         [3, "dcgs_update_kernel(int)", 131072, "FETCH_SIZE", 1000.0],
                         [4, "dcgs_update_kernel(int)", 131072, "FETCH_SIZE", 3000.0]])
    _write(write, chdr, [[3, "dcgs_update_kernel(int)", 131072, "WRITE_SIZE", 500.0],
                         [4, "dcgs_update_kernel(int)", 131072, "WRITE_SIZE", 500.0]])
    ct = profview.counter_table([str(fetch), str(write)])
    assert ct[("dcgs_update_kernel", 131072)]["FETCH_SIZE"] == [1000.0, 3000.0]
    assert ct[("dcgs_update_kernel", 131072)]["WRITE_SIZE"] == [500.0, 500.0]

    assert profview.main(["counters", "--trace", str(tr), str(fetch), str(write), "--fetch-scale", "2.0",
                          "--write-scale", "1.0", "--match", "dcgs_update"]) == 0
    out = capsys.readouterr().out
    row = [line for line in out.splitlines() if line.endswith("dcgs_update_kernel") and " 131072 " in line]
    assert len(row) == 1
    f = row[0].split()
    # mean FETCH 2000 KiB x 2 = 4.096 MB read, WRITE 500 KiB = 0.512 MB, over 30 us per launch
    assert f[1] == "2" and f[2] == "30.00" and f[4] == "4.1" and f[5] == "0.5"
    assert abs(float(f[6]) - (4.096e6 + 0.512e6) / 30e-6 / 1e9) < 1.0
