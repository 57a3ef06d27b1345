"""Host-side parsing of bench.py's large-size summary: synthetic rocprofv3
CSVs (kernel trace, FETCH_SIZE and WRITE_SIZE passes with the calibration
copy) give the expected per-kernel durations and scaled HBM bytes."""
import csv
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)


def test_large_summary_tables(tmp_path, capsys):
    per = bench.LARGE_SETS * (bench.LARGE_ROUNDS + 1)
    n_ops = len(bench.LARGE_OPS)
    trace, fetch, write = [], [], []
    did = 10
    copy_kib = bench.COPY_REF_BYTES / 1024
    for ctr, rows, scale in (("FETCH_SIZE", fetch, 0.5), ("WRITE_SIZE", write, 1.0)):
        rows.append({"Dispatch_Id": 1, "Kernel_Name": "elementwise_copy",
                     "Grid_Size": bench.COPY_REF_BYTES // 16, "Counter_Name": ctr,
                     "Counter_Value": copy_kib * scale})
    for k in range(n_ops):
        for i in range(per):
            did += 1
            us = 100.0 * (k + 1) if i >= bench.LARGE_SETS else 999.0
            name = f"void aw::kern{k}(args)"
            trace.append({"Dispatch_Id": did, "Kernel_Name": name, "Start_Timestamp": 0,
                          "End_Timestamp": int(us * 1000)})
            fetch.append({"Dispatch_Id": did, "Kernel_Name": name, "Grid_Size": 64,
                          "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000.0})
            write.append({"Dispatch_Id": did, "Kernel_Name": name, "Grid_Size": 64,
                          "Counter_Name": "WRITE_SIZE", "Counter_Value": 3000.0})
    t, fp, wp = tmp_path / "t.csv", tmp_path / "f.csv", tmp_path / "w.csv"
    _write(t, ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"], trace)
    cols = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    _write(fp, cols, fetch)
    _write(wp, cols, write)
    bench.large_summary(str(t), str(fp), str(wp))
    out = capsys.readouterr().out.splitlines()
    rows = [ln for ln in out if ln.startswith("| ") and "`aw::kern" in ln]
    assert len(rows) == n_ops
    for k, ln in enumerate(rows):
        cells = [c.strip() for c in ln.strip("|").split("|")]
        assert cells[0] == bench.LARGE_OPS[k]
        assert float(cells[2]) == 100.0 * (k + 1)  # untimed first round excluded
        # fetch counted at half the copy's bytes: factor 2; write factor 1
        assert abs(float(cells[6]) - 1024 * (2 * 1000.0 + 3000.0) / 1e6) < 0.05
