"""The rocprofv3 summaries kept with the library (host logic only): the copy calibration of
the HBM counters, the per-kernel join of trace durations with counter medians, and the
source hash that marks a traffic summary stale."""
import csv
import importlib.util
import json
import os

# loaded from its file: the package's __init__ loads the HIP library, which these host-only
# tests do not need
_spec = importlib.util.spec_from_file_location(
    "prof_summary", os.path.join(os.path.dirname(__file__), "..", "paper_1307_4354_amd", "prof_summary.py"))
ps = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(ps)


def _write(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_ALL)
        w.writerow(header)
        w.writerows(rows)
    return str(path)


def _counters(tmp_path):
    hdr = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    # the copy moves 1 MiB each way: FETCH_SIZE reads half of it (512 KiB), WRITE_SIZE all
    fetch = _write(tmp_path / "f.csv", hdr, [
        ["k_a(int)", 100, "FETCH_SIZE", 1000.0], ["k_a(int)", 100, "FETCH_SIZE", 3000.0],
        ["k_a(int)", 100, "FETCH_SIZE", 2000.0], ["k_b(int)", 50, "FETCH_SIZE", 10.0],
        ["__amd_rocclr_copyBuffer", 9, "FETCH_SIZE", 512.0]])
    write = _write(tmp_path / "w.csv", hdr, [
        ["k_a(int)", 100, "WRITE_SIZE", 100.0], ["k_b(int)", 50, "WRITE_SIZE", 5.0],
        ["__amd_rocclr_copyBuffer", 9, "WRITE_SIZE", 1024.0]])
    return fetch, write


def test_traffic_is_copy_calibrated(tmp_path, capsys):
    fetch, write = _counters(tmp_path)
    ps.main(["traffic", "--fetch", fetch, "--write", write, "--kernel", "k_a", "--grid", "100",
             "--copy-bytes", str(1 << 20), "--cmd", "x"])
    d = json.loads(capsys.readouterr().out)
    assert d["copy_calibration"]["fetch_factor"] == 2.0
    assert d["copy_calibration"]["write_factor"] == 1.0
    assert d["fetch_kib_median"] == 2000.0 and d["write_kib_median"] == 100.0
    assert d["traffic_bytes"] == 2000.0 * 1024 * 2 + 100.0 * 1024
    assert d["source_sha256"] == ps.sources_sha256(ps.EXT_SOURCES)


def test_rates_join_trace_and_counters(tmp_path, capsys):
    fetch, write = _counters(tmp_path)
    trace = _write(tmp_path / "kt.csv", ["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp"], [
        ["k_a(int)", 100, 0, 1000], ["k_a(int)", 100, 0, 3000], ["k_b(int)", 50, 0, 500],
        ["k_c(int)", 7, 0, 9000]])  # k_c has no counter dispatch: left out
    ps.main(["rates", trace, "--fetch", fetch, "--write", write, "--copy-bytes", str(1 << 20), "--cmd", "x"])
    out = capsys.readouterr().out
    rows = [l for l in out.splitlines() if l.startswith("| ") and "`" in l]
    assert len(rows) == 2 and "k_a" in rows[0] and "k_b" in rows[1]
    cells = [c.strip() for c in rows[0].strip("|").split("|")]
    # k_a: 2 calls averaging 2 us; 2000 KiB x 2 fetched, 100 KiB written
    assert cells[1] == "2" and cells[2] == "2.00"
    assert abs(float(cells[3]) - 2000 * 1024 * 2 / 1e6) < 0.05
    assert abs(float(cells[4]) - 100 * 1024 / 1e6) < 0.05
    assert abs(float(cells[5]) - (2000 * 1024 * 2 + 100 * 1024) / 2000.0) < 1.0
